// The ovvo contraction of the IP sigma product (Eq. xplin's T5, T6 and T8 terms through Weff)
// on bf16 matrix cores with two-term operands, for the reduced-precision sigma of the mixed
// solver:
//   Z[(i,a)][(j,c)] = sum_(m,e) W[(i,a)][(m,e)] r_mj^e[c],     r_mj^e = +-X2[pair(m,j)][e][c]
// Both operands are held as bf16 pairs x = hi + lo (hi = bf16(x) rounded to nearest even,
// lo = bf16(x - hi)). Every 16 x 16 block takes hi.hi + hi.lo + lo.hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation: about 16 significant bits per operand
// (|lo| <= 2^-8 |x| after round-to-nearest, so the dropped lo.lo term is at most about 2^-16
// of the product), at three bf16 products per FP32 one.
//
// Layout. The k index (m, e) runs over segments of vp = v rounded up to a multiple of 8 (zeros
// for e >= v), so that every 8-element chunk of k lies inside one segment m.
//  - W: pairs [M][ldk] row-major, split once when the operator is built (ldk = o vp rounded up
//    to the 32-deep slab, zero-filled).
//  - r: expanded once per sigma product by pairs_expand_kernel into the chunked layout
//    R[k/8][N][8] over the N = o nc columns (j, c), with the signs applied and the zero
//    segment m = j and the padding written as zeros. Staging a B tile is then one plain
//    16-byte copy per lane, consecutive lanes on consecutive columns. The expanded operand
//    takes 4 (o vp) (o nc) bytes (5.3 GB at o=70, v=260 and 512 right-hand sides) and its
//    pass costs about 2% of the product.
//
// GEMM. Column blocks of 256 (nc % 256 == 0) take pairs_gemm8_kernel (below: 256 x 256
// tiles, direct global-to-LDS loads). Otherwise tile 256 x 128 x 32, 512 threads as 4 x 2
// wavefronts of 64 x 64, one workgroup per CU. LDS is double-buffered, so one barrier per slab: while a slab's MFMAs
// run, the next slab's global loads are in flight; they are stored to the other buffer after
// the MFMAs. An LDS row of 128 bytes holds 32 k of one tile row (A) or column (B): the four
// 16-byte chunks of the high parts, then the four of the remainders, chunk c stored at
// position c ^ (row & 7). Measured on the bank-conflict counter, fragment reads (16 rows x 4
// chunks per wavefront) and the stores of both tiles are then conflict-free, where 64- or
// 144-byte rows without the permutation stall about 4 cycles per read. The k slabs that lie wholly inside
// the tile's zero segment m = j are skipped (a tile's columns share one j: nc % BN == 0).
// Workgroups are dealt to the 8 XCDs round robin, each XCD taking a contiguous range of a
// tile order that walks 8 M-tiles down before the next N-tile.
#include "common.h"

namespace gfcc {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 b2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef const u4 __attribute__((address_space(1)))* gu4;   // global loads, not flat

constexpr int PBM = 256;   // tile rows
constexpr int PNT = 512;   // threads per workgroup
constexpr int SLAB8 = 4;   // 8-element k chunks per slab (32 k)

struct PairArgs {
  const u4* Ah;   // [M][ldk8] chunks of W's high parts
  const u4* Al;   // and of the remainders
  int64_t ldk8;
  const u4* Bh;   // [K8][N] chunks of the expanded operand, high parts
  const u4* Bl;
  float* C;       // [M][N]
  int M, N, K8;   // K8: k chunks, a multiple of SLAB8
  int mtiles, ntiles;
  int nc, vc;     // column block width (one j) and chunks per k segment (vp / 8)
};

template <int N> struct IC { static constexpr int value = N; };

__device__ __forceinline__ bf8 as_bf8(u4 x) { return __builtin_bit_cast(bf8, x); }
__device__ __forceinline__ gu4 to_global(const u4* q) {
  return reinterpret_cast<gu4>(reinterpret_cast<uintptr_t>(q));
}

template <int BN>
__global__ __launch_bounds__(PNT, 1) void pairs_gemm_kernel(PairArgs p) {
  constexpr int WNW = BN / 2;               // columns per wavefront
  constexpr int NB = WNW / 16;              // 16-column blocks per wavefront
  constexpr int AH = PBM * SLAB8 / PNT;     // A chunks per thread, slab and half (2)
  constexpr int BH = BN * SLAB8 / PNT;      // B chunks per thread, slab and half (1 or 2)
  __shared__ u4 As[2][PBM][2 * SLAB8];      // [buffer][row][hi chunks 0-3, lo chunks 4-7]
  __shared__ u4 Bs[2][BN][2 * SLAB8];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  constexpr int GM = 8;
  const int ntot = p.mtiles * p.ntiles;
  const int T8 = (ntot + 7) / 8;
  const int L = (int)(blockIdx.x & 7) * T8 + (int)(blockIdx.x >> 3);
  if (L >= ntot) return;
  const int grp = L / (GM * p.ntiles);
  const int rows = min(GM, p.mtiles - grp * GM);
  const int idx = L - grp * GM * p.ntiles;
  const int mt = grp * GM + idx % rows, nt = idx / rows;
  const int m0 = mt * PBM, n0 = nt * BN;
  const int nslab = p.K8 / SLAB8;
  // slabs [zlo, zhi) lie wholly inside the tile's zero segment m = j
  const int j = n0 / p.nc;
  const int zlo = (j * p.vc + SLAB8 - 1) / SLAB8, zhi = ((j + 1) * p.vc) / SLAB8;
  auto skip = [&](int s) { return (s >= zlo && s < zhi) ? zhi : s; };

  // staging ownership: A chunk f (= tid + PNT h) is row f / 4, chunk f % 4 (four consecutive
  // lanes read one row's 64 bytes); B chunk f is column f % BN, chunk f / BN (consecutive
  // lanes read consecutive columns: 1 KB contiguous per wavefront)
  gu4 ga[2][AH];
  int arow[AH], aq[AH];
#pragma unroll
  for (int h = 0; h < AH; ++h) {
    const int f = tid + PNT * h;
    arow[h] = f >> 2;
    aq[h] = f & 3;
    const int64_t off = (int64_t)min(m0 + arow[h], p.M - 1) * p.ldk8 + aq[h];
    ga[0][h] = to_global(p.Ah + off);
    ga[1][h] = to_global(p.Al + off);
  }
  gu4 gb[2][BH];
  int bcol[BH], bq[BH];
#pragma unroll
  for (int h = 0; h < BH; ++h) {
    const int f = tid + PNT * h;
    bcol[h] = f % BN;
    bq[h] = f / BN;
    const int64_t off = (int64_t)bq[h] * p.N + n0 + bcol[h];
    gb[0][h] = to_global(p.Bh + off);
    gb[1][h] = to_global(p.Bl + off);
  }
  const int64_t bstep = (int64_t)SLAB8 * p.N;   // chunks between slabs of B

  // two register sets: the loads of a slab are issued two slabs before it is computed, so
  // they have a whole slab of matrix work more to land than with one set
  u4 ra[2][2][AH], rb[2][2][BH];   // [set][hi, lo][chunk]
  auto load = [&](auto SETC, int s) {
    constexpr int q = decltype(SETC)::value;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int h = 0; h < AH; ++h) ra[q][t][h] = ga[t][h][(int64_t)s * SLAB8];
#pragma unroll
      for (int h = 0; h < BH; ++h) rb[q][t][h] = gb[t][h][(int64_t)s * bstep];
    }
  };
  auto store = [&](auto SETC, int b) {
    constexpr int q = decltype(SETC)::value;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
      for (int h = 0; h < AH; ++h) As[b][arow[h]][(4 * t + aq[h]) ^ (arow[h] & 7)] = ra[q][t][h];
#pragma unroll
      for (int h = 0; h < BH; ++h) Bs[b][bcol[h]][(4 * t + bq[h]) ^ (bcol[h] & 7)] = rb[q][t][h];
    }
  };

  f4 acc[4][NB];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < NB; ++q) acc[i][q] = f4{0, 0, 0, 0};

  const int r16 = lane & 15, kq = lane >> 4;
  auto compute = [&](int b) {
    bf8 ah[4], al[4], bh[NB], bl[NB];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = wm * 64 + i * 16 + r16;
      ah[i] = as_bf8(As[b][r][kq ^ (r & 7)]);
      al[i] = as_bf8(As[b][r][(4 + kq) ^ (r & 7)]);
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int c = wn * WNW + q * 16 + r16;
      bh[q] = as_bf8(Bs[b][c][kq ^ (c & 7)]);
      bl[q] = as_bf8(Bs[b][c][(4 + kq) ^ (c & 7)]);
    }
    // lo.hi, hi.lo, then hi.hi, in separate passes over the blocks, so that no MFMA waits on
    // the previous one's accumulator
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < NB; ++q)
          acc[i][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              t == 0 ? al[i] : ah[i], t == 1 ? bl[q] : bh[q], acc[i][q], 0, 0, 0);
  };

  // At the top of a step LDS buffer `cur` holds slab s and register set P holds slab s1 (in
  // flight); the loads of the slab after s1 go to the other set, which is free. At least one
  // slab lies outside the zero segment (o >= 2).
  int s = skip(0);
  int s1 = skip(s + 1);
  load(IC<0>{}, s);
  if (s1 < nslab) load(IC<1>{}, s1);
  store(IC<0>{}, 0);
  __syncthreads();
  int cur = 0;
  auto step = [&](auto PC) -> bool {
    constexpr int P = decltype(PC)::value;
    const int s2 = s1 < nslab ? skip(s1 + 1) : nslab;
    if (s2 < nslab) load(IC<P ^ 1>{}, s2);
    compute(cur);
    if (s1 >= nslab) return false;
    store(IC<P>{}, cur ^ 1);
    __syncthreads();
    cur ^= 1;
    s = s1;
    s1 = s2;
    return true;
  };
  while (step(IC<1>{}) && step(IC<0>{})) {
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int col = n0 + wn * WNW + q * 16 + r16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wm * 64 + i * 16 + 4 * kq + e;
        if (row < p.M) p.C[(int64_t)row * p.N + col] = acc[i][q][e];
      }
    }
}

// R[g][n] (8 k values of chunk g for column n = (j, c)) as bf16 pairs from the packed FP32
// block X2[(pair, e)][ldx]: k = 8 g + t = m vp + e; r_mj^e[c] = X2[pair(m,j) v + e][c] for
// m < j, its negative for m > j, zero for m = j, e >= v or m >= o.
__global__ void pairs_expand_kernel(const float* __restrict__ X2, int64_t ldx, int o, int v,
                                    int vc, int nc, int K8, int64_t N, u4* __restrict__ Bh,
                                    u4* __restrict__ Bl) {
  const int64_t total = (int64_t)K8 * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(idx / N);
    const int64_t n = idx - (int64_t)g * N;
    const int m = g / vc, e0 = (g - m * vc) * 8;
    const int j = (int)(n / nc), c = (int)(n - (int64_t)j * nc);
    float x[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) x[t] = 0.0f;
    if (m < o && m != j) {
      const int lo = min(m, j), hi = max(m, j);
      const int64_t pr = pair_of(lo, hi, o);
      const float* src = X2 + (pr * v + e0) * ldx + c;
      const bool neg = m > j;
#pragma unroll
      for (int t = 0; t < 8; ++t)
        if (e0 + t < v) x[t] = neg ? -src[(int64_t)t * ldx] : src[(int64_t)t * ldx];
    }
    u4 h, l;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // round to nearest even on the packed converter; bf16 -> f32 is exact
      const f2 xv = {x[2 * u], x[2 * u + 1]};
      const b2 hv = __builtin_convertvector(xv, b2);
      const f2 hf = __builtin_convertvector(hv, f2);
      const f2 rem = {xv[0] - hf[0], xv[1] - hf[1]};
      h[u] = __builtin_bit_cast(unsigned, hv);
      l[u] = __builtin_bit_cast(unsigned, __builtin_convertvector(rem, b2));
    }
    Bh[idx] = h;
    Bl[idx] = l;
  }
}

// A plain FP32 operand B[K][N] (row stride ldb) as chunked pairs [K8][ldb8]: chunk (g, n) holds
// k = 8g .. 8g + 7 of column n, zeros for k >= K and n >= N
__global__ void pairs_chunk_kernel(const float* __restrict__ B, int64_t ldb, int K, int N,
                                   int K8, int64_t ldb8, u4* __restrict__ Bh,
                                   u4* __restrict__ Bl) {
  const int64_t total = (int64_t)K8 * ldb8;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int g = (int)(idx / ldb8);
    const int64_t n = idx - (int64_t)g * ldb8;
    float x[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int k = 8 * g + t;
      x[t] = (k < K && n < N) ? B[(int64_t)k * ldb + n] : 0.0f;
    }
    u4 h, l;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const f2 xv = {x[2 * u], x[2 * u + 1]};
      const b2 hv = __builtin_convertvector(xv, b2);
      const f2 hf = __builtin_convertvector(hv, f2);
      const f2 rem = {xv[0] - hf[0], xv[1] - hf[1]};
      h[u] = __builtin_bit_cast(unsigned, hv);
      l[u] = __builtin_bit_cast(unsigned, __builtin_convertvector(rem, b2));
    }
    Bh[idx] = h;
    Bl[idx] = l;
  }
}

// A[r][k] = S[r rs + k cs] as bf16 pairs [Mpad][ldk] (zeros for r >= M or k >= K)
__global__ void pairs_split_general_kernel(const double* __restrict__ S, int64_t rs, int64_t cs,
                                           int64_t M, int64_t K, int64_t Mpad, int64_t ldk,
                                           __hip_bfloat16* __restrict__ hi,
                                           __hip_bfloat16* __restrict__ lo) {
  const int64_t total = Mpad * ldk;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ldk, k = i - r * ldk;
    const double x = (r < M && k < K) ? S[r * rs + k * cs] : 0.0;
    const __hip_bfloat16 h = __float2bfloat16((float)x);
    hi[i] = h;
    lo[i] = __float2bfloat16((float)(x - (double)__bfloat162float(h)));
  }
}

// C[m][n] (+)= sum_z part[z][m][n]
__global__ void pairs_reduce_kernel(const float* __restrict__ part, int nz, int M, int N,
                                    int64_t pstride, float* __restrict__ C, int64_t ldc,
                                    int accumulate) {
  const int64_t total = (int64_t)M * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(i / N), n = (int)(i - (int64_t)m * N);
    float acc = 0.0f;
    for (int z = 0; z < nz; ++z) acc += part[z * pstride + i];
    float* cp = C + (int64_t)m * ldc + n;
    *cp = accumulate ? *cp + acc : acc;
  }
}

// W[r][k'] pairs from the FP64 ovvo matrix S[r][(m, e)] (ld o v) for rows r < Mpad: k' =
// m vp + e, zero for e >= v, m >= o or r >= M; hi = bf16(x), lo = bf16(x - hi)
__global__ void pairs_split_rows_kernel(const double* __restrict__ S, int64_t M, int64_t Mpad,
                                        int o, int v, int vp, int64_t ldk,
                                        __hip_bfloat16* __restrict__ hi,
                                        __hip_bfloat16* __restrict__ lo) {
  const int64_t total = Mpad * ldk;
  const int64_t ov = (int64_t)o * v;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / ldk;
    const int k = (int)(i - r * ldk);
    const int m = k / vp, e = k - m * vp;
    const double x = (r < M && m < o && e < v) ? S[r * ov + (int64_t)m * v + e] : 0.0;
    const __hip_bfloat16 h = __float2bfloat16((float)x);
    hi[i] = h;
    lo[i] = __float2bfloat16((float)(x - (double)__bfloat162float(h)));
  }
}

// The same product on 256 x 256 tiles with 8 wavefronts of 64 x 128 (two per SIMD, the 128
// FP32 accumulators of a wavefront in its accumulation registers). The tiles move from global
// memory to LDS by direct loads (global_load_lds_dwordx4: each lane's 16 bytes land at the
// instruction's LDS base + 16 x lane), so they pass through no vector registers: lane i of an
// instruction filling LDS rows R..R+7 loads the chunk that belongs at row R + i / 8, position
// i % 8, i.e. logical chunk (i % 8) ^ ((i / 8) & 7) of that row. Per wavefront and slab, 96
// MFMAs read 24 fragments (4 per fragment, against 3 for the 64 x 64 wavefront tiles above).
// Two LDS buffers (128 KB): the next slab's direct loads run while the current slab's MFMAs
// do; one barrier per slab.
struct Pair8Args {
  const u4* A;     // W pairs: high parts at A, remainders at A + a_lo (chunks, [Mpad][ldk8])
  int64_t a_lo;
  int64_t ldk8;
  const u4* B;     // expanded operand: high parts at B, remainders at B + b_lo ([K8][ldb8])
  int64_t b_lo;
  int64_t ldb8;    // chunk-row stride of B (a multiple of 256 columns)
  float* C;        // C (+)= A B, row stride ldc; split z writes C + z pstride
  int64_t ldc, pstride;
  int M, N, K8;    // N: columns stored (B's columns past N are zero)
  int mtiles, ntiles;
  int nc, vc;      // zero-segment skip of the ovvo operand (vc = 0: none)
  int nsplit, spz; // split-K: nsplit ranges of spz slabs
  int accumulate;  // add to C instead of storing
};

// One direct load: 16 bytes per lane from gsrc to LDS at lds_off + 16 x lane. Written as
// inline assembly so that the compiler, which does not see the LDS write, does not wait for
// the load before later LDS reads (it cannot tell this tile buffer from the other one and
// otherwise waits for every direct load right after issuing it). The kernel orders the loads
// itself: s_waitcnt before the barrier that precedes any read of the buffer they fill. The
// asm has no result register (nothing of it is in flight in a register).
__device__ __forceinline__ void dma16(const void* gsrc, unsigned lds_off) {
  asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
               :
               : "v"(gsrc), "s"(__builtin_amdgcn_readfirstlane(lds_off))
               : "m0");
}

__global__ __launch_bounds__(512, 1) void pairs_gemm8_kernel(Pair8Args p) {
  constexpr int BM = 256, BN = 256;
  // the two buffers are separate variables, so that the compiler can tell the direct loads into
  // one from the fragment reads of the other and does not wait for the loads before the reads
  __shared__ u4 As0[BM][8], As1[BM][8], Bs0[BN][8], Bs1[BN][8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  constexpr int GM = 8;
  const int ntot = p.mtiles * p.ntiles;
  const int nwork = ntot * p.nsplit;  // (split, tile) pairs, tile-fastest
  const int T8 = (nwork + 7) / 8;
  const int Lw = (int)(blockIdx.x & 7) * T8 + (int)(blockIdx.x >> 3);
  if (Lw >= nwork) return;
  const int z = Lw / ntot;
  const int L = Lw - z * ntot;
  const int grp = L / (GM * p.ntiles);
  const int rows = min(GM, p.mtiles - grp * GM);
  const int idx = L - grp * GM * p.ntiles;
  const int mt = grp * GM + idx % rows, nt = idx / rows;
  const int m0 = mt * BM, n0 = nt * BN;
  // this workgroup's slabs: [sbeg, nslab)
  const int sbeg = z * p.spz;
  const int nslab = min(p.K8 / SLAB8, sbeg + p.spz);
  const int j = n0 / p.nc;
  const int zlo = (j * p.vc + SLAB8 - 1) / SLAB8, zhi = ((j + 1) * p.vc) / SLAB8;
  auto skip = [&](int s) { return (s >= zlo && s < zhi) ? zhi : s; };

  // direct-load sources: instruction t (0..3) of this wavefront fills rows (columns)
  // R = (4 wave + t) 8 .. R + 7 of the A (B) tile; lane i serves row R + i / 8, whose
  // (row & 7) is (i / 8) & 7 for every t, so its logical chunk c is fixed and the sources of
  // the instructions and of every slab follow from one base by uniform steps (W has its rows
  // padded with zeros to a multiple of 256, so no row index needs a clamp)
  const int c = (lane & 7) ^ ((lane >> 3) & 7);
  const u4* sa = p.A + (c >= 4 ? p.a_lo : 0) + (int64_t)(m0 + 32 * wave + (lane >> 3)) * p.ldk8 +
                 (c & 3);
  const u4* sb = p.B + (c >= 4 ? p.b_lo : 0) + (int64_t)(c & 3) * p.ldb8 + n0 + 32 * wave +
                 (lane >> 3);
  const int64_t astep_t = 8 * p.ldk8, bstep_s = (int64_t)SLAB8 * p.ldb8;
  auto issue = [&](auto BUFC, int s) {
    constexpr int b = decltype(BUFC)::value;
    u4(*As)[8] = b ? As1 : As0;
    u4(*Bs)[8] = b ? Bs1 : Bs0;
    const u4* a = sa + (int64_t)s * SLAB8;
    const u4* bb = sb + (int64_t)s * bstep_s;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int R = (4 * wave + t) * 8;
      dma16(a + t * astep_t, (unsigned)(uintptr_t)&As[R][0]);
      dma16(bb + 8 * t, (unsigned)(uintptr_t)&Bs[R][0]);
    }
  };

  f4 acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[i][q] = f4{0, 0, 0, 0};

  const int r16 = lane & 15, kq = lane >> 4;
  // fragment rows of this lane: row (column) 16 i + r16 + a multiple of 64 has (row & 7) =
  // r16 & 7, so chunk c sits at position c ^ (r16 & 7) in every block
  const int sw = r16 & 7;
  const int arow0 = wm * 64 + r16, bcol0 = wn * 128 + r16;
  auto fence = []() { __builtin_amdgcn_sched_barrier(0); };
  auto mfma = [&](const bf8* a, const bf8* bv) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 8; ++q)
        acc[i][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bv[q], acc[i][q], 0, 0, 0);
  };
  auto read_a = [&](auto BUFC, int half, bf8* a) {
    u4(*As)[8] = decltype(BUFC)::value ? As1 : As0;
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = as_bf8(As[arow0 + 16 * i][(4 * half + kq) ^ sw]);
  };
  auto read_b = [&](auto BUFC, int half, bf8* bv) {
    u4(*Bs)[8] = decltype(BUFC)::value ? Bs1 : Bs0;
#pragma unroll
    for (int q = 0; q < 8; ++q) bv[q] = as_bf8(Bs[bcol0 + 16 * q][(4 * half + kq) ^ sw]);
  };
  // Per slab three passes of 32 MFMAs: lo.hi (A's remainders, B's high parts), hi.hi, hi.lo.
  // Each pass carries the fragment reads of the next between its MFMAs. After the second pass
  // every fragment of the slab is in registers, so the barrier sits there: past it the
  // buffer of this slab takes the direct loads of the slab after next, and the third pass
  // runs while the first fragments of the next slab are read, so no pass starts on an empty
  // pipe.
  int s = skip(sbeg);
  int s1 = skip(s + 1);
  issue(IC<0>{}, s);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  issue(IC<1>{}, s1 < nslab ? s1 : s);
  bf8 al[4], bh[8];
  read_a(IC<0>{}, 1, al);
  read_b(IC<0>{}, 0, bh);
  // one slab from buffer B (compile-time, the loop runs two slabs per trip)
  auto step = [&](auto BUFC) -> bool {
    constexpr int b = decltype(BUFC)::value;
    bf8 ah[4], bl[8];
    fence();
    mfma(al, bh);
    read_a(IC<b>{}, 0, ah);
    fence();
    mfma(ah, bh);
    read_b(IC<b>{}, 1, bl);
    fence();
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    // past the last slab the loads repeat a valid slab into a buffer nobody reads again, and
    // the reads below fetch fragments nobody uses: no branch around them
    const int s2 = s1 < nslab ? skip(s1 + 1) : nslab;
    issue(IC<b>{}, s2 < nslab ? s2 : s);
    fence();
    mfma(ah, bl);
    read_a(IC<b ^ 1>{}, 1, al);
    read_b(IC<b ^ 1>{}, 0, bh);
    fence();
    if (s1 >= nslab) return false;
    s = s1;
    s1 = s2;
    return true;
  };
  while (step(IC<0>{}) && step(IC<1>{})) {
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int col = n0 + wn * 128 + q * 16 + r16;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int row = m0 + wm * 64 + i * 16 + 4 * kq + e;
        if (row < p.M && col < p.N) {
          float* cp = p.C + (int64_t)z * p.pstride + (int64_t)row * p.ldc + col;
          *cp = p.accumulate ? *cp + acc[i][q][e] : acc[i][q][e];
        }
      }
    }
}

inline unsigned grid_cap(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

int64_t pairs_ldk(int o, int v) {
  const int64_t vp = (v + 7) / 8 * 8;
  return (vp * o + 8 * SLAB8 - 1) / (8 * SLAB8) * (8 * SLAB8);
}

int64_t pairs_rows(int o, int v) { return ((int64_t)o * v + 255) / 256 * 256; }

void pairs_split_rows(gfcc_ctx* ctx, const double* S, int o, int v, void* hi, void* lo) {
  const int64_t M = (int64_t)o * v, Mpad = pairs_rows(o, v), ldk = pairs_ldk(o, v);
  const int vp = (v + 7) / 8 * 8;
  hipLaunchKernelGGL(pairs_split_rows_kernel, dim3(grid_cap(Mpad * ldk)), dim3(256), 0,
                     ctx->stream, S, M, Mpad, o, v, vp, ldk, static_cast<__hip_bfloat16*>(hi),
                     static_cast<__hip_bfloat16*>(lo));
  GFCC_LAUNCH_CHECK();
}

int64_t pairs_pad_rows(int64_t M) { return (M + 255) / 256 * 256; }
int64_t pairs_pad_k(int64_t K) { return (K + 8 * SLAB8 - 1) / (8 * SLAB8) * (8 * SLAB8); }

void pairs_split_general(gfcc_ctx* ctx, const double* S, int64_t rs, int64_t cs, int64_t M,
                         int64_t K, void* hi, void* lo) {
  const int64_t Mpad = pairs_pad_rows(M), ldk = pairs_pad_k(K);
  hipLaunchKernelGGL(pairs_split_general_kernel, dim3(grid_cap(Mpad * ldk)), dim3(256), 0,
                     ctx->stream, S, rs, cs, M, K, Mpad, ldk, static_cast<__hip_bfloat16*>(hi),
                     static_cast<__hip_bfloat16*>(lo));
  GFCC_LAUNCH_CHECK();
}

void pairs_gemm(gfcc_ctx* ctx, const void* Ah, const void* Al, int M, int K, const float* B,
                int64_t ldb, int N, float* C, int64_t ldc, bool accumulate) {
  if (M <= 0 || N <= 0) return;
  GFCC_REQUIRE(K >= 0 && ldb >= N && ldc >= N, GFCC_EINVAL, "pairs_gemm: bad shape");
  GFCC_REQUIRE(reinterpret_cast<uintptr_t>(Ah) % 16 == 0 && reinterpret_cast<uintptr_t>(Al) % 16 == 0,
               GFCC_EINVAL, "pairs_gemm: operand pairs not 16-byte aligned");
  const int64_t Mpad = pairs_pad_rows(M), ldk = pairs_pad_k(K), K8 = ldk / 8;
  const int64_t ldb8 = ((int64_t)N + 255) / 256 * 256;
  GFCC_REQUIRE(K8 * ldb8 < (1LL << 40) && Mpad < (1LL << 31), GFCC_EINVAL,
               "pairs_gemm: operand too large");
  // B as chunked pairs in the pair workspace
  const size_t bbytes = sizeof(u4) * (size_t)(K8 * ldb8);
  ws_ensure(ctx, ctx->ws_pairs, 2 * bbytes);
  u4* Bh = ctx->ws_pairs.as<u4>();
  u4* Bl = reinterpret_cast<u4*>(ctx->ws_pairs.as<char>() + bbytes);
  hipLaunchKernelGGL(pairs_chunk_kernel, dim3(grid_cap(K8 * ldb8)), dim3(256), 0, ctx->stream,
                     B, ldb, K, N, (int)K8, ldb8, Bh, Bl);
  GFCC_LAUNCH_CHECK();
  Pair8Args q{};
  q.A = static_cast<const u4*>(Ah);
  q.a_lo = (reinterpret_cast<intptr_t>(Al) - reinterpret_cast<intptr_t>(Ah)) / (intptr_t)sizeof(u4);
  q.ldk8 = K8;
  q.B = Bh;
  q.b_lo = K8 * ldb8;
  q.ldb8 = ldb8;
  q.M = M;
  q.N = N;
  q.K8 = (int)K8;
  q.mtiles = (int)(Mpad / 256);
  q.ntiles = (int)(ldb8 / 256);
  q.nc = (int)ldb8;  // one column block: no zero segment
  q.vc = 0;
  const int nslab = (int)(K8 / SLAB8);
  const int64_t tiles = (int64_t)q.mtiles * q.ntiles;
  // split-K when the tiles cannot fill the GPU's 256 CUs (one workgroup each): about 1024
  // (split, tile) pairs, each at least 8 slabs deep
  int nz = 1;
  if (tiles < 512 && nslab >= 16)
    nz = (int)std::min<int64_t>(nslab / 8, (1024 + tiles - 1) / tiles);
  q.spz = (nslab + nz - 1) / nz;
  nz = (nslab + q.spz - 1) / q.spz;
  q.nsplit = nz;
  float* part = nullptr;
  if (nz > 1) {
    q.pstride = (int64_t)M * N;
    ws_ensure(ctx, ctx->ws_gemm, sizeof(float) * (size_t)q.pstride * nz);
    part = ctx->ws_gemm.as<float>();
    q.C = part;
    q.ldc = N;
    q.accumulate = 0;
  } else {
    q.C = C;
    q.ldc = ldc;
    q.accumulate = accumulate ? 1 : 0;
  }
  const int64_t work = tiles * nz;
  GFCC_REQUIRE(work < (1LL << 31) - 8, GFCC_EINVAL, "pairs_gemm: too many tiles");
  hipLaunchKernelGGL(pairs_gemm8_kernel, dim3((unsigned)((work + 7) / 8 * 8)), dim3(512), 0,
                     ctx->stream, q);
  GFCC_LAUNCH_CHECK();
  if (nz > 1) {
    hipLaunchKernelGGL(pairs_reduce_kernel, dim3(grid_cap((int64_t)M * N)), dim3(256), 0,
                       ctx->stream, part, nz, M, N, q.pstride, C, ldc, accumulate ? 1 : 0);
    GFCC_LAUNCH_CHECK();
  }
}

bool ovvo_bf3(gfcc_ctx* ctx, int o, int v, int nc, const void* Wh, const void* Wl,
              const float* X2, int64_t ldx, float* Z) {
  if (o < 2 || v < 1 || nc < 128 || nc % 128 != 0 || ldx < nc) return false;
  if (!Wh || !Wl || reinterpret_cast<uintptr_t>(Wh) % 16 != 0 ||
      reinterpret_cast<uintptr_t>(Wl) % 16 != 0)
    return false;
  const int64_t OV = (int64_t)o * v, ldk = pairs_ldk(o, v), N = (int64_t)o * nc;
  const int vp = (v + 7) / 8 * 8;
  const int64_t K8 = ldk / 8;
  if (OV >= (1LL << 30) || N >= (1LL << 31) || K8 * N >= (1LL << 40)) return false;
  constexpr int BN = 128;  // 256-column tiles need more than the 256 registers of a wavefront at two per SIMD
  // the expanded operand, hi and lo chunks
  const size_t rbytes = sizeof(u4) * (size_t)(K8 * N);
  ws_ensure(ctx, ctx->ws_pairs, 2 * rbytes);
  u4* Bh = ctx->ws_pairs.as<u4>();
  u4* Bl = reinterpret_cast<u4*>(ctx->ws_pairs.as<char>() + rbytes);
  hipLaunchKernelGGL(pairs_expand_kernel, dim3(grid_cap(K8 * N)), dim3(256), 0, ctx->stream, X2,
                     ldx, o, v, vp / 8, nc, (int)K8, N, Bh, Bl);
  GFCC_LAUNCH_CHECK();
  if (nc % 256 == 0) {
    Pair8Args q{};
    q.A = static_cast<const u4*>(Wh);
    q.a_lo = (reinterpret_cast<intptr_t>(Wl) - reinterpret_cast<intptr_t>(Wh)) /
             (intptr_t)sizeof(u4);
    q.ldk8 = K8;
    q.B = Bh;
    q.b_lo = K8 * N;
    q.ldb8 = N;
    q.C = Z;
    q.ldc = N;
    q.M = (int)OV;
    q.N = (int)N;
    q.K8 = (int)K8;
    q.mtiles = (int)(pairs_rows(o, v) / 256);
    q.ntiles = (int)(N / 256);
    q.nc = nc;
    q.vc = vp / 8;
    q.nsplit = 1;
    q.spz = (int)(K8 / SLAB8);
    const int64_t tiles = (int64_t)q.mtiles * q.ntiles;
    if (tiles >= (1LL << 31) - 8) return false;
    hipLaunchKernelGGL(pairs_gemm8_kernel, dim3((unsigned)((tiles + 7) / 8 * 8)), dim3(512), 0,
                       ctx->stream, q);
    GFCC_LAUNCH_CHECK();
    return true;
  }
  PairArgs p{};
  p.Ah = static_cast<const u4*>(Wh);
  p.Al = static_cast<const u4*>(Wl);
  p.ldk8 = K8;
  p.Bh = Bh;
  p.Bl = Bl;
  p.C = Z;
  p.M = (int)OV;
  p.N = (int)N;
  p.K8 = (int)K8;
  p.mtiles = (int)((OV + PBM - 1) / PBM);
  p.ntiles = (int)(N / BN);
  p.nc = nc;
  p.vc = vp / 8;
  const int64_t tiles = (int64_t)p.mtiles * p.ntiles;
  if (tiles >= (1LL << 31) - 8) return false;
  const dim3 grid((unsigned)((tiles + 7) / 8 * 8));
  hipLaunchKernelGGL(pairs_gemm_kernel<BN>, grid, dim3(PNT), 0, ctx->stream, p);
  GFCC_LAUNCH_CHECK();
  return true;
}

}  // namespace gfcc
