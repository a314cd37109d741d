// The ovvo contraction of the IP sigma product on FP64/FP32 matrix cores:
//   Z[(i,a)][(j,c)] = sum_(m,e) W[(i,a)][(m,e)] r_mj^e[c],     r_mj^e = +-X2[pair(m,j)][e][c]
// (91% of the sigma flops at the benzene/cc-pVDZ shape). r is the antisymmetric expansion of
// the packed two-hole-one-particle block (r_mj = X2[pair(m,j)] for m < j, -X2[pair(j,m)] for
// m > j, zero for m = j); it is generated while the B tile is loaded, so the expanded operand
// (twice the size of X2) never exists in memory.
//
// Tile 128 x 128 x BK (one slab is 128 bytes of k: BK = 16 for FP64, 32 for FP32), 256 threads
// as 2 x 2 wavefronts of 64 x 64 = 4 x 4 MFMA 16x16x4 blocks, two workgroups per CU.
//
// Pipeline. Global loads run two slabs ahead of the matrix work and LDS stores one slab ahead:
// while slab s feeds the MFMAs from one LDS buffer, the registers loaded during slab s-1 are
// written to the other buffer and the loads of slab s+2 are issued under the first k-steps.
// Fragments are read one k-step ahead, and the single barrier per slab sits before the last
// k-step, whose MFMAs cover the latency of the next slab's first fragment reads.
//
// LDS holds both tiles k-contiguous ([row][k]) with a 136-byte pitch, which keeps the
// per-k-step fragment reads (lanes 0-15 on 16 rows) and the 8-byte stores free of bank
// conflicts.
//
// B operand. Each thread owns one column n = (j, c) of the tile and RB = BK/2 consecutive rows
// k = (m, e) of every slab; the rows are the same for all lanes of a wavefront, so the (m, e)
// position is scalar. Two loaders:
//  - column-block (nc a multiple of 128): a tile's columns share one j, so liveness, sign and
//    the X2 row address of every row are scalar; a structurally zero row (m = j, or k past
//    the end) is read from a row of zeros, and the sign costs one XOR per row;
//  - general: j varies across the tile; a slab of BK <= v rows crosses at most one m boundary,
//    so two per-lane row bases (for m and m+1) and a scalar carry per row give every address,
//    and liveness / sign are per-lane selects.
#include "common.h"

namespace gfcc {
namespace {

constexpr int BM = 128, BN = 128, NT = 256;

template <typename T> struct MF;
template <> struct MF<double> {
  typedef double C4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ C4 op(double a, double b, C4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
  static __device__ __forceinline__ double flip(double x, unsigned neg) {  // neg: 0 or 1
    return __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, x) ^
                                          ((unsigned long long)neg << 63));
  }
};
template <> struct MF<float> {
  typedef float C4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ C4 op(float a, float b, C4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
  static __device__ __forceinline__ float flip(float x, unsigned neg) {
    return __builtin_bit_cast(float, __builtin_bit_cast(unsigned, x) ^ (neg << 31));
  }
};

template <typename T> struct OvvoArgs {
  const T* W;        // [M][K] (or [K][M] when transposed), followed by zero padding
  const T* X2;       // packed 2h1p block [(pair, e)][ldx]
  const T* zrow;     // >= nc zeros (column-block loader)
  T* Z;              // [M][N]
  int o, v, nc;      // N = o * nc
  int M, N, K;
  int ldx;
  int mtiles, ntiles, nslabs;
};

__device__ __forceinline__ int pair_index(int i, int j, int o) {  // i < j
  return i * o - (i * (i + 1) >> 1) + (j - i - 1);
}

template <int N> struct IC { static constexpr int value = N; };

// TA: W is stored transposed ([K][M]). BLOCKJ: column-block loader (nc % 128 == 0, W padded,
// 16-byte aligned rows). VEC: 16-byte A loads (general loader only).
template <typename T, bool TA, bool BLOCKJ, bool VEC>
__global__ __launch_bounds__(NT, 2) void ovvo_kernel(OvvoArgs<T> p) {
  using M4 = MF<T>;
  using C4 = typename M4::C4;
  constexpr int BK = 128 / (int)sizeof(T);      // k per slab
  constexpr int VPC = 16 / (int)sizeof(T);      // elements per 16-byte chunk
  constexpr int VP8 = 8 / (int)sizeof(T);       // elements per 8-byte LDS store
  constexpr int LDK = BK + VP8;                 // LDS row pitch: 136 bytes
  constexpr int CPR = BK / VPC;                 // 16-byte chunks per tile row and slab (8)
  constexpr int ACH = BM * CPR / NT;            // A chunks per thread and slab (4)
  constexpr int RB = BK / 2;                    // B rows per thread and slab
  constexpr int NS = BK / 4;                    // MFMA k-steps per slab
  typedef T V16 __attribute__((ext_vector_type(VPC)));
  typedef T V8 __attribute__((ext_vector_type(VP8)));
  __shared__ __attribute__((aligned(16))) T As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][BN][LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // Tile order. Workgroups are dealt to the 8 XCDs round robin (b % 8), each XCD with its own
  // L2. XCD x is given the contiguous range [x T8, (x+1) T8) of a grouped tile order in which
  // GM consecutive M-tiles are walked down before moving to the next N-tile, so the
  // workgroups resident on one XCD at a time cover a compact block of tiles that share A and
  // B slabs.
  constexpr int GM = 8;
  const int ntot = p.mtiles * p.ntiles;
  const int T8 = (ntot + 7) / 8;
  const int L = (int)(blockIdx.x & 7) * T8 + (int)(blockIdx.x >> 3);
  if (L >= ntot) return;
  const int grp = L / (GM * p.ntiles);
  const int rows = min(GM, p.mtiles - grp * GM);
  const int idx = L - grp * GM * p.ntiles;
  const int mt = grp * GM + idx % rows, nt = idx / rows;
  const int m0 = mt * BM, n0 = nt * BN;
  const T* __restrict__ W = p.W;
  const T* __restrict__ X2 = p.X2;
  const int K = p.K, M = p.M, v = p.v, o = p.o, ldx = p.ldx;

  // ---- B ownership: column bn, rows kh * RB + r of every slab (kh is wave-uniform)
  const int bn = tid % BN;
  const int kh = __builtin_amdgcn_readfirstlane(tid / BN);
  const int first = kh * RB;
  const int n = n0 + bn;
  const bool ncol = BLOCKJ || n < p.N;
  const int jt = n0 / p.nc;                                  // column-block: the tile's j
  const int j = BLOCKJ ? jt : (ncol ? n / p.nc : 0);
  const int c = ncol ? n - j * p.nc : 0;

  // ---- A ownership. Column-block loader: per-lane base pointers advanced by the slab offset;
  // reads past k = K land in the next row or in the zero padding after W, against B rows
  // that are zero.
  const T* wa[ACH];
  if (BLOCKJ) {
#pragma unroll
    for (int r = 0; r < ACH; ++r) {
      if (!TA) {
        const int row = min(m0 + tid / CPR + (NT / CPR) * r, M - 1);
        wa[r] = W + (int64_t)row * K + (tid % CPR) * VPC;
      } else {
        const int f = tid + NT * r;
        const int mm = min(m0 + (f % (BM / VPC)) * VPC, M - VPC);
        wa[r] = W + (int64_t)(f / (BM / VPC)) * M + mm;
      }
    }
  }

  // slab position being loaded: k0 = ms * v + es (scalar)
  int ms = 0, es = 0;
  T ra[ACH][VPC];
  T rb[RB];
  unsigned nbits = 0;                                      // column-block: row r negated
  bool l0 = false, l1 = false, g0 = false, g1 = false;    // general: live / negated, m and m+1
  unsigned cbits = 0;                                      // general: row r uses base m+1
  // element offset of X2[pair(m, j)][0][c], or 0 when the row is structurally zero (general)
  auto rowbase = [&](int m, bool& live, bool& neg) -> int {
    live = ncol && m < o && m != j;
    neg = m > j;
    const int lo = m < j ? m : j, hi = m < j ? j : m;
    return live ? pair_index(lo, hi, o) * v * ldx + c : 0;
  };

  auto load = [&](int k0) {
    // ---- A
    if (BLOCKJ) {
#pragma unroll
      for (int r = 0; r < ACH; ++r) {
        const V16 x = *reinterpret_cast<const V16*>(wa[r] + (TA ? (int64_t)k0 * M : k0));
#pragma unroll
        for (int u = 0; u < VPC; ++u) ra[r][u] = x[u];
      }
    } else if (!TA) {
      if (VEC) {
#pragma unroll
        for (int r = 0; r < ACH; ++r) {
          const int row = m0 + tid / CPR + (NT / CPR) * r, k = k0 + (tid % CPR) * VPC;
          const int rr = row < M ? row : M - 1, kk = k < K ? k : K - VPC;
          const V16 x = *reinterpret_cast<const V16*>(W + (int64_t)rr * K + kk);
#pragma unroll
          for (int u = 0; u < VPC; ++u) ra[r][u] = x[u];
        }
      } else {
#pragma unroll
        for (int r = 0; r < ACH; ++r)
#pragma unroll
          for (int u = 0; u < VPC; ++u) {
            const int f = tid + NT * (r * VPC + u);
            const int row = m0 + f / BK, k = k0 + f % BK;
            const int rr = row < M ? row : M - 1, kk = k < K ? k : K - 1;
            ra[r][u] = W[(int64_t)rr * K + kk];
          }
      }
    } else {
      // W stored [K][M]: chunks run along m
#pragma unroll
      for (int r = 0; r < ACH; ++r) {
        const int f = tid + NT * r;
        const int k = k0 + f / (BM / VPC), mm = m0 + (f % (BM / VPC)) * VPC;
        const int kk = k < K ? k : K - 1;
        if (VEC) {
          const int rr = mm < M ? mm : M - VPC;
          const V16 x = *reinterpret_cast<const V16*>(W + (int64_t)kk * M + rr);
#pragma unroll
          for (int u = 0; u < VPC; ++u) ra[r][u] = x[u];
        } else {
#pragma unroll
          for (int u = 0; u < VPC; ++u) {
            const int rr = mm + u < M ? mm + u : M - 1;
            ra[r][u] = W[(int64_t)kk * M + rr];
          }
        }
      }
    }
    // ---- B: rows first + r of the slab; at most one carry into m
    if (BLOCKJ) {
      // Scalar row bases of the slab's first owned row in segments m and m+1: the X2 row
      // (pair(m, j), e) with stride ldx, or the zero row with stride 0. Selects are written
      // as masks so that the compiler keeps them in straight-line scalar code.
      auto base = [&](int m, int e, uint64_t& ptr, uint64_t& stride) {
        const int lo = min(m, j), hi = max(m, j);
        const int pr = lo * o - ((lo * (lo + 1)) >> 1) + hi - lo - 1;
        const uint64_t live = 0ull - (uint64_t)((m < o) & (m != j));
        const uint64_t a = reinterpret_cast<uint64_t>(X2) +
                           (uint64_t)(((int64_t)pr * v + e) * ldx) * sizeof(T);
        ptr = (a & live) | (reinterpret_cast<uint64_t>(p.zrow) & ~live);
        stride = (uint64_t)ldx * sizeof(T) & live;
      };
      uint64_t q0, q1, d0, d1;
      base(ms, es + first, q0, d0);
      base(ms + 1, es + first - v, q1, d1);
      const int rc = v - es - first;   // owned rows r >= rc lie in segment m+1
      constexpr unsigned full = (RB >= 32) ? ~0u : ((1u << RB) - 1u);
      const unsigned hi = rc <= 0 ? full : (rc >= RB ? 0u : full & ~((1u << rc) - 1u));
      nbits = (ms > j ? full & ~hi : 0u) | (ms + 1 > j ? hi : 0u);
      typedef const T __attribute__((address_space(1)))* gptr;
#pragma unroll
      for (int r = 0; r < RB; ++r) {   // all scalar but the column c
        const uint64_t mk = 0ull - (uint64_t)(r >= rc);
        const uint64_t rowp = ((q1 + r * d1) & mk) | ((q0 + r * d0) & ~mk);
        rb[r] = reinterpret_cast<gptr>(rowp)[c];
      }
    } else {
      // per-lane row bases for m and m+1
      const int b0 = rowbase(ms, l0, g0) + es * ldx;
      const int b1 = rowbase(ms + 1, l1, g1) + (es - v) * ldx;
      const int z0 = l0 ? b0 : 0, z1 = l1 ? b1 : 0;
      cbits = 0;
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        const bool carry = es + first + r >= v;   // scalar
        cbits |= carry ? 1u << r : 0u;
        rb[r] = X2[(carry ? z1 : z0) + (first + r) * ldx];
      }
    }
    const int cy = es + BK >= v;
    es = es + BK - (cy ? v : 0);
    ms += cy;
  };

  auto store = [&](auto BUFC) {
    constexpr int b = decltype(BUFC)::value;
    if (!TA && (BLOCKJ || VEC)) {
#pragma unroll
      for (int r = 0; r < ACH; ++r) {
        T* d = &As[b][tid / CPR + (NT / CPR) * r][(tid % CPR) * VPC];
#pragma unroll
        for (int h = 0; h < VPC; h += VP8) {
          V8 y;
#pragma unroll
          for (int u = 0; u < VP8; ++u) y[u] = ra[r][h + u];
          *reinterpret_cast<V8*>(d + h) = y;
        }
      }
    } else if (!TA) {
#pragma unroll
      for (int r = 0; r < ACH; ++r)
#pragma unroll
        for (int u = 0; u < VPC; ++u) {
          const int f = tid + NT * (r * VPC + u);
          As[b][f / BK][f % BK] = ra[r][u];
        }
    } else {
#pragma unroll
      for (int r = 0; r < ACH; ++r) {
        const int f = tid + NT * r;
        const int k = f / (BM / VPC), mm = (f % (BM / VPC)) * VPC;
#pragma unroll
        for (int u = 0; u < VPC; ++u) As[b][mm + u][k] = ra[r][u];
      }
    }
#pragma unroll
    for (int t = 0; t < RB; t += VP8) {
      V8 y;
#pragma unroll
      for (int u = 0; u < VP8; ++u) {
        const int r = t + u;
        if (BLOCKJ) {
          y[u] = M4::flip(rb[r], (nbits >> r) & 1u);
        } else {
          const bool cr = (cbits >> r) & 1u;
          const T x = (cr ? l1 : l0) ? rb[r] : T(0);
          y[u] = (cr ? g1 : g0) ? -x : x;
        }
      }
      *reinterpret_cast<V8*>(&Bs[b][bn][first + t]) = y;
    }
  };

  C4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[i][q] = C4{0, 0, 0, 0};

  const int row_l = lane & 15, kq = lane >> 4;
  T af[NS][4], bf[NS][4];   // fragments of the k-steps of a slab
  auto frag = [&](auto BUFC, int s) {
    constexpr int b = decltype(BUFC)::value;
#pragma unroll
    for (int i = 0; i < 4; ++i) af[s][i] = As[b][wm * 64 + i * 16 + row_l][4 * s + kq];
#pragma unroll
    for (int q = 0; q < 4; ++q) bf[s][q] = Bs[b][wn * 64 + q * 16 + row_l][4 * s + kq];
  };
  auto mfma = [&](int s) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[i][q] = M4::op(af[s][i], bf[s][q], acc[i][q]);
  };
  // One slab from LDS buffer b (its first two fragments already in registers).
  auto step = [&](auto BUFC, int kload) {
    constexpr int b = decltype(BUFC)::value;
    store(IC<b ^ 1>{});
#pragma unroll
    for (int s = 0; s + 1 < NS; ++s) {
      mfma(s);
      if (s + 2 < NS) frag(IC<b>{}, s + 2);
      if (s == 0) load(kload);
    }
    __syncthreads();
    frag(IC<b ^ 1>{}, 0);
    mfma(NS - 1);
    frag(IC<b ^ 1>{}, 1);
  };

  // prologue: slab 0 into LDS buffer 0 and its first fragments, slab 1 into registers
  load(0);
  store(IC<0>{});
  load(BK);
  __syncthreads();
  frag(IC<0>{}, 0);
  frag(IC<0>{}, 1);
  // Every step stores and loads ahead. Past the last slab the B rows are structurally zero
  // and the A reads stay in range (clamped, or in the padding after W), and the stores go to
  // the buffer that is no longer read.
  const int ns = p.nslabs;
  for (int s = 0; s < ns; s += 2) {
    step(IC<0>{}, (s + 2) * BK);
    if (s + 1 < ns) step(IC<1>{}, (s + 3) * BK);
  }

  const int col_l = lane & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int nn = n0 + wn * 64 + q * 16 + col_l;
      if (!BLOCKJ && nn >= p.N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int mrow = m0 + wm * 64 + i * 16 + M4::row(lane, e);
        if (mrow < M) p.Z[(int64_t)mrow * p.N + nn] = acc[i][q][e];
      }
    }
}

}  // namespace

// Returns false when the shape is outside what the kernels support (the caller then uses the
// generic gather path). W must be followed by ovvo_pad(M) zero elements; zrow holds at least
// nc zeros (or is null, which disables the column-block loader).
template <typename T>
bool ovvo_fast(gfcc_ctx* ctx, bool transW, int o, int v, int nc, const T* W, const T* X2,
               int64_t ldx, T* Z, const T* zrow) {
  constexpr int BK = 128 / (int)sizeof(T);
  constexpr int VPC = 16 / (int)sizeof(T);
  if (o < 2 || v < BK || nc < 1) return false;
  OvvoArgs<T> p{};
  p.W = W; p.X2 = X2; p.Z = Z; p.zrow = zrow;
  p.o = o; p.v = v; p.nc = nc;
  p.M = o * v; p.K = o * v; p.N = o * nc;
  p.mtiles = (p.M + BM - 1) / BM;
  p.ntiles = (p.N + BN - 1) / BN;
  p.nslabs = (p.K + BK - 1) / BK;
  const int64_t tiles = (int64_t)p.mtiles * p.ntiles;
  if (tiles >= (1LL << 31) - 8) return false;
  // element offsets into X2 are kept in 32 bits by the general loader
  const int64_t P = (int64_t)o * (o - 1) / 2;
  if (P * v * ldx + nc >= (1LL << 31) - 1 || (int64_t)(v + BK) * ldx >= (1LL << 30)) return false;
  p.ldx = (int)ldx;
  const bool vec = (reinterpret_cast<uintptr_t>(W) % 16 == 0) && (p.K % VPC == 0);
  const bool blockj = vec && zrow && nc % BN == 0;
  dim3 grid((unsigned)((tiles + 7) / 8 * 8));
  hipStream_t st = ctx->stream;
  if (transW) {
    if (blockj) hipLaunchKernelGGL((ovvo_kernel<T, true, true, true>), grid, dim3(NT), 0, st, p);
    else if (vec) hipLaunchKernelGGL((ovvo_kernel<T, true, false, true>), grid, dim3(NT), 0, st, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, true, false, false>), grid, dim3(NT), 0, st, p);
  } else {
    if (blockj) hipLaunchKernelGGL((ovvo_kernel<T, false, true, true>), grid, dim3(NT), 0, st, p);
    else if (vec) hipLaunchKernelGGL((ovvo_kernel<T, false, false, true>), grid, dim3(NT), 0, st, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, false, false, false>), grid, dim3(NT), 0, st, p);
  }
  GFCC_LAUNCH_CHECK();
  return true;
}

template bool ovvo_fast<double>(gfcc_ctx*, bool, int, int, int, const double*, const double*,
                                int64_t, double*, const double*);
template bool ovvo_fast<float>(gfcc_ctx*, bool, int, int, int, const float*, const float*,
                               int64_t, float*, const float*);

}  // namespace gfcc
