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
// Pipeline. LDS is double-buffered and global loads run two slabs ahead of the matrix work:
// during slab s, the registers loaded during slab s-1 are stored to the other LDS buffer and
// each store is followed by the loads of slab s+2 into the registers it freed. Fragments are
// read one k-step ahead, and the single barrier per slab sits before the last k-step, whose
// MFMAs cover the next slab's first fragment reads and the address bookkeeping of the slab
// after. The step is written as fenced slots of two MFMAs plus a small group of other work,
// so that every wavefront keeps its matrix pipe fed on its own.
//
// The same kernel also runs plain products C = alpha op(A) B + beta C with a row-major B
// (gemm_pipe): the B rows are then addressed like the column-block loader's, without sign.
// Split-K (gemm_pipe_split): the (split y, tile) pairs are numbered tile-fastest and dealt to
// the XCDs like tiles, so that the workgroups on one XCD share the k range of their split;
// split y takes [y kchunk, (y+1) kchunk) and writes its partial product to slice y of a
// workspace.
//
// LDS holds both tiles k-contiguous ([row][k]) with a 144-byte pitch (128 bytes of k and 16 of
// padding): the per-k-step fragment reads (lanes 0-15 on 16 rows) and the 8-byte stores
// spread over distinct banks, and this pitch measured 1% (FP64) to 2% (FP32) faster than a
// 136-byte one; 152 bytes gave nothing more.
//
// B operand. Each thread owns one column n = (j, c) of the tile and RB = BK/2 consecutive rows
// k = (m, e) of every slab; the rows are the same for all lanes of a wavefront, so the (m, e)
// position is scalar. Two loaders:
//  - column-block (nc a multiple of 128): a tile's columns share one j, so liveness, sign and
//    the X2 row address of every row are scalar; a structurally zero row (m = j, or k past
//    the end) is read from a row of zeros, and the sign costs one XOR per row. The slabs that
//    lie wholly inside the tile's zero segment m = j (v rows) are skipped: the slab sequence
//    jumps over them, in the A offsets and in the B row bookkeeping alike;
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
  const T* W;        // A: [M][lda] (or [K][lda] when transposed); the ovvo Weff is followed by
                     // zero padding
  const T* X2;       // ovvo: packed 2h1p block [(pair, e)][ldx]; dense: B [K][ldb]
  const T* zrow;     // zeros: >= nc (column-block loader) or >= N (dense loader)
  T* Z;              // C [M][ldc]
  int o, v, nc;      // ovvo: N = o * nc
  int M, N, K;
  int ldx;           // ovvo: row stride of X2
  int64_t lda, ldb, ldc;
  T alpha, beta;     // C = alpha A B + beta C (beta == 0 never reads C)
  int mtiles, ntiles, nslabs;
  int kchunk;        // dense split-K: k per split (a multiple of the slab), 0 without split
  int nsplit;        // dense split-K: number of splits (1 without split)
  int64_t sC;        // dense split-K: stride between the partial products
  const T* Zas;      // dense: antisymmetrised ovvo term added in the epilogue (null: none)
  int as_o, as_v, as_nc;
};

__device__ __forceinline__ int pair_index(int i, int j, int o) {  // i < j
  return i * o - (i * (i + 1) >> 1) + (j - i - 1);
}

// (i, j), i < j, of pair index q (the inverse of pair_index): the root of the quadratic in
// double, then an exact integer correction
__device__ __forceinline__ void pair_of(int q, int o, int& i, int& j) {
  const double b = 2.0 * o - 1.0;
  int ii = (int)floor((b - sqrt(b * b - 8.0 * q)) * 0.5);
  ii = max(0, min(ii, o - 2));
  while (ii > 0 && pair_index(ii, ii + 1, o) > q) --ii;
  while (ii + 1 <= o - 2 && pair_index(ii + 1, ii + 2, o) <= q) ++ii;
  i = ii;
  j = q - pair_index(ii, ii + 1, o) + ii + 1;
}

template <int N> struct IC { static constexpr int value = N; };

// B operand loaders
enum { B_GATHER = 0, B_COLBLOCK = 1, B_DENSE = 2 };

// TA: A is stored transposed ([K][lda]). MODE: B_GATHER (ovvo, general), B_COLBLOCK (ovvo,
// nc % 128 == 0, W padded, 16-byte aligned rows) or B_DENSE (plain row-major B). VEC: 16-byte
// A loads.
template <typename T, bool TA, int MODE, bool VEC>
__global__ __launch_bounds__(NT, 2) void ovvo_kernel(OvvoArgs<T> p) {
  constexpr bool BLOCKJ = MODE == B_COLBLOCK;
  constexpr bool DENSE = MODE == B_DENSE;
  constexpr bool SCALARB = MODE != B_GATHER;   // scalar B row addresses
  using M4 = MF<T>;
  using C4 = typename M4::C4;
  constexpr int BK = 128 / (int)sizeof(T);      // k per slab
  constexpr int VPC = 16 / (int)sizeof(T);      // elements per 16-byte chunk
  constexpr int VP8 = 8 / (int)sizeof(T);       // elements per 8-byte LDS store
  constexpr int LDK = BK + 2 * VP8;             // LDS row pitch: 144 bytes
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
  const int nwork = DENSE ? ntot * p.nsplit : ntot;
  const int T8 = (nwork + 7) / 8;
  const int Lw = (int)(blockIdx.x & 7) * T8 + (int)(blockIdx.x >> 3);
  if (Lw >= nwork) return;
  const int ysplit = DENSE ? Lw / ntot : 0;
  const int L = Lw - ysplit * ntot;
  const int grp = L / (GM * p.ntiles);
  const int rows = min(GM, p.mtiles - grp * GM);
  const int idx = L - grp * GM * p.ntiles;
  const int mt = grp * GM + idx % rows, nt = idx / rows;
  const int m0 = mt * BM, n0 = nt * BN;
  const T* __restrict__ W = p.W;
  const T* __restrict__ X2 = p.X2;
  const int K = p.K, M = p.M, v = p.v, o = p.o, ldx = p.ldx;
  const int64_t lda = p.lda;
  // dense split-K: this workgroup's k range starts at kbeg and spans nsl slabs
  const int kbeg = ysplit * p.kchunk;
  const int nsl = (DENSE && p.kchunk > 0) ? (min(K - kbeg, p.kchunk) + BK - 1) / BK : p.nslabs;

  // ---- B ownership: column bn, rows kh * RB + r of every slab (kh is wave-uniform)
  const int bn = tid % BN;
  const int kh = __builtin_amdgcn_readfirstlane(tid / BN);
  const int first = kh * RB;
  const int n = n0 + bn;
  const bool ncol = BLOCKJ || n < p.N;
  const int jt = DENSE ? 0 : n0 / p.nc;                      // column-block: the tile's j
  const int j = (BLOCKJ || DENSE) ? jt : (ncol ? n / p.nc : 0);
  // column read by this lane: of X2 (ovvo) or of B and the zero row (dense)
  const int c = DENSE ? (ncol ? n : 0) : (ncol ? n - j * p.nc : 0);

  // ---- column-block: slabs [slo, slo + nd) lie inside the zero segment m = j and are skipped;
  // the slab processed i-th is i, or i + nd from slo on
  int slo = 1 << 30, nd = 0, ms_to = 0, es_to = 0;
  if (BLOCKJ) {
    const int lo = (j * v + BK - 1) / BK, hi = ((j + 1) * v) / BK;
    if (hi > lo) {
      slo = lo;
      nd = hi - lo;
      ms_to = hi * BK / v;
      es_to = hi * BK - ms_to * v;
    }
  }
  auto slab_k = [&](int i) { return kbeg + (i + (i >= slo ? nd : 0)) * BK; };

  // ---- A ownership. Column-block loader: per-lane base pointers advanced by the slab offset;
  // reads past k = K land in the next row or in the zero padding after W, against B rows
  // that are zero.
  const T* wa[ACH];
  if (BLOCKJ) {
#pragma unroll
    for (int r = 0; r < ACH; ++r) {
      if (!TA) {
        const int row = min(m0 + tid / CPR + (NT / CPR) * r, M - 1);
        wa[r] = W + (int64_t)row * lda + (tid % CPR) * VPC;
      } else {
        const int f = tid + NT * r;
        const int mm = min(m0 + (f % (BM / VPC)) * VPC, M - VPC);
        wa[r] = W + (int64_t)(f / (BM / VPC)) * lda + mm;
      }
    }
  }

  // ---- B row bookkeeping. prep() prepares the rows of the next slab to be loaded (position
  // k0 = ms * v + es for the ovvo operand, kp for a dense B, scalar); its sign / liveness
  // state moves to the "in registers" copy once that slab's loads are issued, and is used when
  // the registers are stored to LDS.
  int ms = 0, es = 0, kp = kbeg;
  int sp = 0;                                             // column-block: slabs prepared
  if (BLOCKJ && slo == 0) {
    ms = ms_to;
    es = es_to;
  }
  typedef const T __attribute__((address_space(1)))* gptr;
  uint64_t prow[RB];                                      // column-block: row addresses
  unsigned pneg = 0, sneg = 0;                            // column-block: row r negated
  int pz0 = 0, pz1 = 0;                                   // general: row bases, m and m+1
  unsigned pcar = 0, scar = 0;                            // general: row r uses base m+1
  bool pl0 = false, pl1 = false, pg0 = false, pg1 = false;  // general: live / negated
  bool sl0 = false, sl1 = false, sg0 = false, sg1 = false;
  // element offset of X2[pair(m, j)][0][c], or 0 when the row is structurally zero (general)
  auto rowbase = [&](int m, bool& live, bool& neg) -> int {
    live = ncol && m < o && m != j;
    neg = m > j;
    const int lo = m < j ? m : j, hi = m < j ? j : m;
    return live ? pair_index(lo, hi, o) * v * ldx + c : 0;
  };
  // column-block: scalar bases of the first owned row in segments m and m+1 (the X2 row
  // (pair(m, j), e) with stride ldx, or the zero row with stride 0); selects are written as
  // masks so that the compiler keeps them in straight-line scalar code
  uint64_t q0 = 0, q1 = 0, d0 = 0, d1 = 0;
  int rc = 0, pb0 = 0, pb1 = 0;
  auto cbase = [&](int m, int e, uint64_t& ptr, uint64_t& stride) {
    const int lo = min(m, j), hi = max(m, j);
    const int pr = lo * o - ((lo * (lo + 1)) >> 1) + hi - lo - 1;
    const uint64_t live = 0ull - (uint64_t)((m < o) & (m != j));
    const uint64_t a = reinterpret_cast<uint64_t>(X2) +
                       (uint64_t)(((int64_t)pr * v + e) * ldx) * sizeof(T);
    ptr = (a & live) | (reinterpret_cast<uint64_t>(p.zrow) & ~live);
    stride = (uint64_t)ldx * sizeof(T) & live;
  };
  // in three parts (segment m, segment m+1, carry / sign / advance) so that they can be spread
  // between MFMAs
  auto prep_base = [&](int part) {
    if (DENSE) {
      // rows kp + first + r of B while below K, the zero row beyond
      if (part == 0) {
        q0 = reinterpret_cast<uint64_t>(X2) + (uint64_t)((int64_t)(kp + first) * p.ldb) * sizeof(T);
        d0 = (uint64_t)p.ldb * sizeof(T);
      } else if (part == 1) {
        q1 = reinterpret_cast<uint64_t>(p.zrow);
        d1 = 0;
      } else {
        rc = K - kp - first;
        pneg = 0;
        kp += BK;
      }
      return;
    }
    if (part == 0) {
      if (BLOCKJ) cbase(ms, es + first, q0, d0);
      else pb0 = rowbase(ms, pl0, pg0) + es * ldx;
    } else if (part == 1) {
      if (BLOCKJ) cbase(ms + 1, es + first - v, q1, d1);
      else pb1 = rowbase(ms + 1, pl1, pg1) + (es - v) * ldx;
    } else {
      if (BLOCKJ) {
        rc = v - es - first;   // owned rows r >= rc lie in segment m+1
        constexpr unsigned full = (RB >= 32) ? ~0u : ((1u << RB) - 1u);
        const unsigned hi = rc <= 0 ? full : (rc >= RB ? 0u : full & ~((1u << rc) - 1u));
        pneg = (ms > j ? full & ~hi : 0u) | (ms + 1 > j ? hi : 0u);
      } else {
        pz0 = pl0 ? pb0 : 0;
        pz1 = pl1 ? pb1 : 0;
        pcar = 0;
#pragma unroll
        for (int r = 0; r < RB; ++r) pcar |= (es + first + r >= v) ? 1u << r : 0u;
      }
      const int cy = es + BK >= v;
      es = es + BK - (cy ? v : 0);
      ms += cy;
      if (BLOCKJ) {
        ++sp;
        const bool jump = sp == slo;
        ms = jump ? ms_to : ms;
        es = jump ? es_to : es;
      }
    }
  };
  auto prep_row = [&](int r) {
    if (SCALARB) {
      const uint64_t mk = 0ull - (uint64_t)(r >= rc);
      prow[r] = ((q1 + r * d1) & mk) | ((q0 + r * d0) & ~mk);
    }
  };
  auto prep_all = [&]() {
    prep_base(0);
    prep_base(1);
    prep_base(2);
#pragma unroll
    for (int r = 0; r < RB; ++r) prep_row(r);
  };
  // the prepared state becomes the state of the slab held in registers
  auto commit = [&]() {
    sneg = pneg;
    scar = pcar;
    sl0 = pl0; sl1 = pl1; sg0 = pg0; sg1 = pg1;
  };

  T ra[ACH][VPC];
  T rb[RB];
  // ---- loads of one slab: ACH A chunks (ops 0 .. ACH-1), then B rows
  auto load_a = [&](int r, int k0) {
    if (BLOCKJ) {
      const V16 x = *reinterpret_cast<const V16*>(wa[r] + (TA ? (int64_t)k0 * lda : k0));
#pragma unroll
      for (int u = 0; u < VPC; ++u) ra[r][u] = x[u];
    } else if (!TA) {
      if (VEC) {
        // past K the chunk is clamped to the last aligned one (read against zero B rows)
        const int row = m0 + tid / CPR + (NT / CPR) * r, k = k0 + (tid % CPR) * VPC;
        const int kmax = K >= VPC ? ((K - VPC) & ~(VPC - 1)) : 0;
        const int rr = row < M ? row : M - 1, kk = k < K ? k : kmax;
        const V16 x = *reinterpret_cast<const V16*>(W + (int64_t)rr * lda + kk);
#pragma unroll
        for (int u = 0; u < VPC; ++u) ra[r][u] = x[u];
      } else {
#pragma unroll
        for (int u = 0; u < VPC; ++u) {
          const int f = tid + NT * (r * VPC + u);
          const int row = m0 + f / BK, k = k0 + f % BK;
          const int rr = row < M ? row : M - 1, kk = k < K ? k : K - 1;
          ra[r][u] = W[(int64_t)rr * lda + kk];
        }
      }
    } else {
      // W stored [K][M]: chunks run along m
      const int f = tid + NT * r;
      const int k = k0 + f / (BM / VPC), mm = m0 + (f % (BM / VPC)) * VPC;
      const int kk = k < K ? k : K - 1;
      if (VEC) {
        const int mmax = M >= VPC ? ((M - VPC) & ~(VPC - 1)) : 0;
        const int rr = mm < M ? mm : mmax;
        const V16 x = *reinterpret_cast<const V16*>(W + (int64_t)kk * lda + rr);
#pragma unroll
        for (int u = 0; u < VPC; ++u) ra[r][u] = x[u];
      } else {
#pragma unroll
        for (int u = 0; u < VPC; ++u) {
          const int rr = mm + u < M ? mm + u : M - 1;
          ra[r][u] = W[(int64_t)kk * lda + rr];
        }
      }
    }
  };
  auto load_b = [&](int r) {
    if (SCALARB) {
      rb[r] = reinterpret_cast<gptr>(prow[r])[c];
    } else {
      const bool carry = (pcar >> r) & 1u;
      rb[r] = X2[(carry ? pz1 : pz0) + (first + r) * ldx];
    }
  };
  // ---- LDS stores of the slab in registers: ops 0 .. ACH-1 are A chunks, ops ACH .. ACH+3
  // each hold RB/4 B rows
  constexpr int BG = RB / 4;
  auto store_op = [&](auto BUFC, int t) {
    constexpr int b = decltype(BUFC)::value;
    if (t < ACH) {
      const int r = t;
      if (!TA && (BLOCKJ || VEC)) {
        T* d = &As[b][tid / CPR + (NT / CPR) * r][(tid % CPR) * VPC];
#pragma unroll
        for (int h = 0; h < VPC; h += VP8) {
          V8 y;
#pragma unroll
          for (int u = 0; u < VP8; ++u) y[u] = ra[r][h + u];
          *reinterpret_cast<V8*>(d + h) = y;
        }
      } else if (!TA) {
#pragma unroll
        for (int u = 0; u < VPC; ++u) {
          const int f = tid + NT * (r * VPC + u);
          As[b][f / BK][f % BK] = ra[r][u];
        }
      } else {
        const int f = tid + NT * r;
        const int k = f / (BM / VPC), mm = (f % (BM / VPC)) * VPC;
#pragma unroll
        for (int u = 0; u < VPC; ++u) As[b][mm + u][k] = ra[r][u];
      }
    } else {
      const int g = t - ACH;
#pragma unroll
      for (int h = 0; h < BG; h += VP8) {
        V8 y;
#pragma unroll
        for (int u = 0; u < VP8; ++u) {
          const int r = g * BG + h + u;
          if (DENSE) {
            y[u] = rb[r];
          } else if (BLOCKJ) {
            y[u] = M4::flip(rb[r], (sneg >> r) & 1u);
          } else {
            const bool cr = (scar >> r) & 1u;
            const T x = (cr ? sl1 : sl0) ? rb[r] : T(0);
            y[u] = (cr ? sg1 : sg0) ? -x : x;
          }
        }
        *reinterpret_cast<V8*>(&Bs[b][bn][first + g * BG + h]) = y;
      }
    }
  };
  // load op issued after store op t, into the registers that store freed
  auto load_op = [&](int t, int k0) {
    if (t < ACH) {
      load_a(t, k0);
    } else {
#pragma unroll
      for (int h = 0; h < BG; ++h) load_b((t - ACH) * BG + h);
    }
  };

  C4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[i][q] = C4{0, 0, 0, 0};

  const int row_l = lane & 15, kq = lane >> 4;
  T af[NS][4], bf[NS][4];   // fragments of the k-steps of a slab
  auto frag_read = [&](auto BUFC, int s, int h) {
    constexpr int b = decltype(BUFC)::value;
    if (h < 4) af[s][h] = As[b][wm * 64 + h * 16 + row_l][4 * s + kq];
    else bf[s][h - 4] = Bs[b][wn * 64 + (h - 4) * 16 + row_l][4 * s + kq];
  };
  auto mfma2 = [&](int s, int t) {   // MFMAs 2t and 2t+1 of k-step s
#pragma unroll
    for (int x = 2 * t; x < 2 * t + 2; ++x)
      acc[x >> 2][x & 3] = M4::op(af[s][x >> 2], bf[s][x & 3], acc[x >> 2][x & 3]);
  };
  auto fence = []() { __builtin_amdgcn_sched_barrier(0); };

  // One slab from LDS buffer b, its first two fragments already in registers. The step is
  // laid out as 8 slots per k-step, each two MFMAs plus a small group of other work, fenced so
  // that the compiler keeps the order:
  //  k-step 0:        the LDS stores of the slab held in registers (next slab, other buffer),
  //                   each followed by the loads of the slab after it into the freed registers;
  //  k-steps 1..NS-2: fragment reads one k-step ahead;
  //  barrier;
  //  k-step NS-1:     the next slab's first two fragments and the row bookkeeping of the
  //                   slab to be loaded in the next step.
  auto step = [&](auto BUFC, int kload) {
    constexpr int b = decltype(BUFC)::value;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      mfma2(0, t);
      store_op(IC<b ^ 1>{}, t);
      load_op(t, kload);
      fence();
    }
    commit();
#pragma unroll
    for (int s = 1; s + 1 < NS; ++s)
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        mfma2(s, t);
        if (t < 4) {
          frag_read(IC<b>{}, s + 1, 2 * t);
          frag_read(IC<b>{}, s + 1, 2 * t + 1);
        }
        fence();
      }
    fence();
    __syncthreads();
    fence();
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      mfma2(NS - 1, t);
      frag_read(IC<b ^ 1>{}, t >> 2, 2 * (t & 3));
      frag_read(IC<b ^ 1>{}, t >> 2, 2 * (t & 3) + 1);
      if (t < 3) prep_base(t);
      constexpr int RPS = (RB + 5) / 6;   // rows prepared per slot, slots 2..7
#pragma unroll
      for (int h = 0; h < RPS; ++h)
        if (t >= 2 && (t - 2) * RPS + h < RB) prep_row((t - 2) * RPS + h);
      fence();
    }
  };

  // prologue: slab 0 into LDS buffer 0 and its first fragments, slab 1 into registers, the
  // rows of slab 2 prepared
  prep_all();
  commit();
#pragma unroll
  for (int t = 0; t < ACH + 4; ++t) load_op(t, slab_k(0));
#pragma unroll
  for (int t = 0; t < ACH + 4; ++t) store_op(IC<0>{}, t);
  prep_all();
#pragma unroll
  for (int t = 0; t < ACH + 4; ++t) load_op(t, slab_k(1));
  commit();
  prep_all();
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 8; ++h) {
    frag_read(IC<0>{}, 0, h);
    frag_read(IC<0>{}, 1, h);
  }
  // Every step stores and loads ahead. Past the last slab the B rows are structurally zero
  // and the A reads stay in range (clamped, or in the padding after W), and the stores go to
  // the buffer that is no longer read.
  const int ns = nsl - nd;
  for (int s = 0; s < ns; s += 2) {
    step(IC<0>{}, slab_k(s + 2));
    if (s + 1 < ns) step(IC<1>{}, slab_k(s + 3));
  }

  const int col_l = lane & 15;
  if (DENSE && p.Zas) {
    // C = Y2 [pair][a nc + c]: row mrow = pair(pi, pj), column nn = a nc + c gets
    // Z[(pi,a)][(pj,c)] - Z[(pj,a)][(pi,c)]; the columns' (a, c) once per thread, the rows'
    // pairs once per row
    const int ao = p.as_o, av = p.as_v, anc = p.as_nc;
    const int64_t ldz = (int64_t)ao * anc;
    int ca[4], cc[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int nn = min(n0 + wn * 64 + q * 16 + col_l, p.N - 1);
      ca[q] = nn / anc;
      cc[q] = nn - ca[q] * anc;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int mrow = m0 + wm * 64 + i * 16 + M4::row(lane, e);
        if (mrow >= M) continue;
        int pi, pj;
        pair_of(mrow, ao, pi, pj);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int nn = n0 + wn * 64 + q * 16 + col_l;
          if (nn >= p.N) continue;
          T* cp = p.Z + (int64_t)ysplit * p.sC + (int64_t)mrow * p.ldc + nn;
          const T zt = p.Zas[((int64_t)pi * av + ca[q]) * ldz + (int64_t)pj * anc + cc[q]] -
                       p.Zas[((int64_t)pj * av + ca[q]) * ldz + (int64_t)pi * anc + cc[q]];
          *cp = p.alpha * acc[i][q][e] + (p.beta != T(0) ? p.beta * *cp : T(0)) + zt;
        }
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int nn = n0 + wn * 64 + q * 16 + col_l;
      if (!BLOCKJ && nn >= p.N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int mrow = m0 + wm * 64 + i * 16 + M4::row(lane, e);
        if (mrow >= M) continue;
        T* cp = p.Z + (int64_t)ysplit * p.sC + (int64_t)mrow * p.ldc + nn;
        if (DENSE) *cp = p.alpha * acc[i][q][e] + (p.beta != T(0) ? p.beta * *cp : T(0));
        else *cp = acc[i][q][e];
      }
    }
}

// The last t <= TAIL rows of Z (rows r0 .. r0 + t - 1) with vector FMAs. When M = o v leaves
// only a few rows for a last 128-row tile (o v = 7812 = 61 x 128 + 4 at the benzene shape),
// that tile row costs the matrix cores a full tile per column tile for a handful of useful
// rows: 1.6% of the contraction there. Here a thread owns one column (j, c) of Z and walks
// k = (m, e), m != j, reading r_mj^e[c] = +-X2[pair][e][c] once (coalesced over c) against the
// t rows of W staged in LDS one segment m at a time, EC values of e per stage. Narrow blocks
// split the segments m over blockIdx.z (mchunk each) so that the grid still fills the chip:
// each split then writes its partial sums to part[z][rr][N] (N = o nc), which
// ovvo_tail_reduce_kernel adds in split order; part null: one split, written to Z.
constexpr int TAIL = 8, TAIL_MIN_NC = 256;
template <typename T>
__global__ __launch_bounds__(256) void ovvo_tail_kernel(const T* __restrict__ W, int64_t lda,
                                                        int transW, int r0, int t,
                                                        const T* __restrict__ X2, int64_t ldx,
                                                        int o, int v, int nc, T* __restrict__ Z,
                                                        int64_t ldc, int mchunk,
                                                        T* __restrict__ part) {
  constexpr int EC = 256, XB = 16;
  static_assert(EC % XB == 0, "a batch stays inside a stage");
  __shared__ __attribute__((aligned(16))) T a_s[EC][TAIL];  // the t rows of one e, contiguous
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  const bool live = c < nc;
  T acc[TAIL];
#pragma unroll
  for (int rr = 0; rr < TAIL; ++rr) acc[rr] = T(0);
  const int m_lo = blockIdx.z * mchunk, m_hi = min(o, m_lo + mchunk);
  for (int m = m_lo; m < m_hi; ++m) {
    if (m == j) continue;  // r_jj = 0
    const int lo = m < j ? m : j, hi = m < j ? j : m;
    const int64_t pr = (int64_t)lo * o - ((int64_t)lo * (lo + 1) >> 1) + (hi - lo - 1);
    const bool neg = m > j;
    for (int e0 = 0; e0 < v; e0 += EC) {
      const int ne = min(EC, v - e0);
      __syncthreads();  // the previous stage has been read
      for (int f = threadIdx.x; f < TAIL * EC; f += 256) {
        const int rr = f % TAIL, ee = f / TAIL;
        T a = T(0);
        if (rr < t && ee < ne) {
          const int64_t k = (int64_t)m * v + e0 + ee;
          a = transW ? W[k * lda + r0 + rr] : W[(int64_t)(r0 + rr) * lda + k];
        }
        a_s[ee][rr] = neg ? -a : a;
      }
      __syncthreads();
      if (!live) continue;
      // XB loads in flight per batch (the kernel is bound by their latency: one thread per
      // column keeps too few bytes in flight otherwise); a_s is zero past ne, and EC is a
      // multiple of XB, so a batch never reads past a_s
      const int lx = (int)ldx;  // v ldx < 2^30 (checked by the launcher)
      for (int eb = 0; eb < ne; eb += XB) {
        const T* x = X2 + (pr * v + e0 + eb) * ldx + c;
        T xv[XB];
#pragma unroll
        for (int u = 0; u < XB; ++u) xv[u] = eb + u < ne ? x[u * lx] : T(0);
#pragma unroll
        for (int u = 0; u < XB; ++u)
#pragma unroll
          for (int rr = 0; rr < TAIL; ++rr) acc[rr] += a_s[eb + u][rr] * xv[u];
      }
    }
  }
  if (!live) return;
  const int64_t N = (int64_t)o * nc;
  for (int rr = 0; rr < t; ++rr) {
    if (part)
      part[((int64_t)blockIdx.z * TAIL + rr) * N + (int64_t)j * nc + c] = acc[rr];
    else
      Z[(int64_t)(r0 + rr) * ldc + (int64_t)j * nc + c] = acc[rr];
  }
}

// Z rows r0 .. r0 + t - 1 = the sum of the ns splits' partial rows, in split order
template <typename T>
__global__ void ovvo_tail_reduce_kernel(const T* __restrict__ part, int ns, int t, int64_t N,
                                        int r0, T* __restrict__ Z, int64_t ldc) {
  const int64_t n = (int64_t)t * N;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int rr = (int)(idx / N);
    const int64_t col = idx - (int64_t)rr * N;
    T s = T(0);
    for (int z = 0; z < ns; ++z) s += part[((int64_t)z * TAIL + rr) * N + col];
    Z[(int64_t)(r0 + rr) * ldc + col] = s;
  }
}

}  // namespace

// Returns false when the shape is outside what the kernels support (the caller then uses the
// generic gather path). W must be followed by ovvo_pad_bytes(M) zero bytes; zrow holds at least
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
  p.lda = transW ? p.M : p.K;
  p.ldb = 0; p.ldc = p.N;
  p.alpha = T(1); p.beta = T(0);
  // a last tile row of at most TAIL rows goes to ovvo_tail_kernel (M stays a multiple of the
  // 16-byte A chunk: o v - t = 128 (o v / 128)) when the block has at least 256 columns
  // (below that the tile row it replaces costs next to nothing)
  const int tail = (p.M > BM && p.M % BM <= TAIL && nc >= TAIL_MIN_NC) ? p.M % BM : 0;
  p.M -= tail;
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
    if (blockj) hipLaunchKernelGGL((ovvo_kernel<T, true, B_COLBLOCK, true>), grid, dim3(NT), 0, st, p);
    else if (vec) hipLaunchKernelGGL((ovvo_kernel<T, true, B_GATHER, true>), grid, dim3(NT), 0, st, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, true, B_GATHER, false>), grid, dim3(NT), 0, st, p);
  } else {
    if (blockj) hipLaunchKernelGGL((ovvo_kernel<T, false, B_COLBLOCK, true>), grid, dim3(NT), 0, st, p);
    else if (vec) hipLaunchKernelGGL((ovvo_kernel<T, false, B_GATHER, true>), grid, dim3(NT), 0, st, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, false, B_GATHER, false>), grid, dim3(NT), 0, st, p);
  }
  GFCC_LAUNCH_CHECK();
  if (tail) {
    // splits of the segments m so that the tail grid has about 512 workgroups: one at the
    // benchmark's 3200 columns (13 x 42 workgroups), five at 640
    const int bx = (nc + 255) / 256;
    int mchunk = o;
    if (bx * o < 512) {
      const int want = std::min(o, (512 + bx * o - 1) / (bx * o));
      mchunk = (o + want - 1) / want;
    }
    const int ns = (o + mchunk - 1) / mchunk;
    T* part = nullptr;
    if (ns > 1) {
      ws_ensure(ctx, ctx->ws_tail, sizeof(T) * (size_t)ns * TAIL * (size_t)p.N);
      part = ctx->ws_tail.as<T>();
    }
    hipLaunchKernelGGL(ovvo_tail_kernel<T>, dim3((unsigned)bx, (unsigned)o, (unsigned)ns),
                       dim3(256), 0, st, W, p.lda, transW ? 1 : 0, p.M, tail, X2, ldx, o, v, nc,
                       Z, p.ldc, mchunk, part);
    GFCC_LAUNCH_CHECK();
    if (part) {
      hipLaunchKernelGGL(ovvo_tail_reduce_kernel<T>,
                         dim3((unsigned)std::min<int64_t>(4096, ((int64_t)tail * p.N + 255) / 256)),
                         dim3(256), 0, st, part, ns, tail, (int64_t)p.N, p.M, Z, p.ldc);
      GFCC_LAUNCH_CHECK();
    }
  }
  return true;
}

// C[M][N] = alpha op(A) B + beta C with B row-major [K][ldb], on the same pipelined kernel.
// op(A) = A ([M][lda]) or A^T (A stored [K][lda]). Returns false when the product is too small
// or too thin to fill the GPU with 128 x 128 tiles (the caller then uses the split-K kernel).
template <typename T>
bool gemm_pipe(gfcc_ctx* ctx, bool transA, int M, int N, int K, T alpha, const T* A, int64_t lda,
               const T* B, int64_t ldb, T beta, T* C, int64_t ldc, bool a_padded, const T* Zas,
               int as_o, int as_v, int as_nc) {
  constexpr int BK = 128 / (int)sizeof(T);
  constexpr int VPC = 16 / (int)sizeof(T);
  // thin products (vectors, a few rows or columns) would waste most of a 128 x 128 tile
  if (M < 64 || N < 64 || K < 1) return false;
  OvvoArgs<T> p{};
  p.M = M; p.N = N; p.K = K;
  p.mtiles = (M + BM - 1) / BM;
  p.ntiles = (N + BN - 1) / BN;
  p.nslabs = (K + BK - 1) / BK;
  const int64_t tiles = (int64_t)p.mtiles * p.ntiles;
  if (tiles < 256 || tiles >= (1LL << 31) - 8) return false;
  p.W = A; p.lda = lda;
  p.X2 = B; p.ldb = ldb;
  p.Z = C; p.ldc = ldc;
  p.alpha = alpha; p.beta = beta;
  p.nsplit = 1;
  p.nc = 1; p.o = 1; p.v = 1; p.ldx = 0;
  if (Zas) {
    GFCC_REQUIRE(as_o >= 2 && as_v >= 1 && as_nc >= 1 && M == as_o * (as_o - 1) / 2 &&
                     (int64_t)N == (int64_t)as_v * as_nc && ldc == N,
                 GFCC_EINVAL, "gemm_pipe: the antisymmetric term needs C = [pairs][v nc]");
    p.Zas = Zas; p.as_o = as_o; p.as_v = as_v; p.as_nc = as_nc;
  }
  p.zrow = static_cast<const T*>(zero_row(ctx, (size_t)N * sizeof(T)));
  // 16-byte A chunks need aligned rows and a chunked dimension that is a multiple of the chunk
  // (the clamp of the last chunk then stays inside the row), or rows padded with finite
  // entries to that multiple (the tail chunk then reads padding against zero B rows, or
  // fills tile rows that are never stored)
  const int64_t cdim = transA ? M : K;
  const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % VPC == 0) &&
                   (cdim % VPC == 0 || (a_padded && lda >= (cdim + VPC - 1) / VPC * VPC));
  dim3 grid((unsigned)((tiles + 7) / 8 * 8));
  hipStream_t st = ctx->stream;
  if (transA) {
    if (vec) hipLaunchKernelGGL((ovvo_kernel<T, true, B_DENSE, true>), grid, dim3(NT), 0, st, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, true, B_DENSE, false>), grid, dim3(NT), 0, st, p);
  } else {
    if (vec) hipLaunchKernelGGL((ovvo_kernel<T, false, B_DENSE, true>), grid, dim3(NT), 0, st, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, false, B_DENSE, false>), grid, dim3(NT), 0, st, p);
  }
  GFCC_LAUNCH_CHECK();
  return true;
}

// Split-K partial products on the pipelined kernel: part[y][M][N] = op(A) B over the k range
// [y kchunk, (y+1) kchunk), y < splits (kchunk a multiple of the slab). The caller reduces.
template <typename T>
void gemm_pipe_split(gfcc_ctx* ctx, bool transA, int M, int N, int K, const T* A, int64_t lda,
                     const T* B, int64_t ldb, T* part, int splits, int kchunk) {
  constexpr int BK = 128 / (int)sizeof(T);
  constexpr int VPC = 16 / (int)sizeof(T);
  GFCC_REQUIRE(M >= 1 && N >= 1 && K >= 1 && splits >= 1 && kchunk % BK == 0 &&
                   (int64_t)splits * kchunk >= K && (int64_t)(splits - 1) * kchunk < K,
               GFCC_EINVAL, "gemm_pipe_split: bad split");
  OvvoArgs<T> p{};
  p.M = M; p.N = N; p.K = K;
  p.mtiles = (M + BM - 1) / BM;
  p.ntiles = (N + BN - 1) / BN;
  p.nslabs = (K + BK - 1) / BK;
  p.kchunk = kchunk;
  p.nsplit = splits;
  p.sC = (int64_t)M * N;
  const int64_t tiles = (int64_t)p.mtiles * p.ntiles;
  GFCC_REQUIRE(tiles * splits < (1LL << 31) - 8, GFCC_EINVAL, "gemm_pipe_split: too many tiles");
  p.W = A; p.lda = lda;
  p.X2 = B; p.ldb = ldb;
  p.Z = part; p.ldc = N;
  p.alpha = T(1); p.beta = T(0);
  p.nc = 1; p.o = 1; p.v = 1; p.ldx = 0;
  p.zrow = static_cast<const T*>(zero_row(ctx, (size_t)N * sizeof(T)));
  const bool vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % VPC == 0) &&
                   ((transA ? M : K) % VPC == 0);
  dim3 grid((unsigned)((tiles * splits + 7) / 8 * 8));
  hipStream_t st = ctx->stream;
  if (transA) {
    if (vec) hipLaunchKernelGGL((ovvo_kernel<T, true, B_DENSE, true>), grid, dim3(NT), 0, st, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, true, B_DENSE, false>), grid, dim3(NT), 0, st, p);
  } else {
    if (vec) hipLaunchKernelGGL((ovvo_kernel<T, false, B_DENSE, true>), grid, dim3(NT), 0, st, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, false, B_DENSE, false>), grid, dim3(NT), 0, st, p);
  }
  GFCC_LAUNCH_CHECK();
}

template void gemm_pipe_split<double>(gfcc_ctx*, bool, int, int, int, const double*, int64_t,
                                      const double*, int64_t, double*, int, int);
template void gemm_pipe_split<float>(gfcc_ctx*, bool, int, int, int, const float*, int64_t,
                                     const float*, int64_t, float*, int, int);
template bool ovvo_fast<double>(gfcc_ctx*, bool, int, int, int, const double*, const double*,
                                int64_t, double*, const double*);
template bool ovvo_fast<float>(gfcc_ctx*, bool, int, int, int, const float*, const float*,
                               int64_t, float*, const float*);
template bool gemm_pipe<double>(gfcc_ctx*, bool, int, int, int, double, const double*, int64_t,
                                const double*, int64_t, double, double*, int64_t, bool,
                                const double*, int, int, int);
template bool gemm_pipe<float>(gfcc_ctx*, bool, int, int, int, float, const float*, int64_t,
                               const float*, int64_t, float, float*, int64_t, bool, const float*,
                               int, int, int);

}  // namespace gfcc
