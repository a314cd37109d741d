// The ovvo contraction of the IP sigma product on FP64/FP32 matrix cores:
//   Z[(i,a)][(j,c)] = sum_(m,e) W[(i,a)][(m,e)] r_mj^e[c],     r_mj^e = +-X2[pair(m,j)][e][c]
// (91% of the sigma flops at the benzene/cc-pVDZ shape). r is the antisymmetric expansion of
// the packed two-hole-one-particle block; it is generated while the B tile is loaded, so the
// expanded operand (twice the size of X2) never exists in memory.
//
// Tile 128 x 128 x 16, 256 threads (2 x 2 wavefronts of 64 x 64 = 4 x 4 MFMA 16x16 blocks).
// LDS is double-buffered: the next K slab is fetched into registers while the current one
// feeds the MFMAs, then stored to the other buffer, so each slab costs one barrier.
// A is read with 16-byte loads. For B, each thread owns one column (j, c) and eight rows;
// the row index k = (m, e) of every owned row is advanced incrementally (e += 16, carry into
// m), and the pair index is computed arithmetically, so the gather has no divisions and no
// dependent table loads.
#include "common.h"

namespace gfcc {
namespace {

constexpr int BM = 128, BN = 128, BK = 16, NT = 256;

template <typename T> struct MF;
template <> struct MF<double> {
  typedef double C4 __attribute__((ext_vector_type(4)));
  typedef double V2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ C4 op(double a, double b, C4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
  static constexpr int PAD = 2;
};
template <> struct MF<float> {
  typedef float C4 __attribute__((ext_vector_type(4)));
  typedef float V2 __attribute__((ext_vector_type(2)));
  static __device__ __forceinline__ C4 op(float a, float b, C4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
  static constexpr int PAD = 4;
};

template <typename T> struct OvvoArgs {
  const T* W;        // [M][K] (or [K][M] when transposed)
  const T* X2;       // packed 2h1p block [(pair, e)][ldx]
  T* Z;              // [M][N]
  int o, v, nc;      // N = o * nc
  int M, N, K;
  int64_t ldx;
  int mtiles, ntiles;
};

__device__ __forceinline__ int pair_index(int i, int j, int o) {  // i < j
  return i * o - (i * (i + 1) >> 1) + (j - i - 1);
}

template <typename T, bool TA, bool VEC>
__global__ __launch_bounds__(NT, 2) void ovvo_kernel(OvvoArgs<T> p) {
  using M4 = MF<T>;
  using C4 = typename M4::C4;
  using V2 = typename M4::V2;
  constexpr int PAD = M4::PAD;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // tile order: N-tiles of one M-tile row are consecutive, so wavefronts resident at the
  // same time share the A (operator) rows
  const int mt = blockIdx.x / p.ntiles, nt = blockIdx.x % p.ntiles;
  const int m0 = mt * BM, n0 = nt * BN;
  const T* __restrict__ W = p.W;
  const T* __restrict__ X2 = p.X2;
  const int K = p.K, M = p.M, v = p.v, o = p.o;

  // ---- B ownership: column n (fixed), rows kr + 2r of every slab
  const int bn = tid % BN, kr = tid / BN;
  const int n = n0 + bn;
  const bool ncol = n < p.N;
  const int j = ncol ? n / p.nc : 0;
  const int c = ncol ? n - j * p.nc : 0;
  // Per owned row: me = (m << 16) | e and the element offset of its X2 entry for this thread's
  // column. Bit r of blive / bneg: row r is non-zero / enters with a minus sign.
  int me[8], off[8];
  unsigned blive = 0, bneg = 0;
  auto locate = [&](int m, int e, int r) {
    const int lo = m < j ? m : j, hi = m < j ? j : m;
    const bool live = ncol && m < o && m != j;
    off[r] = live ? (pair_index(lo, hi, o) * v + e) * (int)p.ldx + c : 0;
    blive = (blive & ~(1u << r)) | (live ? 1u << r : 0u);
    bneg = (bneg & ~(1u << r)) | (m > j ? 1u << r : 0u);
  };
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int k = kr + 2 * r, m = k / v, e = k - m * v;
    me[r] = (m << 16) | e;
    locate(m, e, r);
  }
  const int step = BK * (int)p.ldx;

  // Loads are unconditional (addresses clamped into range) and their values are not touched
  // until they are written to LDS after the MFMAs of the current slab, so the memory latency
  // overlaps the matrix work. Out-of-range elements are zeroed at that point.
  T ra[8], rb[8];
  unsigned amask = 0, slive = 0, sneg = 0;
  auto load = [&](int k0) {
    amask = 0;
    if (!TA) {
      if (VEC) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + (tid >> 3) + 32 * r, k = k0 + 2 * (tid & 7);
          amask |= (row < M && k < K) ? (3u << (2 * r)) : 0u;
          const int rr = row < M ? row : M - 1, kk = k < K ? k : K - 2;
          const V2 x = *reinterpret_cast<const V2*>(W + (int64_t)rr * K + kk);
          ra[2 * r] = x[0];
          ra[2 * r + 1] = x[1];
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int k = k0 + (tid & 15), row = m0 + (tid >> 4) + 16 * r;
          amask |= (row < M && k < K) ? (1u << r) : 0u;
          const int rr = row < M ? row : M - 1, kk = k < K ? k : K - 1;
          ra[r] = W[(int64_t)rr * K + kk];
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = k0 + (tid >> 6) + 4 * r, row = m0 + 2 * (tid & 63);
        amask |= (k < K && row < M) ? (1u << (2 * r)) : 0u;
        amask |= (k < K && row + 1 < M) ? (2u << (2 * r)) : 0u;
        const int kk = k < K ? k : K - 1;
        if (VEC) {
          const int rr = row < M ? row : M - 2;
          const V2 x = *reinterpret_cast<const V2*>(W + (int64_t)kk * M + rr);
          ra[2 * r] = x[0];
          ra[2 * r + 1] = x[1];
        } else {
          const int r0 = row < M ? row : M - 1, r1 = row + 1 < M ? row + 1 : M - 1;
          ra[2 * r] = W[(int64_t)kk * M + r0];
          ra[2 * r + 1] = W[(int64_t)kk * M + r1];
        }
      }
    }
    // B: gathered antisymmetric expansion
    unsigned kmask = 0xffu;
    if (k0 + kr + 14 >= K) {
      kmask = 0u;
#pragma unroll
      for (int r = 0; r < 8; ++r) kmask |= (k0 + kr + 2 * r < K) ? (1u << r) : 0u;
    }
    slive = blive & kmask;
    sneg = bneg;
#pragma unroll
    for (int r = 0; r < 8; ++r) rb[r] = X2[off[r]];
  };
  // advance every owned row to the same row of the next slab (v >= BK: at most one carry
  // into m); done after the matrix work so it never waits on loads in flight
  auto advance = [&]() {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = (me[r] & 0xffff) + BK;
      const int m = me[r] >> 16;
      if (e >= v) {
        me[r] = ((m + 1) << 16) | (e - v);
        locate(m + 1, e - v, r);
      } else {
        me[r] = (m << 16) | e;
        off[r] += ((blive >> r) & 1u) ? step : 0;
      }
    }
  };
  auto store = [&](int buf) {
    if (!TA) {
      if (VEC) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = (tid >> 3) + 32 * r, k = 2 * (tid & 7);
          const bool ok = (amask >> (2 * r)) & 1u;
          As[buf][k][row] = ok ? ra[2 * r] : T(0);
          As[buf][k + 1][row] = ok ? ra[2 * r + 1] : T(0);
        }
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r)
          As[buf][tid & 15][(tid >> 4) + 16 * r] = ((amask >> r) & 1u) ? ra[r] : T(0);
      }
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = (tid >> 6) + 4 * r, row = 2 * (tid & 63);
        As[buf][k][row] = ((amask >> (2 * r)) & 1u) ? ra[2 * r] : T(0);
        As[buf][k][row + 1] = ((amask >> (2 * r)) & 2u) ? ra[2 * r + 1] : T(0);
      }
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const T x = ((slive >> r) & 1u) ? rb[r] : T(0);
      Bs[buf][kr + 2 * r][bn] = ((sneg >> r) & 1u) ? -x : x;
    }
  };

  C4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[i][q] = C4{0, 0, 0, 0};

  const int row_l = lane & 15, kq = lane >> 4;
  load(0);
  advance();
  store(0);
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) load(k0 + BK);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      T af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[buf][s * 4 + kq][wm * 64 + i * 16 + row_l];
#pragma unroll
      for (int q = 0; q < 4; ++q) bf[q] = Bs[buf][s * 4 + kq][wn * 64 + q * 16 + row_l];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[i][q] = M4::op(af[i], bf[q], acc[i][q]);
    }
    if (more) {
      store(buf ^ 1);
      advance();
    }
    __syncthreads();
    buf ^= 1;
  }

  const int col_l = lane & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int nn = n0 + wn * 64 + q * 16 + col_l;
      if (nn >= p.N) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int mrow = m0 + wm * 64 + i * 16 + M4::row(lane, e);
        if (mrow < M) p.Z[(int64_t)mrow * p.N + nn] = acc[i][q][e];
      }
    }
}

}  // namespace

// Returns false when the shape is outside what the kernel supports (the caller then uses the
// generic gather path).
template <typename T>
bool ovvo_fast(gfcc_ctx* ctx, bool transW, int o, int v, int nc, const T* W, const T* X2,
               int64_t ldx, T* Z) {
  if (o < 2 || v < BK) return false;
  OvvoArgs<T> p{};
  p.W = W; p.X2 = X2; p.Z = Z;
  p.o = o; p.v = v; p.nc = nc;
  p.M = o * v; p.K = o * v; p.N = o * nc;
  p.ldx = ldx;
  p.mtiles = (p.M + BM - 1) / BM;
  p.ntiles = (p.N + BN - 1) / BN;
  const int64_t tiles = (int64_t)p.mtiles * p.ntiles;
  if (tiles >= (1LL << 31)) return false;
  // element offsets into X2 are kept in 32 bits
  const int64_t P = (int64_t)o * (o - 1) / 2;
  if (P * v * ldx + nc >= (1LL << 31) - 1 || (int64_t)BK * ldx >= (1LL << 30)) return false;
  const bool vec = (reinterpret_cast<uintptr_t>(W) % (2 * sizeof(T)) == 0) && (p.K % 2 == 0);
  dim3 grid((unsigned)tiles);
  if (transW) {
    if (vec) hipLaunchKernelGGL((ovvo_kernel<T, true, true>), grid, dim3(NT), 0, ctx->stream, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, true, false>), grid, dim3(NT), 0, ctx->stream, p);
  } else {
    if (vec) hipLaunchKernelGGL((ovvo_kernel<T, false, true>), grid, dim3(NT), 0, ctx->stream, p);
    else hipLaunchKernelGGL((ovvo_kernel<T, false, false>), grid, dim3(NT), 0, ctx->stream, p);
  }
  GFCC_LAUNCH_CHECK();
  return true;
}

template bool ovvo_fast<double>(gfcc_ctx*, bool, int, int, int, const double*, const double*,
                                int64_t, double*);
template bool ovvo_fast<float>(gfcc_ctx*, bool, int, int, int, const float*, const float*,
                               int64_t, float*);

}  // namespace gfcc
