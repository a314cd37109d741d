// Dense contractions on CDNA4 matrix cores (MFMA) for FP64 and FP32.
//
// One workgroup = 4 wavefronts (2 x 2) computes a 128 x 128 tile of C; each wavefront owns a
// 64 x 64 sub-tile held as 4 x 4 accumulators of the 16x16x4 MFMA (f64 or f32). K advances in
// slabs of 16: global -> registers (prefetched one slab ahead) -> LDS (k-major, padded) ->
// MFMA operands. Ragged edges are zero-filled on load and masked on store.
//
// The B operand has three modes: row-major [K][N], transposed ([N][K]), or the gather used by
// the ovvo term of the IP sigma product, which expands the packed antisymmetric 2h1p block
// on the fly (r_mj^e = +-X2[pair(m,j)][e], zero for m == j).
#include <algorithm>
#include <cstdlib>

#include "common.h"

namespace gfcc {
namespace {

constexpr int BM = 128, BN = 128, BK = 16, NT = 256;

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double C4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ C4 op(double a, double b, C4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static constexpr int PAD = 2;
  // output element q of lane l sits at row (l/16) + 4q, column l%16
  static __device__ __forceinline__ int row(int lane, int q) { return (lane >> 4) + 4 * q; }
};
template <> struct Mfma<float> {
  typedef float C4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ C4 op(float a, float b, C4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static constexpr int PAD = 4;
  // output element q of lane l sits at row 4(l/16) + q, column l%16
  static __device__ __forceinline__ int row(int lane, int q) { return 4 * (lane >> 4) + q; }
};

enum BMode { B_ROW = 0, B_TRANS = 1, B_OVVO = 2 };

template <typename T> struct Params {
  int M, N, K;
  const T* A; int64_t lda, sA;
  const T* B; int64_t ldb, sB;
  T* C; int64_t ldc, sC;
  T alpha, beta;
  int kchunk;          // split-K chunk (multiple of BK); splits = gridDim.z
  int mtiles, ntiles;
  // ovvo gather
  const int* lut; int o, v, nc;
};

template <typename T, bool TA, int BMODE, bool SPLIT>
__global__ __launch_bounds__(NT, 2) void gemm_kernel(Params<T> p) {
  using M4 = Mfma<T>;
  using C4 = typename M4::C4;
  constexpr int PAD = M4::PAD;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  const int tile = blockIdx.x;
  const int mt = tile % p.mtiles, nt = tile / p.mtiles;
  const int m0 = mt * BM, n0 = nt * BN;
  const int64_t bidx = blockIdx.y;
  const T* __restrict__ A = p.A + bidx * p.sA;
  const T* __restrict__ B = p.B + bidx * p.sB;

  int kbeg = 0, kend = p.K;
  if (SPLIT) {
    kbeg = blockIdx.z * p.kchunk;
    kend = min(p.K, kbeg + p.kchunk);
  }

  // ---- per-thread load coordinates
  // A row-major [M][K]: k = tid%16, rows tid/16 + 16r ; A^T [K][M]: m = tid%128, k = tid/128 + 2r
  // B row-major / gather: n = tid%128, k = tid/128 + 2r ; B^T [N][K]: k = tid%16, n = tid/16+16r
  const int a_c0 = TA ? (tid % BM) : (tid % BK);
  const int a_r0 = TA ? (tid / BM) : (tid / BK);
  const int b_c0 = (BMODE == B_TRANS) ? (tid % BK) : (tid % BN);
  const int b_r0 = (BMODE == B_TRANS) ? (tid / BK) : (tid / BN);

  // gather mode: fixed column -> (j, c)
  int g_j = 0, g_c = 0;
  bool g_nok = false;
  if (BMODE == B_OVVO) {
    int n = n0 + b_c0;
    g_nok = n < p.N;
    if (g_nok) {
      g_j = n / p.nc;
      g_c = n - g_j * p.nc;
    }
  }

  // Loads are unconditional (indices clamped into range); their values are only consumed when
  // the slab is written to LDS after the MFMAs of the current slab, where out-of-range entries
  // are zeroed (bits of amask/bmask) and gathered entries get their sign.
  T ra[8], rb[8];
  unsigned amask = 0, bmask = 0, bneg = 0;
  const int Mc = p.M - 1, Nc = p.N - 1;
  auto load_tile = [&](int k0) {
    amask = bmask = bneg = 0;
    const int kc = kend - 1;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      int m, k;
      if (TA) { m = m0 + a_c0; k = k0 + a_r0 + 2 * r; }
      else    { k = k0 + a_c0; m = m0 + a_r0 + 16 * r; }
      amask |= (m < p.M && k < kend) ? (1u << r) : 0u;
      const int mm = m < Mc ? m : Mc, kk = k < kc ? k : kc;
      ra[r] = TA ? A[(int64_t)kk * p.lda + mm] : A[(int64_t)mm * p.lda + kk];
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (BMODE == B_TRANS) {
        const int k = k0 + b_c0, n = n0 + b_r0 + 16 * r;
        bmask |= (n < p.N && k < kend) ? (1u << r) : 0u;
        const int nn = n < Nc ? n : Nc, kk = k < kc ? k : kc;
        rb[r] = B[(int64_t)nn * p.ldb + kk];
      } else if (BMODE == B_ROW) {
        const int k = k0 + b_r0 + 2 * r, n = n0 + b_c0;
        bmask |= (n < p.N && k < kend) ? (1u << r) : 0u;
        const int nn = n < Nc ? n : Nc, kk = k < kc ? k : kc;
        rb[r] = B[(int64_t)kk * p.ldb + nn];
      } else {
        const int k = k0 + b_r0 + 2 * r;
        const int kk = k < kc ? k : kc;
        const int m = kk / p.v;
        const int e = kk - m * p.v;
        const int s = p.lut[m * p.o + g_j];
        const int64_t pr = (s > 0 ? s : (s < 0 ? -s : 1)) - 1;
        bmask |= (g_nok && k < kend && s != 0) ? (1u << r) : 0u;
        bneg |= (s < 0) ? (1u << r) : 0u;
        rb[r] = B[(pr * p.v + e) * p.ldb + g_c];
      }
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const T x = ((amask >> r) & 1u) ? ra[r] : T(0);
      if (TA) As[buf][a_r0 + 2 * r][a_c0] = x;
      else    As[buf][a_c0][a_r0 + 16 * r] = x;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      T x = ((bmask >> r) & 1u) ? rb[r] : T(0);
      if (BMODE == B_OVVO) x = ((bneg >> r) & 1u) ? -x : x;
      if (BMODE == B_TRANS) Bs[buf][b_c0][b_r0 + 16 * r] = x;
      else                  Bs[buf][b_r0 + 2 * r][b_c0] = x;
    }
  };

  C4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = C4{0, 0, 0, 0};

  if (kbeg < kend) {
    load_tile(kbeg);
    store_tile(0);
    __syncthreads();
    const int row_l = lane & 15, kq = lane >> 4;
    int buf = 0;
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
      const bool more = k0 + BK < kend;
      if (more) load_tile(k0 + BK);
#pragma unroll
      for (int s = 0; s < BK / 4; ++s) {
        T af[4], bf[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) af[i] = As[buf][s * 4 + kq][wm * 64 + i * 16 + row_l];
#pragma unroll
        for (int j = 0; j < 4; ++j) bf[j] = Bs[buf][s * 4 + kq][wn * 64 + j * 16 + row_l];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = M4::op(af[i], bf[j], acc[i][j]);
      }
      if (more) store_tile(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  // ---- epilogue (per-type output layout of the 16x16 block, see Mfma<T>::row)
  T* __restrict__ C = p.C + bidx * p.sC;
  if (SPLIT) C += (int64_t)blockIdx.z * p.sC;  // partial buffer: one [M][N] slab per split
  const int col_l = lane & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + col_l;
      if (n >= p.N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * 64 + i * 16 + M4::row(lane, q);
        if (m >= p.M) continue;
        T* dst = C + (int64_t)m * p.ldc + n;
        if (SPLIT) {
          *dst = acc[i][j][q];
        } else {
          T val = p.alpha * acc[i][j][q];
          if (p.beta != T(0)) val += p.beta * *dst;
          *dst = val;
        }
      }
    }
}

// Sum split-K partials: C = alpha * sum_z part[z] + beta * C
template <typename T>
__global__ void splitk_reduce(const T* __restrict__ part, int splits, int M, int N,
                              int64_t pstride, T* __restrict__ C, int64_t ldc, T alpha, T beta) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)M * N) return;
  int m = (int)(idx / N), n = (int)(idx % N);
  T s = T(0);
  for (int z = 0; z < splits; ++z) s += part[z * pstride + idx];
  T* dst = C + (int64_t)m * ldc + n;
  T val = alpha * s;
  if (beta != T(0)) val += beta * *dst;
  *dst = val;
}

template <typename T, bool TA, int BMODE>
void launch(gfcc_ctx* ctx, Params<T> p, int batch, int splits) {
  dim3 grid(p.mtiles * p.ntiles, batch, splits);
  if (splits > 1)
    hipLaunchKernelGGL((gemm_kernel<T, TA, BMODE, true>), grid, dim3(NT), 0, ctx->stream, p);
  else
    hipLaunchKernelGGL((gemm_kernel<T, TA, BMODE, false>), grid, dim3(NT), 0, ctx->stream, p);
  GFCC_LAUNCH_CHECK();
}

template <typename T>
void dispatch(gfcc_ctx* ctx, bool ta, int bmode, Params<T> p, int batch, int splits) {
  if (ta) {
    if (bmode == B_ROW) launch<T, true, B_ROW>(ctx, p, batch, splits);
    else if (bmode == B_TRANS) launch<T, true, B_TRANS>(ctx, p, batch, splits);
    else launch<T, true, B_OVVO>(ctx, p, batch, splits);
  } else {
    if (bmode == B_ROW) launch<T, false, B_ROW>(ctx, p, batch, splits);
    else if (bmode == B_TRANS) launch<T, false, B_TRANS>(ctx, p, batch, splits);
    else launch<T, false, B_OVVO>(ctx, p, batch, splits);
  }
}

// choose a split-K factor so that small-output, long-K products still fill the chip
inline int choose_splits(int tiles, int batch, int K, int* kchunk) {
  int splits = 1;
  const int64_t work = (int64_t)tiles * batch;
  if (work < 512 && K >= 4 * BK * 8) {
    int64_t want = (1024 + work - 1) / work;
    int64_t maxs = K / (BK * 8);
    splits = (int)std::min<int64_t>(want, maxs);
    if (splits < 1) splits = 1;
  }
  int64_t chunk = ((int64_t)K + splits - 1) / splits;
  chunk = (chunk + BK - 1) / BK * BK;
  splits = (int)(((int64_t)K + chunk - 1) / chunk);
  *kchunk = (int)chunk;
  return splits;
}

template <typename T>
void gemm_impl(gfcc_ctx* ctx, bool transA, int bmode, int M, int N, int K, T alpha, const T* A,
               int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc, int batch,
               int64_t sA, int64_t sB, int64_t sC, const int* lut, int o, int v, int nc) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {  // C = beta * C
    GFCC_REQUIRE(batch == 1, GFCC_EINVAL, "gemm: K == 0 with batch > 1 unsupported");
    Params<T> p{};
    p.M = M; p.N = N; p.K = 0; p.A = A; p.B = B; p.C = C; p.lda = lda; p.ldb = ldb;
    p.ldc = ldc; p.alpha = alpha; p.beta = beta; p.mtiles = (M + BM - 1) / BM;
    p.ntiles = (N + BN - 1) / BN; p.lut = lut; p.o = o; p.v = v; p.nc = nc;
    dispatch<T>(ctx, transA, bmode, p, 1, 1);
    return;
  }
  Params<T> p{};
  p.M = M; p.N = N; p.K = K;
  p.A = A; p.lda = lda; p.sA = sA;
  p.B = B; p.ldb = ldb; p.sB = sB;
  p.alpha = alpha; p.beta = beta;
  p.mtiles = (M + BM - 1) / BM;
  p.ntiles = (N + BN - 1) / BN;
  p.lut = lut; p.o = o; p.v = v; p.nc = nc;
  const int64_t tiles = (int64_t)p.mtiles * p.ntiles;
  GFCC_REQUIRE(tiles < (1LL << 31), GFCC_EINVAL, "gemm: too many tiles");
  int kchunk = K;
  int splits = batch == 1 ? choose_splits((int)tiles, batch, K, &kchunk) : 1;
  if (splits <= 1) {
    p.C = C; p.ldc = ldc; p.sC = sC; p.kchunk = K;
    dispatch<T>(ctx, transA, bmode, p, batch, 1);
    return;
  }
  const int64_t slab = (int64_t)M * N;
  ws_ensure(ctx, ctx->ws_gemm, (size_t)slab * splits * sizeof(T));
  T* part = ctx->ws_gemm.as<T>();
  p.C = part; p.ldc = N; p.sC = slab; p.kchunk = kchunk;
  dispatch<T>(ctx, transA, bmode, p, 1, splits);
  hipLaunchKernelGGL(splitk_reduce<T>, dim3(blocks_for(slab, 256)), dim3(256), 0, ctx->stream,
                     part, splits, M, N, slab, C, ldc, alpha, beta);
  GFCC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------- autotuner
// Products with a row-major B whose 128 x 128 tiles cannot fill the chip but whose K is long
// (the skinny products of the sigma: [W1 ; Vp^T] . X, Vp^T . X2) run split-K. The variants
// are the generic kernel with its heuristic split count and the pipelined kernel with the
// split counts that fill one, two and four rounds of the 512 resident workgroups (two per CU),
// each split keeping at least 8 slabs of k. Products with 256 to 4095 tiles and a long K (the
// operator build's O(o^3 v^3) products) lose up to a third of a round to the last, partly
// filled one; their variants are the plain pipelined kernel and 2 .. 6 splits, which move
// the tail. The first time a
// shape is seen on a context every variant is timed (HIP events, once to warm up and twice
// timed, into a scratch output; this synchronises the stream), and the fastest is kept for
// that context and product class (tile counts, the binary magnitude of K, vector loads).
inline bool tunable(int M, int N, int K, size_t elem) {
  const int64_t tiles = (int64_t)((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  return tiles < 256 && (int64_t)K * (int64_t)elem >= 8 * 128 * 4;
}

constexpr int64_t MID_TILES_MAX = 4096;
constexpr size_t MID_SCRATCH_MAX = size_t(2) << 30;  // bytes of split-K partials
inline bool tunable_mid(int M, int N, int K, size_t elem) {
  const int64_t tiles = (int64_t)((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  return tiles >= 256 && tiles < MID_TILES_MAX && (int64_t)K * (int64_t)elem >= 2 * 8 * 128 &&
         (size_t)M * N * elem * 2 <= MID_SCRATCH_MAX;
}

// splits: 0 the generic kernel; 1 in a mid-size class the plain pipelined kernel; else the
// pipelined kernel over that many k ranges plus a reduction
template <typename T>
void run_variant(gfcc_ctx* ctx, int splits, bool transA, int M, int N, int K, T alpha,
                 const T* A, int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc,
                 bool mid = false) {
  if (splits == 0 ||
      (mid && splits == 1 && !gemm_pipe<T>(ctx, transA, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc))) {
    gemm_impl<T>(ctx, transA, B_ROW, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, 1, 0, 0, 0,
                 nullptr, 0, 0, 0);
    return;
  }
  if (mid && splits == 1) return;
  constexpr int PBK = 128 / (int)sizeof(T);
  int64_t kchunk = ((int64_t)K + splits - 1) / splits;
  kchunk = (kchunk + PBK - 1) / PBK * PBK;
  const int s = (int)(((int64_t)K + kchunk - 1) / kchunk);
  const int64_t slab = (int64_t)M * N;
  ws_ensure(ctx, ctx->ws_gemm, (size_t)slab * s * sizeof(T));
  T* part = ctx->ws_gemm.as<T>();
  gemm_pipe_split<T>(ctx, transA, M, N, K, A, lda, B, ldb, part, s, (int)kchunk);
  hipLaunchKernelGGL(splitk_reduce<T>, dim3(blocks_for(slab, 256)), dim3(256), 0, ctx->stream,
                     part, s, M, N, slab, C, ldc, alpha, beta);
  GFCC_LAUNCH_CHECK();
}

template <typename T>
const TuneChoice& tune_choice(gfcc_ctx* ctx, bool transA, int M, int N, int K, const T* A,
                              int64_t lda, const T* B, int64_t ldb, bool mid = false) {
  constexpr int PBK = 128 / (int)sizeof(T);
  constexpr int VPC = 16 / (int)sizeof(T);
  const int64_t mt = (M + BM - 1) / BM, nt = (N + BN - 1) / BN;
  const int64_t tiles = mt * nt;
  int64_t kb = 0;
  while ((int64_t(1) << (kb + 1)) <= K) ++kb;
  const int64_t vec = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % VPC == 0) &&
                      ((transA ? M : K) % VPC == 0);
  const TuneKey key{(int64_t)sizeof(T), transA ? 1 : 0, mt, nt, kb, vec};
  auto it = ctx->tune.find(key);
  if (it != ctx->tune.end()) return it->second;
  TuneChoice ch;
  ch.M = M;
  ch.N = N;
  ch.K = K;
  if (mid) ch.splits = 1;
  if (ctx->tune_mode == 0) return ctx->tune[key] = ch;
  const int64_t smax = std::max<int64_t>(1, (int64_t)K / (8 * PBK));
  std::vector<int> cand;
  if (mid) {
    // the plain kernel, then 2 .. 6 k ranges while the partials fit the scratch bound
    cand.push_back(1);
    for (int64_t sp = 2; sp <= std::min<int64_t>(6, smax); ++sp)
      if ((size_t)M * N * sizeof(T) * sp <= MID_SCRATCH_MAX) cand.push_back((int)sp);
  } else {
    // split counts that fill r whole rounds of the 512 workgroups resident at once (two per CU)
    cand.push_back(0);
    for (int64_t r : {1, 2, 4}) {
      const int64_t sp = std::min<int64_t>(smax, std::max<int64_t>(1, r * 512 / tiles));
      if (std::find(cand.begin(), cand.end(), (int)sp) == cand.end()) cand.push_back((int)sp);
    }
  }
  if (ctx->tune_mode == 2) {  // no timing: the most split variant (exercises split-K)
    ch.splits = *std::max_element(cand.begin(), cand.end());
    return ctx->tune[key] = ch;
  }
  const bool log = std::getenv("GFCC_TUNE_LOG") != nullptr;  // diagnostic: every timing
  DevBuf scratch;
  scratch.alloc(sizeof(T) * (size_t)M * N);
  hipStream_t st = ctx->stream;
  hipEvent_t e0, e1;
  GFCC_HIP(hipEventCreate(&e0));
  GFCC_HIP(hipEventCreate(&e1));
  double best = 1e300;
  for (int sp : cand) {
    run_variant<T>(ctx, sp, transA, M, N, K, T(1), A, lda, B, ldb, T(0), scratch.as<T>(), N, mid);
    GFCC_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 2; ++r)
      run_variant<T>(ctx, sp, transA, M, N, K, T(1), A, lda, B, ldb, T(0), scratch.as<T>(), N,
                     mid);
    GFCC_HIP(hipEventRecord(e1, st));
    GFCC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    GFCC_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double us = ms * 1e3 / 2;
    if (log) {
      std::fprintf(stderr, "[gfcc autotune] %s M=%d N=%d K=%d transA=%d splits=%d: %.1f us\n",
                   sizeof(T) == 8 ? "f64" : "f32", M, N, K, transA ? 1 : 0, sp, us);
    }
    if (sp == (mid ? 1 : 0)) ch.generic_us = us;
    if (us < best) {
      best = us;
      ch.splits = sp;
      ch.best_us = us;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ctx->tune[key] = ch;
}

}  // namespace

// Products whose 128 x 128 tiles number under 64 with K from 128 up to the split-K products'
// bound (the small build products: one to four workgroups on the 128 x 128 kernels, each
// walking all of K; longer K is the split-K tuner's, whose products are bandwidth-bound)
inline bool small_product(int M, int N, int K, size_t elem) {
  const int64_t tiles = (int64_t)((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  return tiles < 64 && K >= 128 && (int64_t)K * (int64_t)elem < 8 * 128 * 4;
}

template <typename T>
void gemm_route(gfcc_ctx* ctx, bool transA, bool transB, int M, int N, int K, T alpha,
                const T* A, int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc,
                int batch, int64_t sA, int64_t sB, int64_t sC);

// A small row-major product (see small_product): the first call in a class times the generic
// route and every tile and split candidate of the segmented kernel, all into a scratch output
// with beta = 0 (so that a product that accumulates into C is not run more than once on it),
// and keeps the fastest; class = element bytes, TUNE_SMALL, the counts of 32-row and 64-column
// tiles, floor(log2 K).
template <typename T>
void gemm_small(gfcc_ctx* ctx, int M, int N, int K, T alpha, const T* A, int64_t lda,
                const T* B, int64_t ldb, T beta, T* C, int64_t ldc) {
  SegSpec<T> s;
  s.M = M;
  s.N = N;
  s.K[0] = K;
  s.A[0] = A;
  s.lda[0] = lda;
  s.B[0] = B;
  s.ldb[0] = ldb;
  s.C = C;
  s.ldc = ldc;
  s.alpha = alpha;
  s.beta = beta;
  int64_t kb = 0;
  while ((int64_t(1) << (kb + 1)) <= K) ++kb;
  const TuneKey key{(int64_t)sizeof(T), TUNE_SMALL, (M + 31) / 32, (N + 63) / 64, kb, 0};
  auto it = ctx->tune.find(key);
  if (it == ctx->tune.end()) {
    std::vector<std::array<int, 3>> cand;
    segmm_candidates(s, cand);
    TuneChoice ch;
    ch.M = M;
    ch.N = N;
    ch.K = K;
    int pick = 0;  // 0: generic route, i > 0: cand[i - 1]
    if (ctx->tune_mode == 2) {
      pick = 1;  // untimed: the segmented product on its most split candidate
      for (size_t i = 1; i < cand.size(); ++i)
        if (cand[i][2] > cand[pick - 1][2]) pick = (int)i + 1;
    } else if (ctx->tune_mode == 1) {
      DevBuf scratch;
      scratch.alloc(sizeof(T) * (size_t)M * N);
      segmm_reserve(ctx, s, cand);
      SegSpec<T> t = s;
      t.C = scratch.as<T>();
      t.ldc = N;
      t.beta = T(0);
      std::vector<std::function<void()>> fns{[&] {
        gemm_route<T>(ctx, false, false, M, N, K, alpha, A, lda, B, ldb, T(0), t.C, N, 1, 0, 0,
                      0);
      }};
      for (const auto& c : cand)
        fns.push_back([&, c] { segmm_run<T>(ctx, t, c[0], c[1], c[2]); });
      std::vector<double> us;
      pick = time_candidates(ctx, fns, us);
      ch.best_us = us[pick];
      ch.generic_us = us[0];
      if (std::getenv("GFCC_TUNE_LOG")) {
        for (size_t i = 0; i < fns.size(); ++i)
          std::fprintf(stderr, "[gfcc autotune] small M=%d N=%d K=%d %s %dx%d splits=%d: %.1f us\n",
                       M, N, K, i == 0 ? "generic" : "tile", i ? cand[i - 1][0] : 0,
                       i ? cand[i - 1][1] : 0, i ? cand[i - 1][2] : 0, us[i]);
      }
    }
    if (pick > 0) {
      ch.tile_m = cand[pick - 1][0];
      ch.tile_n = cand[pick - 1][1];
      ch.splits = cand[pick - 1][2];
    }
    it = ctx->tune.emplace(key, ch).first;
  }
  const TuneChoice& ch = it->second;
  if (ch.tile_m == 0) {
    gemm_route<T>(ctx, false, false, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, 1, 0, 0, 0);
    return;
  }
  segmm_run<T>(ctx, s, ch.tile_m, ch.tile_n, ch.splits);
}

template <typename T>
void gemm(gfcc_ctx* ctx, bool transA, bool transB, int M, int N, int K, T alpha, const T* A,
          int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc, int batch,
          int64_t sA, int64_t sB, int64_t sC) {
  // a large transposed B ([N][K], contiguous; the operator build's l2 t2^T and oovv tau^T), or
  // that of a small product, is transposed once into the context's transpose workspace so that
  // the product takes the row-major paths below (stream order protects the workspace until the
  // product has read it)
  if (transB && batch == 1 && sizeof(T) == 8 && ldb == K &&
      ((int64_t)K * N >= (1 << 20) ||
       (!transA && M > 0 && N > 0 && small_product(M, N, K, sizeof(T)))) &&
      N < 65536 * 32) {
    ws_ensure(ctx, ctx->ws_trans, sizeof(T) * (size_t)K * N);
    transpose2d(ctx, reinterpret_cast<const double*>(B), N, K, ctx->ws_trans.as<double>());
    gemm<T>(ctx, transA, false, M, N, K, alpha, A, lda, ctx->ws_trans.as<T>(), N, beta, C, ldc);
    return;
  }
  if (!transA && !transB && batch == 1 && M > 0 && N > 0 && small_product(M, N, K, sizeof(T)) &&
      ctx->tune_mode != 0) {
    gemm_small<T>(ctx, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    return;
  }
  gemm_route<T>(ctx, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, batch, sA, sB,
                sC);
}

// the routes of a product that is not small (or whose small-product tuning chose the generic
// route)
template <typename T>
void gemm_route(gfcc_ctx* ctx, bool transA, bool transB, int M, int N, int K, T alpha,
                const T* A, int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc,
                int batch, int64_t sA, int64_t sB, int64_t sC) {
  // mid-size products with a long K: plain pipelined kernel or split-K, as tuned
  if (!transB && batch == 1 && M > 0 && N > 0 && tunable_mid(M, N, K, sizeof(T))) {
    const TuneChoice& ch = tune_choice<T>(ctx, transA, M, N, K, A, lda, B, ldb, true);
    const int pbk = 128 / (int)sizeof(T);
    const int sp = (int)std::max<int64_t>(1, std::min<int64_t>(ch.splits, K / (8 * pbk)));
    run_variant<T>(ctx, sp, transA, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, true);
    return;
  }
  // large single products with a row-major B go to the pipelined kernel
  if (!transB && batch == 1 &&
      gemm_pipe<T>(ctx, transA, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc))
    return;
  // skinny long-K products: split-K variant chosen by the autotuner
  if (!transB && batch == 1 && M > 0 && N > 0 && tunable(M, N, K, sizeof(T))) {
    const TuneChoice& ch = tune_choice<T>(ctx, transA, M, N, K, A, lda, B, ldb);
    // a class member measured on another K keeps at least 8 slabs of k per split
    const int pbk = 128 / (int)sizeof(T);
    const int sp = ch.splits > 0 ? (int)std::max<int64_t>(1, std::min<int64_t>(ch.splits, K / (8 * pbk)))
                                 : 0;
    run_variant<T>(ctx, sp, transA, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    return;
  }
  gemm_impl<T>(ctx, transA, transB ? B_TRANS : B_ROW, M, N, K, alpha, A, lda, B, ldb, beta, C,
               ldc, batch, sA, sB, sC, nullptr, 0, 1, 1);
}

template void gemm<double>(gfcc_ctx*, bool, bool, int, int, int, double, const double*, int64_t,
                           const double*, int64_t, double, double*, int64_t, int, int64_t,
                           int64_t, int64_t);
template void gemm<float>(gfcc_ctx*, bool, bool, int, int, int, float, const float*, int64_t,
                          const float*, int64_t, float, float*, int64_t, int, int64_t, int64_t,
                          int64_t);

namespace {
// The ovvo operand written out: R[(m, e)][(j, c)] = r_mj^e[c] = sign X2[(pair, e)][c] with the
// pair and sign of (m, j) from pairlut (+(pair+1) for m < j, -(pair+1) for m > j, 0 for m = j)
__global__ void ovvo_expand_kernel(const double* __restrict__ X2, int64_t ldx,
                                   const int* __restrict__ lut, int o, int v, int nc,
                                   double* __restrict__ R) {
  const int64_t N = (int64_t)o * nc, total = (int64_t)o * v * N;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / N, col = i - row * N;
    const int m = (int)(row / v), e = (int)(row - (int64_t)m * v);
    const int j = (int)(col / nc), c = (int)(col - (int64_t)j * nc);
    const int l = lut[m * o + j];
    double x = 0.0;
    if (l != 0) {
      const int pr = (l > 0 ? l : -l) - 1;
      x = X2[((int64_t)pr * v + e) * ldx + c];
      if (l < 0) x = -x;
    }
    R[i] = x;
  }
}
}  // namespace

// Small forward FP64 ovvo products (the written-out operand at most 64 MiB): the ovvo kernel
// runs one 128 x 128 tile per CU at most, each walking all of K, so at the small case it is
// bound by one CU's matrix throughput on 200 tiles. The alternative writes the operand out
// (one HBM-bound pass) and runs the segmented kernel on small tiles; the tuner times the ovvo
// kernel against every tile and split of it (class: TUNE_OVVO, o, v, 64-column groups).
static bool ovvo_small(gfcc_ctx* ctx, int o, int v, int nc, const double* W, const double* X2,
                       int64_t ldx, const int* pairlut, double* Z,
                       const std::function<void()>& kernel_route) {
  const int64_t OV = (int64_t)o * v, N = (int64_t)o * nc;
  if (ctx->tune_mode == 0 || OV * N * 8 > (int64_t(64) << 20) || OV >= (1 << 20)) return false;
  SegSpec<double> s;
  s.M = (int)OV;
  s.N = (int)N;
  s.K[0] = (int)OV;
  s.A[0] = W;
  s.lda[0] = OV;
  s.ldb[0] = N;
  s.C = Z;
  s.ldc = N;
  auto expand = [&]() {
    ws_ensure(ctx, ctx->ws_rexp, sizeof(double) * (size_t)(OV * N));
    const int64_t nblk = std::min<int64_t>(16384, std::max<int64_t>(1, (OV * N + 255) / 256));
    hipLaunchKernelGGL(ovvo_expand_kernel, dim3((unsigned)nblk), dim3(256), 0, ctx->stream,
                       X2, ldx, pairlut, o, v, nc, ctx->ws_rexp.as<double>());
    GFCC_LAUNCH_CHECK();
  };
  const TuneKey key{8, TUNE_OVVO, o, v, (nc + 63) / 64, 0};
  auto it = ctx->tune.find(key);
  if (it == ctx->tune.end()) {
    ws_ensure(ctx, ctx->ws_rexp, sizeof(double) * (size_t)(OV * N));
    s.B[0] = ctx->ws_rexp.as<double>();
    std::vector<std::array<int, 3>> cand;
    segmm_candidates(s, cand);
    TuneChoice ch;
    ch.M = s.M;
    ch.N = s.N;
    ch.K = s.K[0];
    int pick = 0;
    if (ctx->tune_mode == 2) {
      pick = 1;
      for (size_t i = 1; i < cand.size(); ++i)
        if (cand[i][2] > cand[pick - 1][2]) pick = (int)i + 1;
    } else {
      segmm_reserve(ctx, s, cand);
      std::vector<std::function<void()>> fns{kernel_route};
      for (const auto& c : cand)
        fns.push_back([&, c] {
          expand();
          segmm_run<double>(ctx, s, c[0], c[1], c[2]);
        });
      std::vector<double> us;
      pick = time_candidates(ctx, fns, us);
      ch.best_us = us[pick];
      ch.generic_us = us[0];
      if (std::getenv("GFCC_TUNE_LOG")) {
        for (size_t i = 0; i < fns.size(); ++i)
          std::fprintf(stderr, "[gfcc autotune] ovvo o=%d v=%d nc=%d %s %dx%d splits=%d: %.1f us\n",
                       o, v, nc, i == 0 ? "kernel" : "expanded", i ? cand[i - 1][0] : 0,
                       i ? cand[i - 1][1] : 0, i ? cand[i - 1][2] : 0, us[i]);
      }
    }
    if (pick > 0) {
      ch.tile_m = cand[pick - 1][0];
      ch.tile_n = cand[pick - 1][1];
      ch.splits = cand[pick - 1][2];
    }
    it = ctx->tune.emplace(key, ch).first;
  }
  const TuneChoice& ch = it->second;
  if (ch.tile_m == 0) return false;
  expand();
  s.B[0] = ctx->ws_rexp.as<double>();
  segmm_run<double>(ctx, s, ch.tile_m, ch.tile_n, ch.splits);
  return true;
}

template <typename T>
void gemm_ovvo(gfcc_ctx* ctx, bool transW, int o, int v, int nc, const T* W, const T* X2,
               int64_t ldx, const int* pairlut, T* Z) {
  const T* zrow = static_cast<const T*>(zero_row(ctx, (size_t)nc * sizeof(T)));
  const int OV = o * v;
  auto kernel_route = [&]() {
    if (ovvo_fast<T>(ctx, transW, o, v, nc, W, X2, ldx, Z, zrow)) return;
    gemm_impl<T>(ctx, transW, B_OVVO, OV, o * nc, OV, T(1), W, OV, X2, ldx, T(0), Z,
                 (int64_t)o * nc, 1, 0, 0, 0, pairlut, o, v, nc);
  };
  if constexpr (sizeof(T) == 8) {
    if (!transW && ovvo_small(ctx, o, v, nc, reinterpret_cast<const double*>(W),
                              reinterpret_cast<const double*>(X2), ldx, pairlut,
                              reinterpret_cast<double*>(Z), kernel_route))
      return;
  }
  kernel_route();
}

template void gemm_ovvo<double>(gfcc_ctx*, bool, int, int, int, const double*, const double*,
                                int64_t, const int*, double*);
template void gemm_ovvo<float>(gfcc_ctx*, bool, int, int, int, const float*, const float*,
                               int64_t, const int*, float*);


// ------------------------------------------------------------------ segmented products
// One workgroup of 4 wavefronts (2 x 2) computes a TBM x TBN tile of C_b (TBM in {32, 64, 128},
// TBN in {64, 128}); each wavefront holds (TBM/32) x (TBN/32) accumulators of the 16x16x4
// MFMA. K runs over the concatenated slabs (16 deep) of the segments, loaded two slabs ahead
// into two register sets and stored into double-buffered LDS (these products are short in K
// per workgroup, so their time is mostly load latency); ragged edges are zero-filled on load
// and masked on store. Split-K (batch 1) gives each blockIdx.z a contiguous run of slabs and writes an
// [M][N] partial per split.
namespace {

template <typename T> struct SegArgs {
  const T* A[SEG_MAX];
  const T* B[SEG_MAX];
  int64_t lda[SEG_MAX], sA[SEG_MAX], ldb[SEG_MAX], sB[SEG_MAX];
  int K[SEG_MAX], ns[SEG_MAX];
  int nseg, M, N, mtiles, msplit, spz;
  T* C;
  T* C2;
  int64_t ldc, sC, pstride;
  T alpha, beta;
  const T* Zas;  // antisymmetrised ovvo term of the epilogue (null: none)
  int as_o, as_v, as_nc;
};

// (i, j) of pair p = i o - i (i + 1) / 2 + (j - i - 1), i < j < o: the root of the quadratic in
// double, then an exact integer correction
__device__ __forceinline__ void pair_ij(int p, int o, int& i, int& j) {
  const double b = 2.0 * o - 1.0;
  int ii = (int)floor((b - sqrt(b * b - 8.0 * p)) * 0.5);
  ii = max(0, min(ii, o - 2));
  while (ii > 0 && ii * o - (ii * (ii + 1) >> 1) > p) --ii;
  while (ii + 1 <= o - 2 && (ii + 1) * o - ((ii + 1) * (ii + 2) >> 1) <= p) ++ii;
  i = ii;
  j = p - (ii * o - (ii * (ii + 1) >> 1)) + ii + 1;
}

template <typename T, int TBM, int TBN, bool SPLIT, bool AS>
__global__ __launch_bounds__(NT, 2) void segmm_kernel(SegArgs<T> p) {
  using M4 = Mfma<T>;
  using C4 = typename M4::C4;
  constexpr int PAD = M4::PAD;
  constexpr int RA = TBM / 16;  // A loads per thread and slab: k = tid % 16, rows tid / 16 + 16 r
  constexpr int RB = TBN / 16;  // B loads: n = tid % TBN, k = tid / TBN + KS r
  constexpr int KS = NT / TBN;
  constexpr int IW = TBM / 32, JW = TBN / 32;
  __shared__ T As[2][BK][TBM + PAD];
  __shared__ T Bs[2][BK][TBN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int mt = blockIdx.x % p.mtiles, nt = blockIdx.x / p.mtiles;
  const int m0 = mt * TBM, n0 = nt * TBN;
  const int64_t bi = blockIdx.y;

  int total = 0;
  for (int q = 0; q < p.nseg; ++q) total += p.ns[q];
  int sbeg = 0, send = total;
  if (SPLIT) {
    sbeg = blockIdx.z * p.spz;
    send = min(total, sbeg + p.spz);
  }
  const int a_k = tid % BK, a_m = tid / BK;
  const int b_n = tid % TBN, b_k = tid / TBN;
  const int Mc = p.M - 1, Nc = p.N - 1;

  // two register sets: the loads of slab s + 2 are in flight while slab s is multiplied
  T ra0[RA], rb0[RB], ra1[RA], rb1[RB];
  unsigned am0 = 0, bm0 = 0, am1 = 0, bm1 = 0;
  auto load_slab = [&](int sl, T(&ra)[RA], T(&rb)[RB], unsigned& amask, unsigned& bmask) {
    int q = 0;
    while (q + 1 < p.nseg && sl >= p.ns[q]) {
      sl -= p.ns[q];
      ++q;
    }
    const int k0 = sl * BK;
    const int K = p.K[q];
    const int kc = K - 1;
    const T* __restrict__ A = p.A[q] + bi * p.sA[q];
    const T* __restrict__ B = p.B[q] + bi * p.sB[q];
    const int64_t lda = p.lda[q], ldb = p.ldb[q];
    amask = bmask = 0;
#pragma unroll
    for (int r = 0; r < RA; ++r) {
      const int m = m0 + a_m + 16 * r, k = k0 + a_k;
      amask |= (m < p.M && k < K) ? (1u << r) : 0u;
      const int mm = m < Mc ? m : Mc, kk = k < kc ? k : kc;
      ra[r] = A[(int64_t)mm * lda + kk];
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      const int k = k0 + b_k + KS * r, n = n0 + b_n;
      bmask |= (n < p.N && k < K) ? (1u << r) : 0u;
      const int nn = n < Nc ? n : Nc, kk = k < kc ? k : kc;
      rb[r] = B[(int64_t)kk * ldb + nn];
    }
  };
  auto store_slab = [&](int buf, const T(&ra)[RA], const T(&rb)[RB], unsigned amask,
                        unsigned bmask) {
#pragma unroll
    for (int r = 0; r < RA; ++r) As[buf][a_k][a_m + 16 * r] = ((amask >> r) & 1u) ? ra[r] : T(0);
#pragma unroll
    for (int r = 0; r < RB; ++r) Bs[buf][b_k + KS * r][b_n] = ((bmask >> r) & 1u) ? rb[r] : T(0);
  };

  C4 acc[IW][JW];
#pragma unroll
  for (int i = 0; i < IW; ++i)
#pragma unroll
    for (int j = 0; j < JW; ++j) acc[i][j] = C4{0, 0, 0, 0};

  // AS: the epilogue's antisymmetric term; small tiles load it before the k loop so that its
  // latency hides behind the slabs (rows and columns clamped into range; out-of-range entries
  // are not stored), larger ones in the epilogue
  constexpr bool PREZ = AS && IW * JW <= 4;
  C4 zdiff[PREZ ? IW : 1][PREZ ? JW : 1];
  auto zterm = [&](int m, int n) {
    const int64_t ldz = (int64_t)p.as_o * p.as_nc;
    int pi, pj;
    pair_ij(m, p.as_o, pi, pj);
    return p.Zas[((int64_t)pi * p.as_v + bi) * ldz + (int64_t)pj * p.as_nc + n] -
           p.Zas[((int64_t)pj * p.as_v + bi) * ldz + (int64_t)pi * p.as_nc + n];
  };
  if (PREZ) {
#pragma unroll
    for (int i = 0; i < IW; ++i)
#pragma unroll
      for (int j = 0; j < JW; ++j) {
        const int n = min(n0 + wn * (TBN / 2) + j * 16 + (lane & 15), Nc);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          zdiff[PREZ ? i : 0][PREZ ? j : 0][q] =
              zterm(min(m0 + wm * (TBM / 2) + i * 16 + M4::row(lane, q), Mc), n);
      }
  }

  const int row_l = lane & 15, kq = lane >> 4;
  auto compute = [&](int buf) {
#pragma unroll
    for (int s4 = 0; s4 < BK / 4; ++s4) {
      T af[IW], bf[JW];
#pragma unroll
      for (int i = 0; i < IW; ++i) af[i] = As[buf][s4 * 4 + kq][wm * (TBM / 2) + i * 16 + row_l];
#pragma unroll
      for (int j = 0; j < JW; ++j) bf[j] = Bs[buf][s4 * 4 + kq][wn * (TBN / 2) + j * 16 + row_l];
#pragma unroll
      for (int i = 0; i < IW; ++i)
#pragma unroll
        for (int j = 0; j < JW; ++j) acc[i][j] = M4::op(af[i], bf[j], acc[i][j]);
    }
  };

  // the FP64 128 x 128 tile has no registers for a second set: one slab ahead
  constexpr bool ONE_AHEAD = sizeof(T) == 8 && TBM * TBN >= 128 * 128;
  if (ONE_AHEAD && sbeg < send) {
    load_slab(sbeg, ra0, rb0, am0, bm0);
    store_slab(0, ra0, rb0, am0, bm0);
    __syncthreads();
    int buf = 0;
    for (int sl = sbeg; sl < send; ++sl) {
      const bool more = sl + 1 < send;
      if (more) load_slab(sl + 1, ra0, rb0, am0, bm0);
      compute(buf);
      if (more) store_slab(buf ^ 1, ra0, rb0, am0, bm0);
      __syncthreads();
      buf ^= 1;
    }
  } else if (sbeg < send) {
    load_slab(sbeg, ra0, rb0, am0, bm0);
    if (sbeg + 1 < send) load_slab(sbeg + 1, ra1, rb1, am1, bm1);
    store_slab(0, ra0, rb0, am0, bm0);
    __syncthreads();
    for (int sl = sbeg; sl < send; sl += 2) {
      // LDS buffer 0 holds slab sl, register set 1 slab sl + 1 (when there is one)
      if (sl + 2 < send) load_slab(sl + 2, ra0, rb0, am0, bm0);
      compute(0);
      if (sl + 1 >= send) break;
      store_slab(1, ra1, rb1, am1, bm1);
      __syncthreads();
      if (sl + 3 < send) load_slab(sl + 3, ra1, rb1, am1, bm1);
      compute(1);
      if (sl + 2 < send) store_slab(0, ra0, rb0, am0, bm0);
      __syncthreads();
    }
  }

  const int col_l = lane & 15;
#pragma unroll
  for (int i = 0; i < IW; ++i)
#pragma unroll
    for (int j = 0; j < JW; ++j) {
      const int n = n0 + wn * (TBN / 2) + j * 16 + col_l;
      if (n >= p.N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * (TBM / 2) + i * 16 + M4::row(lane, q);
        if (m >= p.M) continue;
        if (SPLIT) {
          p.C[(int64_t)blockIdx.z * p.pstride + (int64_t)m * p.N + n] = acc[i][j][q];
        } else {
          T* dst = m < p.msplit ? p.C + bi * p.sC + (int64_t)m * p.ldc + n
                                : p.C2 + bi * p.sC + (int64_t)(m - p.msplit) * p.ldc + n;
          T val = p.alpha * acc[i][j][q];
          if (p.beta != T(0)) val += p.beta * *dst;
          if (PREZ) val += zdiff[PREZ ? i : 0][PREZ ? j : 0][q];
          else if (AS) val += zterm(m, n);
          *dst = val;
        }
      }
    }
}

// C (rows >= msplit: C2) = alpha * sum_z part[z] + beta * C
template <typename T>
__global__ void segmm_reduce(const T* __restrict__ part, int splits, int M, int N,
                             int64_t pstride, T* C, T* C2, int msplit, int64_t ldc, T alpha,
                             T beta) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)M * N) return;
  const int m = (int)(idx / N), n = (int)(idx % N);
  T s = T(0);
  for (int z = 0; z < splits; ++z) s += part[z * pstride + idx];
  T* dst = m < msplit ? C + (int64_t)m * ldc + n : C2 + (int64_t)(m - msplit) * ldc + n;
  T val = alpha * s;
  if (beta != T(0)) val += beta * *dst;
  *dst = val;
}

template <typename T, int TBM, int TBN>
void segmm_launch(gfcc_ctx* ctx, SegArgs<T> a, int batch, int ntiles, int splits) {
  dim3 grid((unsigned)(a.mtiles * ntiles), (unsigned)batch, (unsigned)splits);
  if (splits > 1)
    hipLaunchKernelGGL((segmm_kernel<T, TBM, TBN, true, false>), grid, dim3(NT), 0, ctx->stream, a);
  else if (a.Zas)
    hipLaunchKernelGGL((segmm_kernel<T, TBM, TBN, false, true>), grid, dim3(NT), 0, ctx->stream, a);
  else
    hipLaunchKernelGGL((segmm_kernel<T, TBM, TBN, false, false>), grid, dim3(NT), 0, ctx->stream, a);
  GFCC_LAUNCH_CHECK();
}

inline int seg_slabs(const int* K, int nseg) {
  int t = 0;
  for (int q = 0; q < nseg; ++q) t += (K[q] + BK - 1) / BK;
  return t;
}

}  // namespace

template <typename T>
void segmm_run(gfcc_ctx* ctx, const SegSpec<T>& s, int tm, int tn, int splits) {
  if (s.M <= 0 || s.N <= 0 || s.batch <= 0) return;
  GFCC_REQUIRE(s.nseg >= 1 && s.nseg <= SEG_MAX, GFCC_EINVAL, "segmm: bad segment count");
  GFCC_REQUIRE(s.batch < 65536, GFCC_EINVAL, "segmm: batch too large");
  GFCC_REQUIRE(splits == 1 || s.batch == 1, GFCC_EINVAL, "segmm: split-K needs batch 1");
  SegArgs<T> a{};
  for (int q = 0; q < SEG_MAX; ++q) {
    const bool on = q < s.nseg;
    a.A[q] = on ? s.A[q] : nullptr;
    a.B[q] = on ? s.B[q] : nullptr;
    a.lda[q] = on ? s.lda[q] : 0;
    a.sA[q] = on ? s.sA[q] : 0;
    a.ldb[q] = on ? s.ldb[q] : 0;
    a.sB[q] = on ? s.sB[q] : 0;
    a.K[q] = on ? s.K[q] : 0;
    a.ns[q] = on ? (s.K[q] + BK - 1) / BK : 0;
    GFCC_REQUIRE(!on || s.K[q] >= 0, GFCC_EINVAL, "segmm: negative K");
  }
  a.nseg = s.nseg;
  a.M = s.M;
  a.N = s.N;
  a.mtiles = (s.M + tm - 1) / tm;
  const int ntiles = (s.N + tn - 1) / tn;
  GFCC_REQUIRE((int64_t)a.mtiles * ntiles < (1LL << 31), GFCC_EINVAL, "segmm: too many tiles");
  a.msplit = s.msplit;
  a.C = s.C;
  a.C2 = s.C2 ? s.C2 : s.C;
  a.ldc = s.ldc;
  a.sC = s.sC;
  a.alpha = s.alpha;
  a.beta = s.beta;
  a.Zas = s.Zas;
  a.as_o = s.as_o;
  a.as_v = s.as_v;
  a.as_nc = s.as_nc;
  GFCC_REQUIRE(!s.Zas || splits == 1, GFCC_EINVAL, "segmm: the antisymmetric term needs no split");
  const int total = seg_slabs(a.K, a.nseg);
  T* part = nullptr;
  int nz = 1;
  if (splits > 1 && total > 1) {
    a.spz = (total + splits - 1) / splits;
    nz = (total + a.spz - 1) / a.spz;
  } else {
    a.spz = total;
  }
  if (nz > 1) {
    a.pstride = (int64_t)s.M * s.N;
    ws_ensure(ctx, ctx->ws_gemm, sizeof(T) * (size_t)a.pstride * nz);
    part = ctx->ws_gemm.as<T>();
    a.C = part;
  }
#define GFCC_SEG_TILE(BMv, BNv) \
  if (tm == BMv && tn == BNv) { segmm_launch<T, BMv, BNv>(ctx, a, s.batch, ntiles, nz); } else
  GFCC_SEG_TILE(32, 64) GFCC_SEG_TILE(32, 128) GFCC_SEG_TILE(64, 64) GFCC_SEG_TILE(64, 128)
  GFCC_SEG_TILE(128, 64) GFCC_SEG_TILE(128, 128) {
    throw Error(GFCC_EINVAL, "segmm: unsupported tile");
  }
#undef GFCC_SEG_TILE
  if (nz > 1) {
    const int64_t slab = (int64_t)s.M * s.N;
    hipLaunchKernelGGL(segmm_reduce<T>, dim3(blocks_for(slab, 256)), dim3(256), 0, ctx->stream,
                       part, nz, s.M, s.N, slab, s.C, s.C2 ? s.C2 : s.C, s.msplit, s.ldc,
                       s.alpha, s.beta);
    GFCC_LAUNCH_CHECK();
  }
}

template <typename T>
void segmm_candidates(const SegSpec<T>& s, std::vector<std::array<int, 3>>& out) {
  out.clear();
  const int total = seg_slabs(s.K, s.nseg);
  for (int tm : {32, 64, 128}) {
    // a tile more than twice as tall as the product only adds empty rows
    if (tm > 32 && tm >= 2 * s.M) continue;
    for (int tn : {64, 128}) {
      if (tn > 64 && tn >= 2 * s.N) continue;
      const int64_t tiles = (int64_t)((s.M + tm - 1) / tm) * ((s.N + tn - 1) / tn) * s.batch;
      out.push_back({tm, tn, 1});
      if (s.batch != 1 || s.Zas) continue;
      // split counts that fill one, two and four rounds of 512 workgroups, keeping at least
      // four slabs of k per split
      for (int64_t r : {1, 2, 4}) {
        const int64_t sp = std::min<int64_t>(total / 4, r * 512 / std::max<int64_t>(1, tiles));
        if (sp < 2) continue;
        bool dup = false;
        for (const auto& c : out) dup |= (c[0] == tm && c[1] == tn && c[2] == (int)sp);
        if (!dup) out.push_back({tm, tn, (int)sp});
      }
    }
  }
}

int time_candidates(gfcc_ctx* ctx, const std::vector<std::function<void()>>& cands,
                    std::vector<double>& us) {
  hipStream_t st = ctx->stream;
  hipEvent_t e0, e1;
  GFCC_HIP(hipEventCreate(&e0));
  GFCC_HIP(hipEventCreate(&e1));
  us.assign(cands.size(), 0.0);
  int best = 0;
  auto timed = [&](const std::function<void()>& f, int reps) {
    GFCC_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < reps; ++r) f();
    GFCC_HIP(hipEventRecord(e1, st));
    GFCC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    GFCC_HIP(hipEventElapsedTime(&ms, e0, e1));
    return ms * 1e3 / reps;
  };
  for (size_t i = 0; i < cands.size(); ++i) {
    // the first run warms up; a candidate already twice as slow as the best is not run again
    const double warm = timed(cands[i], 1);
    if (i > 0 && warm > 2.0 * us[best]) {
      us[i] = warm;
      continue;
    }
    us[i] = timed(cands[i], 2);
    if (us[i] < us[best]) best = (int)i;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

template <typename T>
void segmm_reserve(gfcc_ctx* ctx, const SegSpec<T>& s,
                   const std::vector<std::array<int, 3>>& cands) {
  size_t need = 0;
  const int total = seg_slabs(s.K, s.nseg);
  for (const auto& c : cands) {
    if (c[2] <= 1 || s.batch != 1 || s.Zas || total <= 1) continue;
    const int spz = (total + c[2] - 1) / c[2];
    const int nz = (total + spz - 1) / spz;
    if (nz > 1) need = std::max(need, sizeof(T) * (size_t)s.M * s.N * nz);
  }
  ws_ensure(ctx, ctx->ws_gemm, need);
}

template void segmm_reserve<double>(gfcc_ctx*, const SegSpec<double>&,
                                    const std::vector<std::array<int, 3>>&);
template void segmm_reserve<float>(gfcc_ctx*, const SegSpec<float>&,
                                   const std::vector<std::array<int, 3>>&);
template void segmm_run<double>(gfcc_ctx*, const SegSpec<double>&, int, int, int);
template void segmm_run<float>(gfcc_ctx*, const SegSpec<float>&, int, int, int);
template void segmm_candidates<double>(const SegSpec<double>&, std::vector<std::array<int, 3>>&);
template void segmm_candidates<float>(const SegSpec<float>&, std::vector<std::array<int, 3>>&);

}  // namespace gfcc
