// The IP sigma product y = Hbar_N x on a block of vectors (Eq. xplin's operator).
//
// Vectors are stored D-major: X[D][nc] with nc real columns (complex right-hand sides are
// interleaved column pairs), so every term is a matrix product whose N dimension runs over
// the right-hand sides:
//   sigma_1h   = W1 . X
//   tau        = Vp^T . X_2h1p                 (three-body intermediate, v x nc)
// (the FP64 forward product forms both at once from the stacked [W1 ; 0 | Vp^T])
//   sigma_2h1p = W4c . [X_1h ; tau] + (Woo (x) I_v) . X_2h1p + antisym(Weff . r)
// where r_mj^e is the antisymmetric expansion of the packed 2h1p block, generated inside
// the ovvo product (gemm_ovvo), and antisym(Z)_(i<j),a = Z[(i,a)][j] - Z[(j,a)][i].
// The transpose product uses the same pieces with transposed A operands.
#include <cstdlib>

#include "common.h"

namespace gfcc {
namespace {

// Y2[(i<j, a)][c] += Z[(i,a)][j*nc + c] - Z[(j,a)][i*nc + c]; one workgroup per 2h1p row
// (pair, a), whose (i, j) it recovers once, with a wave-uniform scan over i
template <typename T>
__global__ __launch_bounds__(256) void antisym_add_kernel(const T* __restrict__ Z, int o, int v,
                                                          int nc, T* __restrict__ Y2) {
  const int64_t row = blockIdx.x;
  const int a = (int)(row % v);
  const int64_t pr = row / v;
  int i = 0;
  int64_t base = 0;
  while (i < o - 1 && pr >= base + (o - 1 - i)) {
    base += o - 1 - i;
    ++i;
  }
  const int j = (int)(i + 1 + (pr - base));
  const int64_t ldz = (int64_t)o * nc;
  const T* zij = Z + ((int64_t)i * v + a) * ldz + (int64_t)j * nc;
  const T* zji = Z + ((int64_t)j * v + a) * ldz + (int64_t)i * nc;
  T* y = Y2 + row * nc;
  for (int c = threadIdx.x; c < nc; c += blockDim.x) y[c] += zij[c] - zji[c];
}

template <typename T>
__global__ void copy_kernel(T* __restrict__ dst, const T* __restrict__ src, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <typename T>
__global__ void add_kernel(T* __restrict__ y, const T* __restrict__ x, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += x[i];
}

// complex (16-byte element) transpose: dst[c][r] = src[r][c], src is [rows][cols]
__global__ void ctranspose_kernel(const double2* __restrict__ src, int64_t rows, int64_t cols,
                                  int64_t lds, double2* __restrict__ dst, int64_t ldd) {
  __shared__ double2 tile[16][17];
  int64_t c0 = (int64_t)blockIdx.x * 16, r0 = (int64_t)blockIdx.y * 16;
  int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  {
    int64_t r = r0 + ty, c = c0 + tx;
    if (r < rows && c < cols) tile[ty][tx] = src[r * lds + c];
  }
  __syncthreads();
  {
    int64_t c = c0 + ty, r = r0 + tx;
    if (r < rows && c < cols) dst[c * ldd + r] = tile[tx][ty];
  }
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

// Y2 += (Woo (x) I_v) . X2 (or Woo^T): Woo's rows are padded with zeros to ldw, which lets the
// pipelined kernel use 16-byte loads although P is odd. With Z (forward sigma), antisym(Z) is
// added in the epilogue of the pipelined kernel when that kernel takes the product; returns
// whether it was.
template <typename T>
bool woo_product(gfcc_ctx* ctx, bool transW, int64_t P, int64_t N, const T* Woo, int64_t ldw,
                 const T* X2, T* Y2, const T* Z = nullptr, int o = 0, int v = 0, int nc = 0) {
  if (gemm_pipe<T>(ctx, transW, (int)P, (int)N, (int)P, T(1), Woo, ldw, X2, N, T(1), Y2, N, true,
                   Z, o, v, nc))
    return Z != nullptr;
  gemm<T>(ctx, transW, false, (int)P, (int)N, (int)P, T(1), Woo, ldw, X2, N, T(1), Y2, N);
  return false;
}

template <typename T>
void copy_async(gfcc_ctx* ctx, T* dst, const T* src, int64_t n) {
  hipLaunchKernelGGL(copy_kernel<T>, dim3(grid_for(n)), dim3(256), 0, ctx->stream, dst, src, n);
  GFCC_LAUNCH_CHECK();
}

// The tuned route of one of the sigma's linear products: the first call in a class times the
// unfused route (candidate 0) and every tile and split candidate of the fused segmented
// product, each a complete computation of the same outputs, and keeps the fastest.
// Returns true when the fused product ran (false: the unfused route).
template <typename T>
bool tuned_route(gfcc_ctx* ctx, int64_t kind, const SegSpec<T>& fused,
                 const std::function<void()>& unfused) {
  auto pin = ctx->tune_pins.find(kind);
  if (pin != ctx->tune_pins.end()) {
    const auto& c = pin->second;
    if (c[0] == 0) {
      unfused();
      return false;
    }
    segmm_run<T>(ctx, fused, c[0], c[1], fused.batch == 1 && !fused.Zas ? c[2] : 1);
    return true;
  }
  int64_t K = 0;
  for (int q = 0; q < fused.nseg; ++q) K += fused.K[q];
  const TuneKey key{(int64_t)sizeof(T), kind, fused.M, fused.N, K, fused.batch};
  auto it = ctx->tune.find(key);
  if (it == ctx->tune.end()) {
    std::vector<std::array<int, 3>> cand;
    segmm_candidates(fused, cand);
    TuneChoice ch;
    ch.M = fused.M;
    ch.N = fused.N;
    ch.K = (int)K;
    int pick = 0;  // 0: unfused, i > 0: cand[i - 1]
    if (ctx->tune_mode == 2) {
      pick = 1;  // untimed: the fused product on its most split candidate
      for (size_t i = 1; i < cand.size(); ++i)
        if (cand[i][2] > cand[pick - 1][2]) pick = (int)i + 1;
    } else if (ctx->tune_mode == 1) {
      segmm_reserve(ctx, fused, cand);
      std::vector<std::function<void()>> fns{unfused};
      for (const auto& c : cand)
        fns.push_back([&, c] { segmm_run<T>(ctx, fused, c[0], c[1], c[2]); });
      std::vector<double> us;
      pick = time_candidates(ctx, fns, us);
      ch.best_us = us[pick];
      ch.generic_us = us[0];
      if (std::getenv("GFCC_TUNE_LOG")) {
        for (size_t i = 0; i < fns.size(); ++i) {
          if (i == 0) {
            std::fprintf(stderr, "[gfcc autotune] sigma kind %lld M=%d N=%d K=%lld batch=%d "
                         "unfused: %.1f us\n", (long long)kind, fused.M, fused.N, (long long)K,
                         fused.batch, us[0]);
          } else {
            std::fprintf(stderr, "[gfcc autotune] sigma kind %lld tile %dx%d splits=%d: %.1f us\n",
                         (long long)kind, cand[i - 1][0], cand[i - 1][1], cand[i - 1][2], us[i]);
          }
        }
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
    unfused();
    return false;
  }
  segmm_run<T>(ctx, fused, ch.tile_m, ch.tile_n, ch.splits);
  return true;
}

}  // namespace

void ctranspose(gfcc_ctx* ctx, const void* src, int64_t rows, int64_t cols, int64_t lds,
                void* dst, int64_t ldd) {
  if (rows == 0 || cols == 0) return;
  int64_t gy = (rows + 15) / 16, gx = (cols + 15) / 16;
  GFCC_REQUIRE(gy < 65536 && gx < (1LL << 31), GFCC_EINVAL, "ctranspose: shape too large");
  hipLaunchKernelGGL(ctranspose_kernel, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0,
                     ctx->stream, (const double2*)src, rows, cols, lds, (double2*)dst, ldd);
  GFCC_LAUNCH_CHECK();
}

void sigma_block_f64(gfcc_ctx* ctx, int nc, const double* X, double* Y, bool transpose) {
  Operator& op = ctx->op;
  GFCC_REQUIRE(op.built, GFCC_ESTATE, "sigma: no operator built");
  const int o = op.o, v = op.v;
  const int64_t D = op.D, P = op.P, PV = op.PV, OV = op.OV;
  const OpPieces<double>& f = op.f64;
  const double* X1 = X;
  const double* X2 = X + (int64_t)o * nc;
  double* Y1 = Y;
  double* Y2 = Y + (int64_t)o * nc;
  ws_ensure(ctx, ctx->ws_a, sizeof(double) * (size_t)(o + v) * nc);
  ws_ensure(ctx, ctx->ws_b, sizeof(double) * (size_t)OV * o * nc);
  double* S = ctx->ws_a.as<double>();
  double* Z = ctx->ws_b.as<double>();
  hipEvent_t e_all = nullptr, e_ovvo = nullptr;
  timer_begin(ctx, 1, &e_all);
  // Z = Weff . r (the ovvo contraction), then the linear products; the fused 2h1p product, or
  // the Woo product when the pipelined kernel takes it, adds antisym(Z) in its epilogue,
  // otherwise antisym_add_kernel does
  timer_begin(ctx, 0, &e_ovvo);
  gemm_ovvo<double>(ctx, transpose, o, v, nc, f.Weff.as<double>(), X2, nc,
                    op.pairlut.as<int>(), Z);
  timer_end(ctx, 0, e_ovvo);
  GFCC_REQUIRE(PV < (1LL << 31), GFCC_EINVAL, "sigma: too many 2h1p rows");
  bool antisym_done = false;
  if (!transpose) {
    // [sigma_1h ; tau] = [W1 ; 0 | Vp^T] . X: sigma_1h into Y1, tau into S[o:o+v]. Unfused:
    // the whole product into S, then its 1h rows copied to Y1.
    double* tau = S + (int64_t)o * nc;
    SegSpec<double> h;
    h.M = o + v;
    h.N = nc;
    h.K[0] = (int)D;
    h.A[0] = f.W1V.as<double>();
    h.lda[0] = D;
    h.B[0] = X;
    h.ldb[0] = nc;
    h.C = Y1;
    h.C2 = tau;
    h.ldc = nc;
    h.msplit = o;
    tuned_route<double>(ctx, TUNE_SIGMA_1H, h, [&] {
      gemm<double>(ctx, false, false, o + v, nc, (int)D, 1.0, f.W1V.as<double>(), D, X, nc, 0.0,
                   S, nc);
      copy_async<double>(ctx, Y1, S, (int64_t)o * nc);
    });
    // sigma_2h1p's linear part, per virtual index a (rows (pair, a) are v rows apart):
    //   Y2_a = W4c_a[:, :o] . X_1h + W4c_a[:, o:] . tau + Woo . X2_a
    // Unfused: S[0:o] = X_1h, Y2 = W4c . S, then Y2 += (Woo (x) I_v) . X2.
    SegSpec<double> g;
    g.M = (int)P;
    g.N = nc;
    g.batch = v;
    g.nseg = 3;
    g.K[0] = o;
    g.A[0] = f.W4c.as<double>();
    g.lda[0] = (int64_t)v * (o + v);
    g.sA[0] = o + v;
    g.B[0] = X1;
    g.ldb[0] = nc;
    g.K[1] = v;
    g.A[1] = f.W4c.as<double>() + o;
    g.lda[1] = (int64_t)v * (o + v);
    g.sA[1] = o + v;
    g.B[1] = tau;
    g.ldb[1] = nc;
    g.K[2] = (int)P;
    g.A[2] = f.Woo.as<double>();
    g.lda[2] = op.ldwoo;
    g.B[2] = X2;
    g.ldb[2] = (int64_t)v * nc;
    g.sB[2] = nc;
    g.C = Y2;
    g.ldc = (int64_t)v * nc;
    g.sC = nc;
    g.Zas = Z;
    g.as_o = o;
    g.as_v = v;
    g.as_nc = nc;
    // both routes add antisym(Z): the fused one in its epilogue, the unfused one last
    antisym_done = true;
    tuned_route<double>(ctx, TUNE_SIGMA_2H1P, g, [&] {
      copy_async<double>(ctx, S, X1, (int64_t)o * nc);
      gemm<double>(ctx, false, false, (int)PV, nc, o + v, 1.0, f.W4c.as<double>(), o + v, S, nc,
                   0.0, Y2, nc);
      if (!woo_product<double>(ctx, false, P, (int64_t)v * nc, f.Woo.as<double>(), op.ldwoo,
                               X2, Y2, Z, o, v, nc)) {
        hipLaunchKernelGGL(antisym_add_kernel<double>, dim3((unsigned)PV), dim3(256), 0,
                           ctx->stream, Z, o, v, nc, Y2);
        GFCC_LAUNCH_CHECK();
      }
    });
  } else {
    gemm<double>(ctx, true, false, (int)D, nc, o, 1.0, f.W1.as<double>(), D, X1, nc, 0.0, Y, nc);
    gemm<double>(ctx, true, false, o + v, nc, (int)PV, 1.0, f.W4c.as<double>(), o + v, X2, nc,
                 0.0, S, nc);
    hipLaunchKernelGGL(add_kernel<double>, dim3(grid_for((int64_t)o * nc)), dim3(256), 0,
                       ctx->stream, Y1, S, (int64_t)o * nc);
    GFCC_LAUNCH_CHECK();
    gemm<double>(ctx, false, false, (int)PV, nc, v, 1.0, f.Vp.as<double>(), v,
                 S + (int64_t)o * nc, nc, 1.0, Y2, nc);
    antisym_done = woo_product<double>(ctx, true, P, (int64_t)v * nc, f.Woo.as<double>(),
                                       op.ldwoo, X2, Y2, Z, o, v, nc);
  }
  if (!antisym_done) {
    hipLaunchKernelGGL(antisym_add_kernel<double>, dim3((unsigned)PV), dim3(256), 0,
                       ctx->stream, Z, o, v, nc, Y2);
    GFCC_LAUNCH_CHECK();
  }
  timer_end(ctx, 1, e_all);
}

void sigma_block_f32(gfcc_ctx* ctx, int nc, const float* X, float* Y, int precision) {
  Operator& op = ctx->op;
  GFCC_REQUIRE(op.built, GFCC_ESTATE, "sigma: no operator built");
  GFCC_REQUIRE(op.keep & GFCC_KEEP_FP32, GFCC_ESTATE,
               "sigma: FP32 operator copies were not kept at build time");
  const int o = op.o, v = op.v;
  const int64_t D = op.D, P = op.P, PV = op.PV, OV = op.OV;
  const OpPieces<float>& f = op.f32;
  const float* X1 = X;
  const float* X2 = X + (int64_t)o * nc;
  float* Y1 = Y;
  float* Y2 = Y + (int64_t)o * nc;
  ws_ensure(ctx, ctx->ws_a, sizeof(float) * (size_t)(o + v) * nc);
  ws_ensure(ctx, ctx->ws_b, sizeof(float) * (size_t)OV * o * nc);
  float* S = ctx->ws_a.as<float>();
  float* Z = ctx->ws_b.as<float>();
  hipEvent_t e_all = nullptr, e_ovvo = nullptr;
  timer_begin(ctx, 1, &e_all);
  gemm<float>(ctx, false, false, o, nc, (int)D, 1.0f, f.W1.as<float>(), D, X, nc, 0.0f, Y1, nc);
  if (precision != GFCC_FP32_BF16_3BODY) {
    copy_async<float>(ctx, S, X1, (int64_t)o * nc);
    gemm<float>(ctx, true, false, v, nc, (int)PV, 1.0f, f.Vp.as<float>(), v, X2, nc, 0.0f,
                S + (int64_t)o * nc, nc);
    gemm<float>(ctx, false, false, (int)PV, nc, o + v, 1.0f, f.W4c.as<float>(), o + v, S, nc,
                0.0f, Y2, nc);
  } else {
    // three-body term on bf16 matrix cores: tau = Vp^T X2, then Y2 = W4 X1 + (-t2) tau. Both
    // operands of each product are held as hi + lo bf16 pairs (the operator's split once at
    // build time, the vector's on the way into the product) and every block is formed as
    // hi.hi + hi.lo + lo.hi with FP32 accumulation, one launch per product (the lo.lo term is
    // below the FP32 sum's rounding), so the term carries about 16 significant bits instead of
    // bf16's 8, which keeps the refinement's contraction per cycle at the FP32 path's level
    ws_ensure(ctx, ctx->ws_d, sizeof(float) * (size_t)v * nc);
    float* tau = ctx->ws_d.as<float>();
    pairs_gemm(ctx, op.VpT_bf16.p, op.VpT_bf16_lo.p, v, (int)PV, X2, nc, nc, tau, nc, false);
    gemm<float>(ctx, false, false, (int)PV, nc, o, 1.0f, f.W4.as<float>(), o, X1, nc, 0.0f, Y2, nc);
    pairs_gemm(ctx, op.T2p_bf16.p, op.T2p_bf16_lo.p, (int)PV, v, tau, nc, nc, Y2, nc, true);
  }
  // the ovvo contraction before the Woo product, whose epilogue then adds antisym(Z) when the
  // pipelined kernel takes it
  timer_begin(ctx, 0, &e_ovvo);
  hipEvent_t e_bf3 = nullptr;
  timer_begin(ctx, 2, &e_bf3);
  if (precision == GFCC_BF16_PAIRS &&
      ovvo_bf3(ctx, o, v, nc, op.Weff_bf16.p, op.Weff_bf16_lo.p, X2, nc, Z)) {
    timer_end(ctx, 2, e_bf3);
  } else {
    timer_cancel(ctx, e_bf3);
    gemm_ovvo<float>(ctx, false, o, v, nc, f.Weff.as<float>(), X2, nc, op.pairlut.as<int>(), Z);
  }
  timer_end(ctx, 0, e_ovvo);
  GFCC_REQUIRE(PV < (1LL << 31), GFCC_EINVAL, "sigma: too many 2h1p rows");
  if (!woo_product<float>(ctx, false, P, (int64_t)v * nc, f.Woo.as<float>(), op.ldwoo, X2, Y2,
                          Z, o, v, nc)) {
    hipLaunchKernelGGL(antisym_add_kernel<float>, dim3((unsigned)PV), dim3(256), 0,
                       ctx->stream, Z, o, v, nc, Y2);
    GFCC_LAUNCH_CHECK();
  }
  timer_end(ctx, 1, e_all);
}

}  // namespace gfcc

extern "C" gfcc_status sigma_apply(gfcc_ctx* ctx, int nrhs, const void* x, void* y,
                                   int transpose, int precision) {
  if (!ctx) return GFCC_EINVAL;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_REQUIRE(ctx->op.built, GFCC_ESTATE, "sigma_apply: no operator built");
  GFCC_REQUIRE(nrhs >= 0, GFCC_EINVAL, "sigma_apply: nrhs < 0");
  if (nrhs == 0) return GFCC_OK;
  GFCC_REQUIRE(x && y, GFCC_EINVAL, "sigma_apply: null pointer");
  GFCC_REQUIRE(precision >= GFCC_FP64 && precision <= GFCC_BF16_PAIRS, GFCC_EINVAL,
               "sigma_apply: unknown precision");
  GFCC_REQUIRE(!(transpose && precision != GFCC_FP64), GFCC_EINVAL,
               "sigma_apply: the transpose product is FP64 only");
  GFCC_REQUIRE(x != y, GFCC_EINVAL, "sigma_apply: x and y must not overlap");
  const int64_t D = ctx->op.D;
  // chunks of at most 2048 right-hand sides (the solver's largest block)
  constexpr int CH = 2048;
  const int nb = std::min(nrhs, CH);
  // D-major copies of x and y (and their FP32 forms) in a context-owned, grow-only workspace:
  // repeated calls of the same size allocate nothing
  auto up256 = [](size_t n) { return (n + 255) / 256 * 256; };
  const size_t vd = up256(sizeof(double) * (size_t)D * 2 * nb);
  const size_t vf = up256(sizeof(float) * (size_t)D * 2 * nb);
  ws_ensure(ctx, ctx->ws_io, 2 * vd + (precision != GFCC_FP64 ? 2 * vf : 0));
  char* io = ctx->ws_io.as<char>();
  double* bx = reinterpret_cast<double*>(io);
  double* by = reinterpret_cast<double*>(io + vd);
  float* fx = reinterpret_cast<float*>(io + 2 * vd);
  float* fy = reinterpret_cast<float*>(io + 2 * vd + vf);
  const double2* xc = static_cast<const double2*>(x);
  double2* yc = static_cast<double2*>(y);
  for (int r0 = 0; r0 < nrhs; r0 += CH) {
    const int cnt = std::min(CH, nrhs - r0);
    const int nc = 2 * cnt;
    // [cnt][D] complex -> [D][cnt] complex
    ctranspose(ctx, xc + (int64_t)r0 * D, cnt, D, D, bx, cnt);
    if (precision == GFCC_FP64) {
      sigma_block_f64(ctx, nc, bx, by, transpose != 0);
    } else {
      cast_f64_f32(ctx, bx, fx, D * nc);
      sigma_block_f32(ctx, nc, fx, fy, precision);
      cast_f32_f64(ctx, fy, by, D * nc);
    }
    ctranspose(ctx, by, D, cnt, cnt, yc + (int64_t)r0 * D, D);
  }
  GFCC_HIP(hipStreamSynchronize(ctx->stream));
  timers_collect(ctx);
  GFCC_API_END(ctx)
}
