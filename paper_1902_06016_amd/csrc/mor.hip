// Reduced-order model of the GFCC linear system (Methodology: Eq. model and the adaptive
// refinement strategy that follows it).
//
// Basis. S (real, D x m, orthonormal) spans Re X_p(omega_k) and Im X_p(omega_k) for every
// sampled frequency and orbital. Since H-bar_N, b and c are real, a real basis makes
// S^T = S^H, keeps the projected matrix real and preserves interpolation at omega_k. New
// columns are orthogonalised against S by two block passes of classical Gram-Schmidt (matrix
// products), then one by one against the columns accepted in the same round (two passes);
// a column whose norm drops below defl_tol times its original norm is dropped.
// Storage is row-major per basis vector: St[m][D], HSt[m][D] = (H-bar_N S)^T.
//
// Projection. Hhat = S^T H-bar_N S, bhat = S^T b_p, chat = c_q^T S.
// Residual. With F = H-bar_N S - S Hhat (the part of H-bar_N S outside span S) and
// ((omega - i eta) I + Hhat) xhat = bhat, the full-space residual is
//   b - (omega - i eta) S xhat - H-bar_N S xhat = (I - S S^T) b - F xhat,
// so ||r||^2 = ||b||^2 - ||bhat||^2 - 2 Re(f_p^T xhat) + xhat^H (F^T F) xhat, f_p = F^T b_p.
// Evaluation. One workgroup per frequency: complex LU with partial pivoting of
// (omega - i eta) I + Hhat, solves for every orbital, Ghat = chat^T xhat and the residual.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "common.h"

namespace gfcc {
gfcc_status solve_all(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                      double eta, double tol, int maxit, int restart, int block, int precision,
                      int transpose, void* X_out, void* G_out, int* iters_out, double* resid_out);
}

struct gfcc_mor {
  gfcc_ctx* ctx = nullptr;
  int np = 0;
  std::vector<int> p;
  double eta = 0.0, solve_tol = 1e-10, defl_tol = 1e-10;
  int64_t D = 0;
  int m = 0, mcap = 0;
  gfcc::DevBuf St, HSt, Ft, Hhat, Gff, bhat, fvec, chat, bperp2, prows;
  std::vector<double> omega_k;
  int solve_maxit = 2000, solve_restart = 30;
};

namespace gfcc {
namespace {

inline unsigned gridn(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  return (unsigned)(b < 1 ? 1 : b);
}

// W[d][2r] = Re X[r][d], W[d][2r+1] = Im X[r][d]   (X complex [nr][D])
__global__ void split_reim_kernel(const double2* __restrict__ X, int nr, int64_t D,
                                  double* __restrict__ W) {
  const int64_t n = D * nr;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int r = (int)(idx % nr);
    int64_t d = idx / nr;
    double2 x = X[(int64_t)r * D + d];
    W[d * 2 * nr + 2 * r] = x.x;
    W[d * 2 * nr + 2 * r + 1] = x.y;
  }
}

// per-row 2-norms of Wt[n][D]
__global__ void rownorm_kernel(const double* __restrict__ Wt, int64_t D, double* __restrict__ out) {
  __shared__ double red[256];
  const double* w = Wt + (int64_t)blockIdx.x * D;
  double acc = 0.0;
  for (int64_t d = threadIdx.x; d < D; d += blockDim.x) acc += w[d] * w[d];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(red[0]);
}

__global__ void scale_row_kernel(const double* __restrict__ src, int64_t D, double s,
                                 double* __restrict__ dst) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < D;
       d += (int64_t)gridDim.x * blockDim.x)
    dst[d] = src[d] * s;
}

// out[k][i] = Rows[i][p_k]   (Rows is [m][D])
__global__ void gather_cols_kernel(const double* __restrict__ Rows, int m, int64_t D,
                                   const int* __restrict__ p, int np, double* __restrict__ out) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * np) return;
  int k = idx / m, i = idx % m;
  out[idx] = Rows[(int64_t)i * D + p[k]];
}

__global__ void bperp_kernel(const double* __restrict__ bhat, int m, int np, double* __restrict__ out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= np) return;
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += bhat[(int64_t)k * m + i] * bhat[(int64_t)k * m + i];
  out[k] = 1.0 - s;
}

__device__ __forceinline__ double2 cm(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cdv(double2 a, double2 b) {
  double s = fabs(b.x) + fabs(b.y);
  double ar = a.x / s, ai = a.y / s, br = b.x / s, bi = b.y / s;
  double d = br * br + bi * bi;
  return make_double2((ar * br + ai * bi) / d, (ai * br - ar * bi) / d);
}

// One workgroup per frequency. Work space per frequency: A (m x m complex) and Xs (np x m).
__global__ __launch_bounds__(256) void rom_solve_kernel(
    const double* __restrict__ Hhat, const double* __restrict__ bhat,
    const double* __restrict__ chat, const double* __restrict__ Gff,
    const double* __restrict__ fvec, const double* __restrict__ bperp2,
    const double* __restrict__ omega, double eta, int m, int np, int w0, int nw,
    double2* __restrict__ work, double2* __restrict__ G, double* __restrict__ resid) {
  const int wl = blockIdx.x;
  const int w = w0 + wl;
  if (w >= nw) return;
  const int t = threadIdx.x, nt = blockDim.x;
  double2* A = work + (int64_t)wl * ((int64_t)m * m + (int64_t)np * m);
  double2* Xs = A + (int64_t)m * m;
  __shared__ int piv_s;
  __shared__ double red_v[256];
  __shared__ int red_i[256];
  __shared__ double2 red_c[256];
  __shared__ double rmax;
  const double2 z = make_double2(omega[w], -eta);
  for (int64_t e = t; e < (int64_t)m * m; e += nt) {
    int i = (int)(e / m), j = (int)(e % m);
    double h = Hhat[e];
    A[e] = make_double2(h + (i == j ? z.x : 0.0), i == j ? z.y : 0.0);
  }
  for (int64_t e = t; e < (int64_t)np * m; e += nt) Xs[e] = make_double2(bhat[e], 0.0);
  __syncthreads();
  // LU with partial pivoting, applied to the np right-hand sides on the fly
  for (int k = 0; k < m; ++k) {
    double best = -1.0;
    int bi = k;
    for (int i = k + t; i < m; i += nt) {
      double2 a = A[(int64_t)i * m + k];
      double mag = fabs(a.x) + fabs(a.y);
      if (mag > best) { best = mag; bi = i; }
    }
    red_v[t] = best;
    red_i[t] = bi;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (t < s) {
        if (red_v[t + s] > red_v[t] || (red_v[t + s] == red_v[t] && red_i[t + s] < red_i[t])) {
          red_v[t] = red_v[t + s];
          red_i[t] = red_i[t + s];
        }
      }
      __syncthreads();
    }
    if (t == 0) piv_s = red_i[0];
    __syncthreads();
    const int pv = piv_s;
    if (pv != k) {
      for (int j = t; j < m; j += nt) {
        double2 a = A[(int64_t)k * m + j];
        A[(int64_t)k * m + j] = A[(int64_t)pv * m + j];
        A[(int64_t)pv * m + j] = a;
      }
      for (int q = t; q < np; q += nt) {
        double2 a = Xs[(int64_t)q * m + k];
        Xs[(int64_t)q * m + k] = Xs[(int64_t)q * m + pv];
        Xs[(int64_t)q * m + pv] = a;
      }
    }
    __syncthreads();
    const double2 akk = A[(int64_t)k * m + k];
    const int rows = m - k - 1;
    if (rows > 0 && (akk.x != 0.0 || akk.y != 0.0)) {
      for (int i = k + 1 + t; i < m; i += nt) {
        double2 l = cdv(A[(int64_t)i * m + k], akk);
        A[(int64_t)i * m + k] = l;
      }
      __syncthreads();
      const int64_t cols = m - k - 1;
      for (int64_t e = t; e < (int64_t)rows * cols; e += nt) {
        int i = k + 1 + (int)(e / cols), j = k + 1 + (int)(e % cols);
        double2 l = A[(int64_t)i * m + k];
        double2 p = cm(l, A[(int64_t)k * m + j]);
        A[(int64_t)i * m + j].x -= p.x;
        A[(int64_t)i * m + j].y -= p.y;
      }
      for (int64_t e = t; e < (int64_t)rows * np; e += nt) {
        int q = (int)(e / rows), i = k + 1 + (int)(e % rows);
        double2 l = A[(int64_t)i * m + k];
        double2 p = cm(l, Xs[(int64_t)q * m + k]);
        Xs[(int64_t)q * m + i].x -= p.x;
        Xs[(int64_t)q * m + i].y -= p.y;
      }
    }
    __syncthreads();
  }
  // back substitution, one right-hand side per thread group
  for (int q = 0; q < np; ++q) {
    for (int i = m - 1; i >= 0; --i) {
      double2 acc = make_double2(0.0, 0.0);
      for (int j = i + 1 + t; j < m; j += nt) {
        double2 p = cm(A[(int64_t)i * m + j], Xs[(int64_t)q * m + j]);
        acc.x += p.x;
        acc.y += p.y;
      }
      red_c[t] = acc;
      __syncthreads();
      for (int s = nt / 2; s > 0; s >>= 1) {
        if (t < s) { red_c[t].x += red_c[t + s].x; red_c[t].y += red_c[t + s].y; }
        __syncthreads();
      }
      if (t == 0) {
        double2 rhs = Xs[(int64_t)q * m + i];
        rhs.x -= red_c[0].x;
        rhs.y -= red_c[0].y;
        Xs[(int64_t)q * m + i] = cdv(rhs, A[(int64_t)i * m + i]);
      }
      __syncthreads();
    }
  }
  // Ghat[q][p] = chat_q . xhat_p
  for (int e = t; e < np * np; e += nt) {
    int q = e / np, pk = e % np;
    double2 acc = make_double2(0.0, 0.0);
    for (int i = 0; i < m; ++i) {
      double c = chat[(int64_t)q * m + i];
      double2 x = Xs[(int64_t)pk * m + i];
      acc.x += c * x.x;
      acc.y += c * x.y;
    }
    G[((int64_t)w * np + q) * np + pk] = acc;
  }
  // residual: max_p sqrt(bperp2 - 2 Re(f_p . x) + x^H Gff x)
  if (t == 0) rmax = 0.0;
  __syncthreads();
  for (int pk = 0; pk < np; ++pk) {
    double acc = 0.0;
    const double2* x = Xs + (int64_t)pk * m;
    for (int i = t; i < m; i += nt) {
      double2 gx = make_double2(0.0, 0.0);
      for (int j = 0; j < m; ++j) {
        double g = Gff[(int64_t)i * m + j];
        gx.x += g * x[j].x;
        gx.y += g * x[j].y;
      }
      acc += x[i].x * gx.x + x[i].y * gx.y;  // Re(conj(x_i) gx)
      acc -= 2.0 * fvec[(int64_t)pk * m + i] * x[i].x;
    }
    red_v[t] = acc;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (t < s) red_v[t] += red_v[t + s];
      __syncthreads();
    }
    if (t == 0) {
      double r2 = bperp2[pk] + red_v[0];
      double r = sqrt(r2 > 0.0 ? r2 : 0.0);
      rmax = fmax(rmax, r);
    }
    __syncthreads();
  }
  if (t == 0 && resid) resid[w] = rmax;
}

}  // namespace

// Append the real and imaginary parts of the solutions at omega_new to the basis.
static void mor_extend(gfcc_mor* M, const std::vector<double>& omega_new) {
  gfcc_ctx* ctx = M->ctx;
  hipStream_t st = ctx->stream;
  const int64_t D = M->D;
  const int np = M->np, nk = (int)omega_new.size();
  const int nr = nk * np, nn = 2 * nr;
  // full solves
  DevBuf bX, bG;
  bX.alloc(sizeof(double2) * (size_t)nr * D);
  bG.alloc(sizeof(double2) * (size_t)nr * np);
  std::vector<int> its(nr);
  std::vector<double> res(nr);
  gfcc_status s = solve_all(ctx, nk, omega_new.data(), np, M->p.data(), M->eta, M->solve_tol,
                            M->solve_maxit, M->solve_restart, 0, GFCC_FP64, 0, bX.p, bG.p,
                            its.data(), res.data());
  GFCC_REQUIRE(s == GFCC_OK, s, "mor: full solve failed: " + ctx->last_error);
  // new columns, D-major [D][nn]
  DevBuf bW, bWt;
  bW.alloc(sizeof(double) * (size_t)D * nn);
  bWt.alloc(sizeof(double) * (size_t)D * nn);
  double* W = bW.as<double>();
  double* Wt = bWt.as<double>();
  hipLaunchKernelGGL(split_reim_kernel, dim3(gridn(D * nr)), dim3(256), 0, st,
                     bX.as<double2>(), nr, D, W);
  GFCC_LAUNCH_CHECK();
  GFCC_HIP(hipStreamSynchronize(st));
  bX.release();
  // original norms (rows of W^T)
  transpose2d(ctx, W, D, nn, Wt);
  DevBuf bn;
  bn.alloc(sizeof(double) * nn);
  hipLaunchKernelGGL(rownorm_kernel, dim3(nn), dim3(256), 0, st, Wt, D, bn.as<double>());
  GFCC_LAUNCH_CHECK();
  std::vector<double> n0(nn), n1(1);
  GFCC_HIP(hipMemcpyAsync(n0.data(), bn.p, sizeof(double) * nn, hipMemcpyDeviceToHost, st));
  const int m_old = M->m;
  // capacity
  if (m_old + nn > M->mcap) {
    int cap = std::max(M->mcap * 2, m_old + nn);
    DevBuf nS, nHS;
    nS.alloc(sizeof(double) * (size_t)cap * D);
    nHS.alloc(sizeof(double) * (size_t)cap * D);
    if (m_old > 0) {
      GFCC_HIP(hipMemcpyAsync(nS.p, M->St.p, sizeof(double) * (size_t)m_old * D,
                              hipMemcpyDeviceToDevice, st));
      GFCC_HIP(hipMemcpyAsync(nHS.p, M->HSt.p, sizeof(double) * (size_t)m_old * D,
                              hipMemcpyDeviceToDevice, st));
    }
    GFCC_HIP(hipStreamSynchronize(st));
    M->St = std::move(nS);
    M->HSt = std::move(nHS);
    M->mcap = cap;
  }
  double* St = M->St.as<double>();
  // two block passes against the existing basis
  if (m_old > 0) {
    DevBuf bh;
    bh.alloc(sizeof(double) * (size_t)m_old * nn);
    for (int pass = 0; pass < 2; ++pass) {
      gemm<double>(ctx, false, false, m_old, nn, (int)D, 1.0, St, D, W, nn, 0.0, bh.as<double>(), nn);
      gemm<double>(ctx, true, false, (int)D, nn, m_old, -1.0, St, D, bh.as<double>(), nn, 1.0, W, nn);
    }
    GFCC_HIP(hipStreamSynchronize(st));
    transpose2d(ctx, W, D, nn, Wt);
  }
  GFCC_HIP(hipStreamSynchronize(st));
  // one by one against this round's accepted columns
  int m_cur = m_old;
  DevBuf bh;
  bh.alloc(sizeof(double) * (size_t)(nn + 1));
  for (int j = 0; j < nn; ++j) {
    double* wj = Wt + (int64_t)j * D;
    const int acc = m_cur - m_old;
    if (acc > 0) {
      for (int pass = 0; pass < 2; ++pass) {
        gemm<double>(ctx, false, false, acc, 1, (int)D, 1.0, St + (int64_t)m_old * D, D, wj, 1, 0.0,
                     bh.as<double>(), 1);
        gemm<double>(ctx, false, false, 1, (int)D, acc, -1.0, bh.as<double>(), acc,
                     St + (int64_t)m_old * D, D, 1.0, wj, D);
      }
    }
    hipLaunchKernelGGL(rownorm_kernel, dim3(1), dim3(256), 0, st, wj, D, bn.as<double>());
    GFCC_LAUNCH_CHECK();
    GFCC_HIP(hipMemcpyAsync(n1.data(), bn.p, sizeof(double), hipMemcpyDeviceToHost, st));
    GFCC_HIP(hipStreamSynchronize(st));
    if (n0[j] > 0.0 && n1[0] > M->defl_tol * n0[j]) {
      hipLaunchKernelGGL(scale_row_kernel, dim3(gridn(D)), dim3(256), 0, st, wj, D, 1.0 / n1[0],
                         St + (int64_t)m_cur * D);
      GFCC_LAUNCH_CHECK();
      ++m_cur;
    }
  }
  const int nacc = m_cur - m_old;
  if (nacc > 0) {
    // H-bar_N applied to the accepted columns (D-major block through sigma)
    DevBuf bB, bY;
    bB.alloc(sizeof(double) * (size_t)D * nacc);
    bY.alloc(sizeof(double) * (size_t)D * nacc);
    transpose2d(ctx, St + (int64_t)m_old * D, nacc, D, bB.as<double>());
    sigma_block_f64(ctx, nacc, bB.as<double>(), bY.as<double>(), false);
    transpose2d(ctx, bY.as<double>(), D, nacc, M->HSt.as<double>() + (int64_t)m_old * D);
    GFCC_HIP(hipStreamSynchronize(st));
  }
  M->m = m_cur;
  for (double w : omega_new) M->omega_k.push_back(w);
  GFCC_HIP(hipStreamSynchronize(st));
}

// Hhat, F, Gff, bhat, f, chat, ||b_perp||^2 for the current basis.
static void mor_project(gfcc_mor* M) {
  gfcc_ctx* ctx = M->ctx;
  hipStream_t st = ctx->stream;
  const int64_t D = M->D;
  const int m = M->m, np = M->np;
  GFCC_REQUIRE(m > 0, GFCC_EINVAL, "mor: empty basis");
  const double* St = M->St.as<double>();
  const double* HSt = M->HSt.as<double>();
  M->Hhat.alloc(sizeof(double) * (size_t)m * m);
  M->Gff.alloc(sizeof(double) * (size_t)m * m);
  M->Ft.alloc(sizeof(double) * (size_t)m * D);
  M->bhat.alloc(sizeof(double) * (size_t)np * m);
  M->fvec.alloc(sizeof(double) * (size_t)np * m);
  M->chat.alloc(sizeof(double) * (size_t)np * m);
  M->bperp2.alloc(sizeof(double) * (size_t)np);
  // Hhat[i][j] = S_i . (H S)_j
  gemm<double>(ctx, false, true, m, m, (int)D, 1.0, St, D, HSt, D, 0.0, M->Hhat.as<double>(), m);
  // Ft = HSt - Hhat^T St
  GFCC_HIP(hipMemcpyAsync(M->Ft.p, HSt, sizeof(double) * (size_t)m * D, hipMemcpyDeviceToDevice, st));
  gemm<double>(ctx, true, false, m, (int)D, m, -1.0, M->Hhat.as<double>(), m, St, D, 1.0,
               M->Ft.as<double>(), D);
  gemm<double>(ctx, false, true, m, m, (int)D, 1.0, M->Ft.as<double>(), D, M->Ft.as<double>(), D,
               0.0, M->Gff.as<double>(), m);
  hipLaunchKernelGGL(gather_cols_kernel, dim3(blocks_for((int64_t)m * np, 256)), dim3(256), 0, st,
                     St, m, D, M->prows.as<int>(), np, M->bhat.as<double>());
  GFCC_LAUNCH_CHECK();
  hipLaunchKernelGGL(gather_cols_kernel, dim3(blocks_for((int64_t)m * np, 256)), dim3(256), 0, st,
                     M->Ft.as<double>(), m, D, M->prows.as<int>(), np, M->fvec.as<double>());
  GFCC_LAUNCH_CHECK();
  hipLaunchKernelGGL(bperp_kernel, dim3(1), dim3(256), 0, st, M->bhat.as<double>(), m, np,
                     M->bperp2.as<double>());
  GFCC_LAUNCH_CHECK();
  // chat[k][i] = c_{p_k} . S_i
  DevBuf bC;
  bC.alloc(sizeof(double) * (size_t)np * D);
  for (int k = 0; k < np; ++k)
    GFCC_HIP(hipMemcpyAsync(bC.as<double>() + (int64_t)k * D,
                            ctx->op.Crows.as<double>() + (int64_t)M->p[k] * D,
                            sizeof(double) * D, hipMemcpyDeviceToDevice, st));
  gemm<double>(ctx, false, true, np, m, (int)D, 1.0, bC.as<double>(), D, St, D, 0.0,
               M->chat.as<double>(), m);
  GFCC_HIP(hipStreamSynchronize(st));
}

static void mor_eval_impl(gfcc_mor* M, int nw, const double* omega, double2* G, double* resid_host) {
  gfcc_ctx* ctx = M->ctx;
  hipStream_t st = ctx->stream;
  const int m = M->m, np = M->np;
  const int64_t per = (int64_t)m * m + (int64_t)np * m;
  int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nw, (int64_t)(1ULL << 31) / (per * 16)));
  chunk = std::min(chunk, 2048);
  DevBuf bw, bom, bres;
  bw.alloc(sizeof(double2) * (size_t)per * chunk);
  bom.alloc(sizeof(double) * nw);
  bres.alloc(sizeof(double) * nw);
  GFCC_HIP(hipMemcpyAsync(bom.p, omega, sizeof(double) * nw, hipMemcpyHostToDevice, st));
  for (int w0 = 0; w0 < nw; w0 += chunk) {
    int cnt = std::min(chunk, nw - w0);
    hipLaunchKernelGGL(rom_solve_kernel, dim3(cnt), dim3(256), 0, st, M->Hhat.as<double>(),
                       M->bhat.as<double>(), M->chat.as<double>(), M->Gff.as<double>(),
                       M->fvec.as<double>(), M->bperp2.as<double>(), bom.as<double>(), M->eta, m,
                       np, w0, nw, bw.as<double2>(), G, bres.as<double>());
    GFCC_LAUNCH_CHECK();
  }
  if (resid_host)
    GFCC_HIP(hipMemcpyAsync(resid_host, bres.p, sizeof(double) * nw, hipMemcpyDeviceToHost, st));
  GFCC_HIP(hipStreamSynchronize(st));
}

}  // namespace gfcc

extern "C" {

gfcc_status mor_build(gfcc_ctx* ctx, int nk, const double* omega_k, int np, const int* p,
                      double eta, double solve_tol, double defl_tol, gfcc_mor** model) {
  if (!ctx || !model) return GFCC_EINVAL;
  *model = nullptr;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_REQUIRE(ctx->op.built, GFCC_ESTATE, "mor_build: no operator built");
  GFCC_REQUIRE(nk >= 1 && np >= 1 && omega_k && p, GFCC_EINVAL, "mor_build: bad arguments");
  GFCC_REQUIRE(eta > 0.0 && solve_tol > 0.0 && defl_tol >= 0.0, GFCC_EINVAL,
               "mor_build: bad tolerances");
  std::vector<char> seen(ctx->op.o, 0);
  for (int k = 0; k < np; ++k) {
    GFCC_REQUIRE(p[k] >= 0 && p[k] < ctx->op.o && !seen[p[k]], GFCC_EINVAL,
                 "mor_build: p must be distinct occupied orbitals");
    seen[p[k]] = 1;
  }
  for (int k = 0; k < nk; ++k)
    GFCC_REQUIRE(std::isfinite(omega_k[k]), GFCC_EINVAL, "mor_build: non-finite omega");
  auto* M = new gfcc_mor();
  M->ctx = ctx;
  M->np = np;
  M->p.assign(p, p + np);
  M->eta = eta;
  M->solve_tol = solve_tol;
  M->defl_tol = defl_tol;
  M->D = ctx->op.D;
  try {
    M->prows.alloc(sizeof(int) * np);
    GFCC_HIP(hipMemcpy(M->prows.p, p, sizeof(int) * np, hipMemcpyHostToDevice));
    mor_extend(M, std::vector<double>(omega_k, omega_k + nk));
    GFCC_REQUIRE(M->m > 0, GFCC_EINVAL, "mor_build: all basis columns deflated");
    mor_project(M);
  } catch (...) {
    delete M;
    throw;
  }
  *model = M;
  GFCC_API_END(ctx)
}

gfcc_status mor_refine(gfcc_mor* M, int nw, const double* grid, double wmin, double wmax,
                       int per_round, double resid_tol, int max_order, int max_rounds,
                       int* rounds_out, double* max_resid_out) {
  if (!M) return GFCC_EINVAL;
  gfcc_ctx* ctx = M->ctx;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_REQUIRE(nw >= 1 && grid && per_round >= 1 && resid_tol > 0 && max_rounds >= 0 &&
                   wmin <= wmax,
               GFCC_EINVAL, "mor_refine: bad arguments");
  std::vector<double> g;
  for (int i = 0; i < nw; ++i)
    if (grid[i] >= wmin && grid[i] <= wmax) g.push_back(grid[i]);
  GFCC_REQUIRE(!g.empty(), GFCC_EINVAL, "mor_refine: no grid point inside the window");
  std::sort(g.begin(), g.end());
  const int ng = (int)g.size();
  DevBuf bG;
  bG.alloc(sizeof(double2) * (size_t)ng * M->np * M->np);
  std::vector<double> res(ng);
  int rounds = 0;
  double rmax = 0.0;
  for (;;) {
    mor_eval_impl(M, ng, g.data(), bG.as<double2>(), res.data());
    rmax = *std::max_element(res.begin(), res.end());
    if (rmax <= resid_tol || rounds >= max_rounds || M->m >= max_order) break;
    // intervals between adjacent sampled frequencies inside the window
    std::vector<double> ks;
    for (double w : M->omega_k) ks.push_back(w);
    ks.push_back(wmin);
    ks.push_back(wmax);
    std::sort(ks.begin(), ks.end());
    ks.erase(std::unique(ks.begin(), ks.end()), ks.end());
    struct Iv { double lo, hi, e; };
    std::vector<Iv> iv;
    for (size_t i = 0; i + 1 < ks.size(); ++i) {
      double lo = ks[i], hi = ks[i + 1];
      if (hi < wmin || lo > wmax) continue;
      double e = 0.0;
      for (int q = 0; q < ng; ++q)
        if (g[q] >= lo && g[q] <= hi) e = std::max(e, res[q]);
      if (e > resid_tol) iv.push_back({lo, hi, e});
    }
    if (iv.empty()) break;
    std::stable_sort(iv.begin(), iv.end(), [](const Iv& a, const Iv& b) {
      if (a.e != b.e) return a.e > b.e;
      return a.lo < b.lo;
    });
    std::vector<double> add;
    for (size_t i = 0; i < iv.size() && (int)add.size() < per_round; ++i)
      add.push_back(0.5 * (iv[i].lo + iv[i].hi));
    mor_extend(M, add);
    mor_project(M);
    ++rounds;
  }
  if (rounds_out) *rounds_out = rounds;
  if (max_resid_out) *max_resid_out = rmax;
  GFCC_API_END(ctx)
}

gfcc_status mor_eval(gfcc_mor* M, int nw, const double* omega, void* G_out, double* resid_out) {
  if (!M) return GFCC_EINVAL;
  gfcc_ctx* ctx = M->ctx;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_REQUIRE(nw >= 0 && (nw == 0 || (omega && G_out)), GFCC_EINVAL, "mor_eval: bad arguments");
  if (nw == 0) return GFCC_OK;
  for (int i = 0; i < nw; ++i)
    GFCC_REQUIRE(std::isfinite(omega[i]), GFCC_EINVAL, "mor_eval: non-finite omega");
  mor_eval_impl(M, nw, omega, static_cast<double2*>(G_out), resid_out);
  GFCC_API_END(ctx)
}

gfcc_status mor_info(const gfcc_mor* M, int* m_out, int* nk_out, double* omega_k_out, int cap) {
  if (!M) return GFCC_EINVAL;
  if (m_out) *m_out = M->m;
  if (nk_out) *nk_out = (int)M->omega_k.size();
  if (omega_k_out)
    for (int i = 0; i < cap && i < (int)M->omega_k.size(); ++i) omega_k_out[i] = M->omega_k[i];
  return GFCC_OK;
}

gfcc_status mor_destroy(gfcc_mor* M) {
  if (!M) return GFCC_OK;
  (void)hipStreamSynchronize(M->ctx->stream);
  delete M;
  return GFCC_OK;
}

}  // extern "C"
