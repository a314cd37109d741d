// Reduced-order model of the GFCC linear system (Methodology: Eq. model and the adaptive
// refinement strategy that follows it).
//
// Basis. S (real, D x m, orthonormal) spans Re X_p(omega_k) and Im X_p(omega_k) for every
// sampled frequency and orbital. Since H-bar_N, b and c are real, a real basis makes
// S^T = S^H, keeps the projected matrix real and preserves interpolation at omega_k. New
// columns are orthogonalised against S by two block passes of classical Gram-Schmidt (matrix
// products), then one by one against S and the columns accepted in the same round (two
// passes); a column whose norm drops below defl_tol times its original norm is dropped.
// Storage is row-major per basis vector: St[m][D], HSt[m][D] = (H-bar_N S)^T.
//
// Projection. Hhat = S^T H-bar_N S, bhat = S^T b_p, chat = c_q^T S.
// Residual. With F = H-bar_N S - S Hhat (the part of H-bar_N S outside span S) and
// ((omega - i eta) I + Hhat) xhat = bhat, the full-space residual is
//   b - (omega - i eta) S xhat - H-bar_N S xhat = (I - S S^T) b - F xhat.
// With F = Q R (Q orthonormal, orthogonal to S) this splits into orthogonal pieces,
//   ||r||^2 = ||(I - S S^T - Q Q^T) b||^2 + ||Q^T b - R xhat||^2,
// a sum of squares: the first term is formed once from an explicit vector, the second is a
// short vector per frequency, so neither cancels as the residual becomes small.
// Evaluation. One workgroup per frequency: complex LU with partial pivoting of
// (omega - i eta) I + Hhat, solves for every orbital, Ghat = chat^T xhat and the residual.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>

#include "common.h"

struct gfcc_mor {
  gfcc_ctx* ctx = nullptr;
  int np = 0;
  std::vector<int> p;
  double eta = 0.0, solve_tol = 1e-10, defl_tol = 1e-10;
  int64_t D = 0;
  int m = 0, mcap = 0;
  gfcc::DevBuf St, HSt, Hhat, bhat, chat, prows;
  gfcc::DevBuf Qt, Rm, beta, cnst;  // QR of F = H S - S Hhat, Q^T b_p, ||(I - SS^T - QQ^T) b_p||^2
  int r = 0;                        // rank of F
  std::vector<double> omega_k;
  int solve_maxit = 2000, solve_restart = 30;
  gfcc::DevBuf ews, eom, eres;  // evaluation work arrays, kept between calls
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

// R0[k][d] = (d == p_k)
__global__ void unit_rows_kernel(const int* __restrict__ p, int np, int64_t D, double* __restrict__ R0) {
  const int64_t n = (int64_t)np * D;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int k = (int)(idx / D);
    int64_t d = idx - (int64_t)k * D;
    R0[idx] = (d == p[k]) ? 1.0 : 0.0;
  }
}

__global__ void square_kernel(double* __restrict__ a, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = a[i] * a[i];
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
    const double* __restrict__ chat, const double* __restrict__ Rm,
    const double* __restrict__ beta, const double* __restrict__ cnst, int rk,
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
  // residual: max_p sqrt(cnst_p + ||beta_p - R xhat_p||^2)
  if (t == 0) rmax = 0.0;
  __syncthreads();
  for (int pk = 0; pk < np; ++pk) {
    double acc = 0.0;
    const double2* x = Xs + (int64_t)pk * m;
    for (int i = t; i < rk; i += nt) {
      double2 rx = make_double2(0.0, 0.0);
      const double* Ri = Rm + (int64_t)i * m;
      for (int j = 0; j < m; ++j) {
        rx.x += Ri[j] * x[j].x;
        rx.y += Ri[j] * x[j].y;
      }
      double dr = beta[(int64_t)pk * (rk > 0 ? rk : 1) + i] - rx.x, di = -rx.y;
      acc += dr * dr + di * di;
    }
    red_v[t] = acc;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (t < s) red_v[t] += red_v[t + s];
      __syncthreads();
    }
    if (t == 0) rmax = fmax(rmax, sqrt(cnst[pk] + red_v[0]));
    __syncthreads();
  }
  if (t == 0 && resid) resid[w] = rmax;
}

// The same solve with one wavefront per frequency and the matrix and right-hand sides in LDS
// (dynamic, (m^2 + np m) complex entries, at most ROM_LDS_MAX bytes): the pivot search is a
// wavefront reduction and the back substitution runs column by column for all orbitals at
// once, so no step waits on other wavefronts. Only the solutions go to the work buffer (at
// the offset rom_solve_kernel uses, for lift_kernel).
constexpr int ROM_LDS_MAX = 65536;

__global__ __launch_bounds__(64) void rom_solve_wave_kernel(
    const double* __restrict__ Hhat, const double* __restrict__ bhat,
    const double* __restrict__ chat, const double* __restrict__ Rm,
    const double* __restrict__ beta, const double* __restrict__ cnst, int rk,
    const double* __restrict__ omega, double eta, int m, int np, int w0, int nw,
    double2* __restrict__ work, double2* __restrict__ G, double* __restrict__ resid) {
  extern __shared__ double2 rom_lds[];
  const int wl = blockIdx.x;
  const int w = w0 + wl;
  if (w >= nw) return;
  const int t = threadIdx.x;
  double2* A = rom_lds;
  double2* Xs = rom_lds + (int64_t)m * m;
  const double2 z = make_double2(omega[w], -eta);
  for (int e = t; e < m * m; e += 64) {
    const int i = e / m, j = e - (e / m) * m;
    A[e] = make_double2(Hhat[e] + (i == j ? z.x : 0.0), i == j ? z.y : 0.0);
  }
  for (int e = t; e < np * m; e += 64) Xs[e] = make_double2(bhat[e], 0.0);
  __syncthreads();
  const int ti = t / 8, tj = t % 8;  // 8 x 8 lane grid for the trailing update
  for (int k = 0; k < m; ++k) {
    // partial pivoting: largest |re| + |im| in column k, the smallest row among equals
    double best = -1.0;
    int bi = k;
    for (int i = k + t; i < m; i += 64) {
      const double2 a = A[i * m + k];
      const double mag = fabs(a.x) + fabs(a.y);
      if (mag > best) { best = mag; bi = i; }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oi = __shfl_xor(bi, off);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const int pv = __shfl(bi, 0);
    if (pv != k) {
      for (int j = t; j < m; j += 64) {
        const double2 a = A[k * m + j];
        A[k * m + j] = A[pv * m + j];
        A[pv * m + j] = a;
      }
      for (int q = t; q < np; q += 64) {
        const double2 a = Xs[q * m + k];
        Xs[q * m + k] = Xs[q * m + pv];
        Xs[q * m + pv] = a;
      }
    }
    __syncthreads();
    const double2 akk = A[k * m + k];
    if (k + 1 < m && (akk.x != 0.0 || akk.y != 0.0)) {
      for (int i = k + 1 + t; i < m; i += 64) A[i * m + k] = cdv(A[i * m + k], akk);
      __syncthreads();
      for (int i = k + 1 + ti; i < m; i += 8) {
        const double2 l = A[i * m + k];
        for (int j = k + 1 + tj; j < m; j += 8) {
          const double2 p = cm(l, A[k * m + j]);
          A[i * m + j].x -= p.x;
          A[i * m + j].y -= p.y;
        }
      }
      for (int q = ti; q < np; q += 8) {
        const double2 xk = Xs[q * m + k];
        for (int i = k + 1 + tj; i < m; i += 8) {
          const double2 p = cm(A[i * m + k], xk);
          Xs[q * m + i].x -= p.x;
          Xs[q * m + i].y -= p.y;
        }
      }
    }
    __syncthreads();
  }
  // back substitution, column by column, every orbital at once
  for (int i = m - 1; i >= 0; --i) {
    const double2 aii = A[i * m + i];
    for (int q = t; q < np; q += 64) Xs[q * m + i] = cdv(Xs[q * m + i], aii);
    __syncthreads();
    for (int q = ti; q < np; q += 8) {
      const double2 xi = Xs[q * m + i];
      for (int r = tj; r < i; r += 8) {
        const double2 p = cm(A[r * m + i], xi);
        Xs[q * m + r].x -= p.x;
        Xs[q * m + r].y -= p.y;
      }
    }
    __syncthreads();
  }
  // Ghat[q][p] = chat_q . xhat_p
  for (int e = t; e < np * np; e += 64) {
    const int q = e / np, pk = e - (e / np) * np;
    double2 acc = make_double2(0.0, 0.0);
    for (int i = 0; i < m; ++i) {
      const double c = chat[(int64_t)q * m + i];
      const double2 x = Xs[pk * m + i];
      acc.x += c * x.x;
      acc.y += c * x.y;
    }
    G[((int64_t)w * np + q) * np + pk] = acc;
  }
  // residual: max_p sqrt(cnst_p + ||beta_p - R xhat_p||^2)
  double rmax = 0.0;
  for (int pk = 0; pk < np; ++pk) {
    double acc = 0.0;
    const double2* x = Xs + pk * m;
    for (int i = t; i < rk; i += 64) {
      double2 rx = make_double2(0.0, 0.0);
      const double* Ri = Rm + (int64_t)i * m;
      for (int j = 0; j < m; ++j) {
        rx.x += Ri[j] * x[j].x;
        rx.y += Ri[j] * x[j].y;
      }
      const double dr = beta[(int64_t)pk * (rk > 0 ? rk : 1) + i] - rx.x, di = -rx.y;
      acc += dr * dr + di * di;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    rmax = fmax(rmax, sqrt(cnst[pk] + __shfl(acc, 0)));
  }
  if (t == 0 && resid) resid[w] = rmax;
  double2* xo = work + (int64_t)wl * ((int64_t)m * m + (int64_t)np * m) + (int64_t)m * m;
  for (int e = t; e < np * m; e += 64) xo[e] = Xs[e];
}

// X[(w0 + wl) np + q][d] = sum_i xhat_wl,q[i] St[i][d] for the cnt frequencies of a chunk,
// xhat read from rom_solve_kernel's work buffer (the m solution entries follow the m x m
// factor of each frequency). Grid (ceil(D / 256), ceil(cnt np / LR)); LR rows per thread.
constexpr int LR = 8;
__global__ __launch_bounds__(256) void lift_kernel(const double* __restrict__ St, int64_t D, int m,
                                                   int np, const double2* __restrict__ work,
                                                   int64_t per, int cnt, int w0,
                                                   double2* __restrict__ X) {
  const int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (d >= D) return;
  const int rows = cnt * np;
  const int row0 = blockIdx.y * LR;
  double2 acc[LR];
#pragma unroll
  for (int r = 0; r < LR; ++r) acc[r] = make_double2(0.0, 0.0);
  for (int i = 0; i < m; ++i) {
    const double s = St[(int64_t)i * D + d];
#pragma unroll
    for (int r = 0; r < LR; ++r) {
      const int row = row0 + r;
      if (row < rows) {
        const int wl = row / np, q = row - wl * np;
        const double2 xh = work[(int64_t)wl * per + (int64_t)m * m + (int64_t)q * m + i];
        acc[r].x += xh.x * s;
        acc[r].y += xh.y * s;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < LR; ++r) {
    const int row = row0 + r;
    if (row < rows) X[((int64_t)w0 * np + row) * D + d] = acc[r];
  }
}

// ---- row-by-row Gram-Schmidt on the device (orth_rows). The projection set is the nb fixed
// rows B followed by the acc rows accepted so far (Out); acc lives in device memory, so the
// loop over rows needs no host round trip.
struct OrthState {
  int acc;     // rows accepted so far
  int slot;    // index in Out of the row being decided
  int take;    // 1 if that row is accepted
  int pad;
  double inv;  // 1 / its norm
};

constexpr int ODR = 8;        // projection rows per dots workgroup
constexpr int OSL = 4096;     // elements of D per dots slice

__device__ __forceinline__ const double* orth_row(const double* B, int nb, const double* Out,
                                                  int64_t D, int i) {
  return i < nb ? B + (int64_t)i * D : Out + (int64_t)(i - nb) * D;
}

// sum of v over the 256 threads of the workgroup in a fixed order (wave shuffles, then the
// four wave sums in turn); the result is valid in every thread
__device__ __forceinline__ double orth_block_sum(double v, double* red4) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if (threadIdx.x % 64 == 0) red4[threadIdx.x / 64] = v;
  __syncthreads();
  return ((red4[0] + red4[1]) + red4[2]) + red4[3];
}

// partial[s][i] = sum over slice s of Q_i[d] w[d] for the rows i in
// [blockIdx.y ODR, blockIdx.y ODR + ODR) below nb + acc. Grid (ceil(D / OSL), ceil(kmax / ODR)).
__global__ __launch_bounds__(256) void orth_dots_kernel(const double* __restrict__ B, int nb,
                                                        const double* __restrict__ Out,
                                                        const OrthState* __restrict__ stt,
                                                        const double* __restrict__ w, int64_t D,
                                                        int kmax, double* __restrict__ partial) {
  __shared__ double red4[4];
  const int k = nb + stt->acc;
  const int row0 = blockIdx.y * ODR;
  if (row0 >= k) return;
  const int64_t d0 = (int64_t)blockIdx.x * OSL;
  const int64_t d1 = min(D, d0 + (int64_t)OSL);
  const double* q[ODR];
#pragma unroll
  for (int r = 0; r < ODR; ++r) q[r] = orth_row(B, nb, Out, D, min(row0 + r, k - 1));
  double acc[ODR];
#pragma unroll
  for (int r = 0; r < ODR; ++r) acc[r] = 0.0;
  for (int64_t d = d0 + threadIdx.x; d < d1; d += 256) {
    const double x = w[d];
#pragma unroll
    for (int r = 0; r < ODR; ++r) acc[r] += q[r][d] * x;
  }
#pragma unroll
  for (int r = 0; r < ODR; ++r) {
    const double t = orth_block_sum(acc[r], red4);
    if (threadIdx.x == 0 && row0 + r < k) partial[(int64_t)blockIdx.x * kmax + row0 + r] = t;
  }
}

// h[i] = sum_s partial[s][i] for i < nb + acc; coefficients along the accepted rows are
// accumulated into coef_row[i - nb]. Grid ceil(kmax / 64), 256 threads: lane r of wavefront g
// sums the slices g, g + 4, ... of row i = 64 blockIdx.x + r (independent loads), and the four
// wavefront sums are added in a fixed order.
__global__ __launch_bounds__(256) void orth_reduce_kernel(const double* __restrict__ partial,
                                                          int nsl, int kmax,
                                                          const OrthState* __restrict__ stt,
                                                          int nb, double* __restrict__ h,
                                                          double* __restrict__ coef_row) {
  __shared__ double red[4][64];
  const int k = nb + stt->acc;
  const int r = threadIdx.x % 64, g = threadIdx.x / 64;
  const int i = blockIdx.x * 64 + r;
  double s0 = 0.0, s1 = 0.0;
  if (i < k) {
    int sl = g;
    for (; sl + 4 < nsl; sl += 8) {
      s0 += partial[(int64_t)sl * kmax + i];
      s1 += partial[(int64_t)(sl + 4) * kmax + i];
    }
    for (; sl < nsl; sl += 4) s0 += partial[(int64_t)sl * kmax + i];
  }
  red[g][r] = s0 + s1;
  __syncthreads();
  if (g == 0 && i < k) {
    const double s = ((red[0][r] + red[1][r]) + red[2][r]) + red[3][r];
    h[i] = s;
    if (coef_row && i >= nb) coef_row[i - nb] += s;
  }
}

// w[d] -= sum_{i < nb + acc} h[i] Q_i[d]; with nrm_part, the workgroup's partial sum of w[d]^2
// after the update. Grid ceil(D / 256), one element per thread.
__global__ __launch_bounds__(256) void orth_update_kernel(const double* __restrict__ B, int nb,
                                                          const double* __restrict__ Out,
                                                          const OrthState* __restrict__ stt,
                                                          const double* __restrict__ h,
                                                          double* __restrict__ w, int64_t D,
                                                          double* __restrict__ nrm_part) {
  __shared__ double red4[4];
  const int k = nb + stt->acc;
  const int64_t d = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double ss = 0.0;
  if (d < D) {
    double x = w[d];
    for (int i = 0; i < min(k, nb); ++i) x -= h[i] * B[(int64_t)i * D + d];
    for (int i = nb; i < k; ++i) x -= h[i] * Out[(int64_t)(i - nb) * D + d];
    w[d] = x;
    ss = x * x;
  }
  if (nrm_part) {
    const double t = orth_block_sum(ss, red4);
    if (threadIdx.x == 0) nrm_part[blockIdx.x] = t;
  }
}

// norm of the row from the update's partial sums; accept it if it exceeds thresh (its norm
// becomes the coefficient along its own accepted row). One workgroup.
__global__ __launch_bounds__(256) void orth_accept_kernel(const double* __restrict__ nrm_part,
                                                          int npart, double thresh,
                                                          OrthState* __restrict__ stt,
                                                          double* __restrict__ coef_row) {
  __shared__ double red4[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < npart; b += 256) s += nrm_part[b];
  const double nrm = sqrt(orth_block_sum(s, red4));
  if (threadIdx.x == 0) {
    const int acc = stt->acc;
    const int take = (nrm > 0.0 && nrm > thresh) ? 1 : 0;
    stt->slot = acc;
    stt->take = take;
    stt->inv = take ? 1.0 / nrm : 0.0;
    if (take) {
      if (coef_row) coef_row[acc] = nrm;
      stt->acc = acc + 1;
    }
  }
}

// Out[slot] = w / ||w|| for an accepted row
__global__ void orth_store_kernel(const OrthState* __restrict__ stt, const double* __restrict__ w,
                                  int64_t D, double* __restrict__ Out) {
  if (!stt->take) return;
  const double s = stt->inv;
  double* o = Out + (int64_t)stt->slot * D;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < D;
       d += (int64_t)gridDim.x * blockDim.x)
    o[d] = w[d] * s;
}

}  // namespace

// Orthogonalise the rows W[0..n) ([n][D], overwritten) against the fixed orthonormal rows
// B[0..nb) by two block passes of classical Gram-Schmidt, then one by one (two passes each,
// every pass classical Gram-Schmidt against B and the rows accepted so far together; accepted
// rows are written to Out). Projecting each pass on B as well keeps accepted rows orthogonal
// to B even when a row's remainder is many orders of magnitude below its original norm. Row j
// is accepted when its norm after orthogonalisation exceeds thresh[j]. If coef is given ([ldc]
// per row j), it receives the coefficients of row j along the accepted Out rows (the norm for
// its own row). The row loop runs on the device (the count of accepted rows stays in device
// memory), with one synchronisation at the end. Returns the number of accepted rows.
static int orth_rows(gfcc_ctx* ctx, int64_t D, const double* B, int nb, double* W, int n,
                     double* Out, const std::vector<double>& thresh, std::vector<double>* coef,
                     int ldc) {
  hipStream_t st = ctx->stream;
  if (n == 0) return 0;
  DevBuf bblk;  // freed after the final synchronisation, like every buffer below
  if (nb > 0) {
    bblk.alloc(sizeof(double) * (size_t)nb * n);
    for (int pass = 0; pass < 2; ++pass) {
      gemm<double>(ctx, false, true, nb, n, (int)D, 1.0, B, D, W, D, 0.0, bblk.as<double>(), n);
      gemm<double>(ctx, true, false, n, (int)D, nb, -1.0, bblk.as<double>(), n, B, D, 1.0, W, D);
    }
  }
  const int kmax = nb + n;
  const int nsl = (int)((D + OSL - 1) / OSL);
  const unsigned nupd = (unsigned)((D + 255) / 256);
  GFCC_REQUIRE(nupd < (1u << 31), GFCC_EINVAL, "orth_rows: D too large");
  DevBuf bstate, bpart, bh, bnrm, bcoef;
  bstate.alloc(sizeof(OrthState));
  bpart.alloc(sizeof(double) * (size_t)nsl * kmax);
  bh.alloc(sizeof(double) * (size_t)kmax);
  bnrm.alloc(sizeof(double) * nupd);
  OrthState s0{};
  GFCC_HIP(hipMemcpyAsync(bstate.p, &s0, sizeof(OrthState), hipMemcpyHostToDevice, st));
  if (coef) {
    coef->assign((size_t)n * ldc, 0.0);
    bcoef.alloc(sizeof(double) * coef->size());
    GFCC_HIP(hipMemcpyAsync(bcoef.p, coef->data(), sizeof(double) * coef->size(),
                            hipMemcpyHostToDevice, st));
  }
  OrthState* stt = bstate.as<OrthState>();
  for (int j = 0; j < n; ++j) {
    double* wj = W + (int64_t)j * D;
    double* crow = coef ? bcoef.as<double>() + (size_t)j * ldc : nullptr;
    const int kj = nb + j;  // bound on nb + acc before row j
    for (int pass = 0; pass < 2; ++pass) {
      if (kj > 0) {
        hipLaunchKernelGGL(orth_dots_kernel, dim3(nsl, (kj + ODR - 1) / ODR), dim3(256), 0, st, B,
                           nb, Out, stt, wj, D, kmax, bpart.as<double>());
        GFCC_LAUNCH_CHECK();
        hipLaunchKernelGGL(orth_reduce_kernel, dim3((kj + 63) / 64), dim3(256), 0, st,
                           bpart.as<double>(), nsl, kmax, stt, nb, bh.as<double>(), crow);
        GFCC_LAUNCH_CHECK();
      }
      if (kj > 0 || pass == 1) {
        hipLaunchKernelGGL(orth_update_kernel, dim3(nupd), dim3(256), 0, st, B, nb, Out, stt,
                           bh.as<double>(), wj, D, pass == 1 ? bnrm.as<double>() : nullptr);
        GFCC_LAUNCH_CHECK();
      }
    }
    hipLaunchKernelGGL(orth_accept_kernel, dim3(1), dim3(256), 0, st, bnrm.as<double>(),
                       (int)nupd, thresh[j], stt, crow);
    GFCC_LAUNCH_CHECK();
    hipLaunchKernelGGL(orth_store_kernel, dim3(gridn(D)), dim3(256), 0, st, stt, wj, D, Out);
    GFCC_LAUNCH_CHECK();
  }
  OrthState sf{};
  GFCC_HIP(hipMemcpyAsync(&sf, bstate.p, sizeof(OrthState), hipMemcpyDeviceToHost, st));
  if (coef)
    GFCC_HIP(hipMemcpyAsync(coef->data(), bcoef.p, sizeof(double) * coef->size(),
                            hipMemcpyDeviceToHost, st));
  GFCC_HIP(hipStreamSynchronize(st));
  return sf.acc;
}

// Append the real and imaginary parts of nr full solutions X [nr][D] (device, complex; the
// solutions at omega_new for the model's orbitals) to the basis.
static void mor_add(gfcc_mor* M, const double2* X, int nr, const std::vector<double>& omega_new) {
  gfcc_ctx* ctx = M->ctx;
  hipStream_t st = ctx->stream;
  const int64_t D = M->D;
  const int nn = 2 * nr;
  // new columns, D-major [D][nn]
  DevBuf bW, bWt;
  bW.alloc(sizeof(double) * (size_t)D * nn);
  bWt.alloc(sizeof(double) * (size_t)D * nn);
  double* W = bW.as<double>();
  double* Wt = bWt.as<double>();
  hipLaunchKernelGGL(split_reim_kernel, dim3(gridn(D * nr)), dim3(256), 0, st, X, nr, D, W);
  GFCC_LAUNCH_CHECK();
  GFCC_HIP(hipStreamSynchronize(st));
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
  transpose2d(ctx, W, D, nn, Wt);
  std::vector<double> n0(nn);
  DevBuf bn;
  bn.alloc(sizeof(double) * nn);
  hipLaunchKernelGGL(rownorm_kernel, dim3(nn), dim3(256), 0, st, Wt, D, bn.as<double>());
  GFCC_LAUNCH_CHECK();
  GFCC_HIP(hipMemcpyAsync(n0.data(), bn.p, sizeof(double) * nn, hipMemcpyDeviceToHost, st));
  GFCC_HIP(hipStreamSynchronize(st));
  std::vector<double> thresh(nn);
  for (int j = 0; j < nn; ++j) thresh[j] = M->defl_tol * n0[j];
  const int nacc_rows = orth_rows(ctx, D, St, m_old, Wt, nn, St + (int64_t)m_old * D, thresh,
                                  nullptr, 0);
  const int m_cur = m_old + nacc_rows;
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

// Full solves at omega_new for the model's orbitals, appended to the basis.
static void mor_extend(gfcc_mor* M, const std::vector<double>& omega_new) {
  gfcc_ctx* ctx = M->ctx;
  const int64_t D = M->D;
  const int np = M->np, nk = (int)omega_new.size();
  const int nr = nk * np;
  DevBuf bX, bG;
  bX.alloc(sizeof(double2) * (size_t)nr * D);
  bG.alloc(sizeof(double2) * (size_t)nr * np);
  std::vector<int> its(nr);
  std::vector<double> res(nr);
  gfcc_status s = solve_all(ctx, nk, omega_new.data(), np, M->p.data(), M->eta, M->solve_tol,
                            M->solve_maxit, M->solve_restart, 0, GFCC_FP64, 0, bX.p, bG.p,
                            its.data(), res.data(), nullptr);
  GFCC_REQUIRE(s == GFCC_OK, s, "mor: full solve failed: " + ctx->last_error);
  mor_add(M, bX.as<double2>(), nr, omega_new);
}

// Hhat, bhat, chat and the residual factors (Q, R, Q^T b, constant term) for the current basis.
static void mor_project(gfcc_mor* M) {
  gfcc_ctx* ctx = M->ctx;
  hipStream_t st = ctx->stream;
  const int64_t D = M->D;
  const int m = M->m, np = M->np;
  GFCC_REQUIRE(m > 0, GFCC_EINVAL, "mor: empty basis");
  const double* St = M->St.as<double>();
  const double* HSt = M->HSt.as<double>();
  M->Hhat.alloc(sizeof(double) * (size_t)m * m);
  M->bhat.alloc(sizeof(double) * (size_t)np * m);
  M->chat.alloc(sizeof(double) * (size_t)np * m);
  // Hhat[i][j] = S_i . (H S)_j
  gemm<double>(ctx, false, true, m, m, (int)D, 1.0, St, D, HSt, D, 0.0, M->Hhat.as<double>(), m);
  // F rows: Ft = HSt - Hhat^T St
  DevBuf bF, bnrm;
  bF.alloc(sizeof(double) * (size_t)m * D);
  double* Ft = bF.as<double>();
  GFCC_HIP(hipMemcpyAsync(Ft, HSt, sizeof(double) * (size_t)m * D, hipMemcpyDeviceToDevice, st));
  gemm<double>(ctx, true, false, m, (int)D, m, -1.0, M->Hhat.as<double>(), m, St, D, 1.0, Ft, D);
  // F = Q R: a row of F whose part outside span{S, earlier Q} is below
  // max(1e-10 ||F_j||, 1e-13 ||(H S)_j||) is rounding-level and adds no direction (its R
  // column has no diagonal entry)
  bnrm.alloc(sizeof(double) * 2 * m);
  hipLaunchKernelGGL(rownorm_kernel, dim3(m), dim3(256), 0, st, HSt, D, bnrm.as<double>());
  GFCC_LAUNCH_CHECK();
  hipLaunchKernelGGL(rownorm_kernel, dim3(m), dim3(256), 0, st, Ft, D, bnrm.as<double>() + m);
  GFCC_LAUNCH_CHECK();
  std::vector<double> hsn(2 * m), thresh(m);
  GFCC_HIP(hipMemcpyAsync(hsn.data(), bnrm.p, sizeof(double) * 2 * m, hipMemcpyDeviceToHost, st));
  GFCC_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < m; ++j) thresh[j] = std::max(1e-10 * hsn[m + j], 1e-13 * hsn[j]);
  M->Qt.alloc(sizeof(double) * (size_t)m * D);
  std::vector<double> coef;
  const int r = orth_rows(ctx, D, St, m, Ft, m, M->Qt.as<double>(), thresh, &coef, m);
  M->r = r;
  // R[i][j] = coefficient of F_j along Q_i
  std::vector<double> R((size_t)std::max(r, 1) * m, 0.0);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < r; ++i) R[(size_t)i * m + j] = coef[(size_t)j * m + i];
  M->Rm.alloc(sizeof(double) * R.size());
  GFCC_HIP(hipMemcpyAsync(M->Rm.p, R.data(), sizeof(double) * R.size(), hipMemcpyHostToDevice, st));
  // bhat[k][i] = S_i[p_k], beta[k][i] = Q_i[p_k]
  hipLaunchKernelGGL(gather_cols_kernel, dim3(blocks_for((int64_t)m * np, 256)), dim3(256), 0, st,
                     St, m, D, M->prows.as<int>(), np, M->bhat.as<double>());
  GFCC_LAUNCH_CHECK();
  M->beta.alloc(sizeof(double) * (size_t)np * std::max(r, 1));
  if (r > 0) {
    hipLaunchKernelGGL(gather_cols_kernel, dim3(blocks_for((int64_t)r * np, 256)), dim3(256), 0,
                       st, M->Qt.as<double>(), r, D, M->prows.as<int>(), np, M->beta.as<double>());
    GFCC_LAUNCH_CHECK();
  }
  // constant term: || e_p - S bhat_p - Q beta_p ||^2, from the explicit vector
  DevBuf bR0;
  bR0.alloc(sizeof(double) * (size_t)np * D);
  double* R0 = bR0.as<double>();
  hipLaunchKernelGGL(unit_rows_kernel, dim3(gridn((int64_t)np * D)), dim3(256), 0, st,
                     M->prows.as<int>(), np, D, R0);
  GFCC_LAUNCH_CHECK();
  gemm<double>(ctx, false, false, np, (int)D, m, -1.0, M->bhat.as<double>(), m, St, D, 1.0, R0, D);
  if (r > 0)
    gemm<double>(ctx, false, false, np, (int)D, r, -1.0, M->beta.as<double>(), r,
                 M->Qt.as<double>(), D, 1.0, R0, D);
  M->cnst.alloc(sizeof(double) * np);
  hipLaunchKernelGGL(rownorm_kernel, dim3(np), dim3(256), 0, st, R0, D, M->cnst.as<double>());
  GFCC_LAUNCH_CHECK();
  hipLaunchKernelGGL(square_kernel, dim3(1), dim3(256), 0, st, M->cnst.as<double>(), np);
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

// Solves of the reduced system at omega[w0 .. w0 + cnt) (work, G and resid as in
// rom_solve_kernel): one wavefront per frequency with the matrix in LDS when it fits, else
// one workgroup per frequency on the work buffer.
static void rom_solve(gfcc_mor* M, const double* omega, int w0, int cnt, int nw, double2* work,
                      double2* G, double* resid) {
  hipStream_t st = M->ctx->stream;
  const int m = M->m, np = M->np;
  const int64_t lds = ((int64_t)m * m + (int64_t)np * m) * (int64_t)sizeof(double2);
  if (lds <= ROM_LDS_MAX) {
    hipLaunchKernelGGL(rom_solve_wave_kernel, dim3(cnt), dim3(64), (unsigned)lds, st,
                       M->Hhat.as<double>(), M->bhat.as<double>(), M->chat.as<double>(),
                       M->Rm.as<double>(), M->beta.as<double>(), M->cnst.as<double>(), M->r, omega,
                       M->eta, m, np, w0, nw, work, G, resid);
  } else {
    hipLaunchKernelGGL(rom_solve_kernel, dim3(cnt), dim3(256), 0, st, M->Hhat.as<double>(),
                       M->bhat.as<double>(), M->chat.as<double>(), M->Rm.as<double>(),
                       M->beta.as<double>(), M->cnst.as<double>(), M->r, omega, M->eta, m, np, w0,
                       nw, work, G, resid);
  }
  GFCC_LAUNCH_CHECK();
}

static void mor_eval_impl(gfcc_mor* M, int nw, const double* omega, double2* G, double* resid_host) {
  gfcc_ctx* ctx = M->ctx;
  hipStream_t st = ctx->stream;
  const int m = M->m, np = M->np;
  const int64_t per = (int64_t)m * m + (int64_t)np * m;
  int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nw, (int64_t)(1ULL << 31) / (per * 16)));
  chunk = std::min(chunk, 2048);
  M->ews.ensure(sizeof(double2) * (size_t)per * chunk);
  M->eom.ensure(sizeof(double) * nw);
  M->eres.ensure(sizeof(double) * nw);
  GFCC_HIP(hipMemcpyAsync(M->eom.p, omega, sizeof(double) * nw, hipMemcpyHostToDevice, st));
  for (int w0 = 0; w0 < nw; w0 += chunk) {
    int cnt = std::min(chunk, nw - w0);
    rom_solve(M, M->eom.as<double>(), w0, cnt, nw, M->ews.as<double2>(), G, M->eres.as<double>());
  }
  if (resid_host)
    GFCC_HIP(hipMemcpyAsync(resid_host, M->eres.p, sizeof(double) * nw, hipMemcpyDeviceToHost, st));
  GFCC_HIP(hipStreamSynchronize(st));
}

static void mor_lift_impl(gfcc_mor* M, int nw, const double* omega, double2* X) {
  gfcc_ctx* ctx = M->ctx;
  hipStream_t st = ctx->stream;
  const int m = M->m, np = M->np;
  const int64_t D = M->D;
  const int64_t per = (int64_t)m * m + (int64_t)np * m;
  int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nw, (int64_t)(1ULL << 31) / (per * 16)));
  chunk = std::min(chunk, 2048);
  DevBuf bw, bom, bres, bG;
  bw.alloc(sizeof(double2) * (size_t)per * chunk);
  bom.alloc(sizeof(double) * nw);
  bres.alloc(sizeof(double) * nw);
  bG.alloc(sizeof(double2) * (size_t)nw * np * np);
  GFCC_HIP(hipMemcpyAsync(bom.p, omega, sizeof(double) * nw, hipMemcpyHostToDevice, st));
  for (int w0 = 0; w0 < nw; w0 += chunk) {
    const int cnt = std::min(chunk, nw - w0);
    rom_solve(M, bom.as<double>(), w0, cnt, nw, bw.as<double2>(), bG.as<double2>(),
              bres.as<double>());
    const int64_t gy = ((int64_t)cnt * np + LR - 1) / LR;
    GFCC_REQUIRE(gy < 65536, GFCC_EINVAL, "mor_lift: too many frequencies x orbitals per chunk");
    hipLaunchKernelGGL(lift_kernel, dim3((unsigned)((D + 255) / 256), (unsigned)gy), dim3(256), 0,
                       st, M->St.as<double>(), D, m, np, bw.as<double2>(), per, cnt, w0, X);
    GFCC_LAUNCH_CHECK();
  }
  GFCC_HIP(hipStreamSynchronize(st));
}

// ------------------------------------------------------------------------------------------
// Evaluation without allocation (mor_eval_noalloc). The reduced solves of a chunk of
// frequencies need per-frequency work space (the shifted m x m matrix and the solutions), the
// frequencies on the device and the residuals; here they live in one file-scope device array
// of EVAL_SCRATCH_BYTES. Each device holds its own copy; its address is looked up once per
// device (eval_scratch_setup, called by gfcc_create with the device current) and only that
// address is used on the host. Calls on one device share the array: calls that overlap in
// time on one device race.
constexpr size_t EVAL_SCRATCH_BYTES = (size_t)32 << 20;
constexpr int EVAL_MAX_DEVICES = 64;

}  // namespace gfcc

static __device__ __align__(256) unsigned char scratch[gfcc::EVAL_SCRATCH_BYTES];

namespace gfcc {

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[EVAL_MAX_DEVICES];

void eval_scratch_setup(int device) {
  GFCC_REQUIRE(device >= 0 && device < EVAL_MAX_DEVICES, GFCC_EINVAL,
               "gfcc_create: device index beyond the evaluation scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* ptr = nullptr;
  GFCC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  GFCC_REQUIRE(ptr != nullptr, GFCC_EHIP, "gfcc_create: no address for the evaluation scratch");
  g_scratch_ptr[device] = ptr;
}

static char* eval_scratch(int device) {
  if (device < 0 || device >= EVAL_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return static_cast<char*>(g_scratch_ptr[device]);
}

// mor_eval on the scratch array: chunks of as many frequencies as fit, each with its
// frequencies copied in, the reduced solves (the kernels of mor_eval) and its residuals copied
// out. No device memory is allocated or freed.
static void mor_eval_scratch(gfcc_mor* M, int nw, const double* omega, double2* G,
                             double* resid_host) {
  gfcc_ctx* ctx = M->ctx;
  hipStream_t st = ctx->stream;
  const int m = M->m, np = M->np;
  char* base = eval_scratch(ctx->device);
  GFCC_REQUIRE(base != nullptr, GFCC_ESTATE,
               "mor_eval_noalloc: no evaluation scratch on this device");
  const size_t per = sizeof(double2) * ((size_t)m * m + (size_t)np * m);
  auto up = [](size_t n) { return (n + 255) / 256 * 256; };
  // omega and resid take 8 bytes per frequency each, rounded up to 256 bytes
  const size_t avail = EVAL_SCRATCH_BYTES - 2 * 256;
  GFCC_REQUIRE(per + 16 <= avail, GFCC_ENOMEM,
               "mor_eval_noalloc: a model of order " + std::to_string(m) + " with " +
                   std::to_string(np) + " orbitals needs " + std::to_string(per) +
                   " bytes per frequency; the evaluation scratch holds " +
                   std::to_string(EVAL_SCRATCH_BYTES) + " bytes");
  int chunk = (int)std::min<size_t>(avail / (per + 16), 2048);
  chunk = std::min(chunk, nw);
  double* om = reinterpret_cast<double*>(base);
  double* res = reinterpret_cast<double*>(base + up(sizeof(double) * chunk));
  double2* work = reinterpret_cast<double2*>(base + 2 * up(sizeof(double) * chunk));
  for (int w0 = 0; w0 < nw; w0 += chunk) {
    const int cnt = std::min(chunk, nw - w0);
    GFCC_HIP(hipMemcpyAsync(om, omega + w0, sizeof(double) * cnt, hipMemcpyHostToDevice, st));
    rom_solve(M, om, 0, cnt, cnt, work, G + (int64_t)w0 * np * np, res);
    if (resid_host)
      GFCC_HIP(hipMemcpyAsync(resid_host + w0, res, sizeof(double) * cnt,
                              hipMemcpyDeviceToHost, st));
  }
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

gfcc_status mor_build_diag(gfcc_ctx* ctx, int nk, const double* omega_k, int np, const int* p,
                           double eta, double solve_tol, double defl_tol, gfcc_mor** models) {
  if (!ctx || !models) return GFCC_EINVAL;
  for (int k = 0; k < np; ++k) models[k] = nullptr;
  std::vector<gfcc_mor*> made;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_REQUIRE(ctx->op.built, GFCC_ESTATE, "mor_build_diag: no operator built");
  GFCC_REQUIRE(nk >= 1 && np >= 1 && omega_k && p, GFCC_EINVAL, "mor_build_diag: bad arguments");
  GFCC_REQUIRE(eta > 0.0 && solve_tol > 0.0 && defl_tol >= 0.0, GFCC_EINVAL,
               "mor_build_diag: bad tolerances");
  std::vector<char> seen(ctx->op.o, 0);
  for (int k = 0; k < np; ++k) {
    GFCC_REQUIRE(p[k] >= 0 && p[k] < ctx->op.o && !seen[p[k]], GFCC_EINVAL,
                 "mor_build_diag: p must be distinct occupied orbitals");
    seen[p[k]] = 1;
  }
  for (int k = 0; k < nk; ++k)
    GFCC_REQUIRE(std::isfinite(omega_k[k]), GFCC_EINVAL, "mor_build_diag: non-finite omega");
  const int64_t D = ctx->op.D;
  hipStream_t st = ctx->stream;
  const std::vector<double> om(omega_k, omega_k + nk);
  try {
    // one set of full solves for every (omega_k, p) ...
    DevBuf bX, bG, bXk;
    bX.alloc(sizeof(double2) * (size_t)nk * np * D);
    bG.alloc(sizeof(double2) * (size_t)nk * np * np);
    bXk.alloc(sizeof(double2) * (size_t)nk * D);
    std::vector<int> its((size_t)nk * np);
    std::vector<double> res((size_t)nk * np);
    gfcc_status s = solve_all(ctx, nk, omega_k, np, p, eta, solve_tol, 2000, 30, 0, GFCC_FP64, 0,
                              bX.p, bG.p, its.data(), res.data(), nullptr);
    GFCC_REQUIRE(s == GFCC_OK, s, "mor_build_diag: full solve failed: " + ctx->last_error);
    // ... then one model per orbital from its own solutions
    for (int k = 0; k < np; ++k) {
      auto* M = new gfcc_mor();
      made.push_back(M);
      M->ctx = ctx;
      M->np = 1;
      M->p.assign(1, p[k]);
      M->eta = eta;
      M->solve_tol = solve_tol;
      M->defl_tol = defl_tol;
      M->D = D;
      M->prows.alloc(sizeof(int));
      GFCC_HIP(hipMemcpy(M->prows.p, p + k, sizeof(int), hipMemcpyHostToDevice));
      for (int w = 0; w < nk; ++w)
        GFCC_HIP(hipMemcpyAsync(bXk.as<double2>() + (int64_t)w * D,
                                bX.as<double2>() + ((int64_t)w * np + k) * D,
                                sizeof(double2) * D, hipMemcpyDeviceToDevice, st));
      mor_add(M, bXk.as<double2>(), nk, om);
      GFCC_REQUIRE(M->m > 0, GFCC_EINVAL, "mor_build_diag: all basis columns deflated");
      mor_project(M);
    }
  } catch (...) {
    for (gfcc_mor* M : made) delete M;
    throw;
  }
  for (int k = 0; k < np; ++k) models[k] = made[k];
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

gfcc_status mor_eval_noalloc(gfcc_mor* M, int nw, const double* omega, void* G_out,
                             double* resid_out) {
  if (!M) return GFCC_EINVAL;
  gfcc_ctx* ctx = M->ctx;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_REQUIRE(nw >= 0 && (nw == 0 || (omega && G_out)), GFCC_EINVAL,
               "mor_eval_noalloc: bad arguments");
  if (nw == 0) return GFCC_OK;
  GFCC_REQUIRE(M->m > 0, GFCC_ESTATE, "mor_eval_noalloc: empty model");
  for (int i = 0; i < nw; ++i)
    GFCC_REQUIRE(std::isfinite(omega[i]), GFCC_EINVAL, "mor_eval_noalloc: non-finite omega");
  mor_eval_scratch(M, nw, omega, static_cast<double2*>(G_out), resid_out);
  GFCC_API_END(ctx)
}

gfcc_status mor_lift(gfcc_mor* M, int nw, const double* omega, void* X_out) {
  if (!M) return GFCC_EINVAL;
  gfcc_ctx* ctx = M->ctx;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_REQUIRE(nw >= 0 && (nw == 0 || (omega && X_out)), GFCC_EINVAL, "mor_lift: bad arguments");
  if (nw == 0) return GFCC_OK;
  GFCC_REQUIRE(M->m > 0, GFCC_ESTATE, "mor_lift: empty model");
  for (int i = 0; i < nw; ++i)
    GFCC_REQUIRE(std::isfinite(omega[i]), GFCC_EINVAL, "mor_lift: non-finite omega");
  mor_lift_impl(M, nw, omega, static_cast<double2*>(X_out));
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
