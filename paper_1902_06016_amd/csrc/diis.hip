// Complex DIIS solver for the shifted GFCC systems (Eq. xplin), the linear solver of the
// paper's convergence study (Results, Fig. 3: DIIS carried over to complex vectors with 10
// micro-iteration iterates).
//
// Periodic DIIS, one right-hand side per column of a block [D][nb]:
//   micro-iteration  e_k = P^{-1} (b - M x_k),  x_{k+1} = x_k + e_k,
//                    P = diag(M), M = (omega - i eta) I + Hbar_N;
//   after m steps    x <- sum_k c_k x_{k+1}, with the complex c minimising ||sum_k c_k e_k||
//                    subject to sum_k c_k = 1, and the subspace starts afresh.
// The true relative residual ||b - M x|| / ||b|| is formed before every micro-iteration and
// is the stopping test.
//
// The minimum is taken in its unconstrained form: with gamma_k = sum_{j<=k} c_j,
//   sum_k c_k e_k = e_{m-1} - F gamma,   F = [e_1 - e_0, ..., e_{m-1} - e_{m-2}],
//   sum_k c_k x_{k+1} = x_m - sum_k gamma_k e_{k+1},
// and gamma = R^{-1} Q^H e_{m-1} from a QR factorisation of F that grows by one column per
// micro-iteration (classical Gram-Schmidt applied twice, as in the GMRES Arnoldi). Forming
// the Gram matrix e_i^H e_j of Pulay's bordered system instead would square the condition
// number of the error vectors, which become nearly parallel as the iteration settles.
//
// Per micro-iteration: one FP64 sigma product of the block; a residual sweep (B, X, S in, R
// out, column norms); a step sweep (e into slot k, X += e, the new difference and its first
// projections); two Gram-Schmidt sweeps and a scaling sweep for the new column of Q.
#include <algorithm>
#include <cmath>

#include "blockvec.h"

namespace gfcc {
namespace {

// R = B - z X - S (has_x == 0: R = B), and per-column partial sums of |R|^2.
// Grid (nblk, ceil(nb / 64)), one wavefront per block, one lane per right-hand side.
__global__ __launch_bounds__(CW) void diis_resid_kernel(const double2* __restrict__ B,
                                                        const double2* __restrict__ X,
                                                        const double2* __restrict__ S,
                                                        const double2* __restrict__ z, int has_x,
                                                        int64_t D, int nb,
                                                        double2* __restrict__ R,
                                                        double* __restrict__ partial) {
  const int r = blockIdx.y * CW + threadIdx.x;
  if (r >= nb) return;
  const int64_t rows = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows;
  const int64_t d1 = min(D, d0 + rows);
  const double2 zz = z[r];
  double acc = 0.0;
#pragma unroll 4
  for (int64_t d = d0; d < d1; ++d) {
    const int64_t idx = d * nb + r;
    double2 v = B[idx];
    if (has_x) {
      const double2 p = cmul(zz, X[idx]);
      const double2 s = S[idx];
      v.x -= s.x + p.x;
      v.y -= s.y + p.y;
    }
    R[idx] = v;
    acc += v.x * v.x + v.y * v.y;
  }
  partial[(int64_t)blockIdx.x * nb + r] = acc;
}

// Micro-iteration k of a cycle. Slot k of E holds the residual R on entry and
// e = R / (diag + z) on exit (zero for inactive columns); X += e. For k >= 1 the new
// difference d = e_k - e_{k-1} goes to column j = k - 1 of Q (unnormalised), with
// partial[blk][i][r] = sum conj(Q_i) d over the block's rows, i < j.
// Grid (nblk, ceil(nb / 64)), one lane per right-hand side.
__global__ __launch_bounds__(CW) void diis_step_kernel(double2* __restrict__ E,
                                                       double2* __restrict__ Q, int64_t vs,
                                                       int k, const double* __restrict__ diag,
                                                       const double2* __restrict__ z,
                                                       const int* __restrict__ active,
                                                       int64_t D, int nb,
                                                       double2* __restrict__ X,
                                                       double2* __restrict__ partial) {
  const int r = blockIdx.y * CW + threadIdx.x;
  if (r >= nb) return;
  const int j = k - 1;
  double2 acc[JG];
#pragma unroll
  for (int i = 0; i < JG; ++i) acc[i] = make_double2(0.0, 0.0);
  const bool act = active[r] != 0;
  const double2 zz = z[r];
  double2* __restrict__ Ek = E + (int64_t)k * vs;
  const int64_t rows = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows;
  const int64_t d1 = min(D, d0 + rows);
#pragma unroll 2
  for (int64_t d = d0; d < d1; ++d) {
    const int64_t idx = d * nb + r;
    double2 e = make_double2(0.0, 0.0);
    if (act) {
      e = cdiv(Ek[idx], make_double2(diag[d] + zz.x, zz.y));
      const double2 x = X[idx];
      X[idx] = make_double2(x.x + e.x, x.y + e.y);
    }
    Ek[idx] = e;
    if (j >= 0) {
      double2 df = make_double2(0.0, 0.0);
      if (act) {
        const double2 ep = E[(int64_t)j * vs + idx];
        df = make_double2(e.x - ep.x, e.y - ep.y);
      }
      Q[(int64_t)j * vs + idx] = df;
#pragma unroll
      for (int i = 0; i < JG; ++i) {
        if (i < j) {
          const double2 p = cconjmul(Q[(int64_t)i * vs + idx], df);
          acc[i].x += p.x;
          acc[i].y += p.y;
        }
      }
    }
  }
  double2* out = partial + (int64_t)blockIdx.x * JG * nb + r;
#pragma unroll
  for (int i = 0; i < JG; ++i)
    if (i < j) out[(int64_t)i * nb] = acc[i];
}

// One Gram-Schmidt pass on column j of Q: d = Q_j - sum_{i<j} Q_i h_i, stored back; then
// either the projections partial_h[blk][i][r] = sum conj(Q_i) d (i < j, dots != 0) or
// partial_n[blk][r] = sum |d|^2. Same grid as diis_step_kernel.
__global__ __launch_bounds__(CW) void diis_orth_kernel(double2* __restrict__ Q, int64_t vs,
                                                       int j, const double2* __restrict__ h,
                                                       int dots, int64_t D, int nb,
                                                       double2* __restrict__ partial_h,
                                                       double* __restrict__ partial_n) {
  const int r = blockIdx.y * CW + threadIdx.x;
  if (r >= nb) return;
  double2 hc[JG], acc[JG];
#pragma unroll
  for (int i = 0; i < JG; ++i) {
    hc[i] = i < j ? h[(int64_t)i * nb + r] : make_double2(0.0, 0.0);
    acc[i] = make_double2(0.0, 0.0);
  }
  double nacc = 0.0;
  double2* __restrict__ Qj = Q + (int64_t)j * vs;
  const int64_t rows = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows;
  const int64_t d1 = min(D, d0 + rows);
  for (int64_t d = d0; d < d1; ++d) {
    const int64_t idx = d * nb + r;
    double2 q[JG];
    double2 df = Qj[idx];
#pragma unroll
    for (int i = 0; i < JG; ++i) {
      if (i < j) {
        q[i] = Q[(int64_t)i * vs + idx];
        const double2 p = cmul(q[i], hc[i]);
        df.x -= p.x;
        df.y -= p.y;
      }
    }
    Qj[idx] = df;
    if (dots) {
#pragma unroll
      for (int i = 0; i < JG; ++i) {
        if (i < j) {
          const double2 p = cconjmul(q[i], df);
          acc[i].x += p.x;
          acc[i].y += p.y;
        }
      }
    } else {
      nacc += df.x * df.x + df.y * df.y;
    }
  }
  if (dots) {
    double2* out = partial_h + (int64_t)blockIdx.x * JG * nb + r;
#pragma unroll
    for (int i = 0; i < JG; ++i)
      if (i < j) out[(int64_t)i * nb] = acc[i];
  } else {
    partial_n[(int64_t)blockIdx.x * nb + r] = nacc;
  }
}

// Column j of R (mm x mm per right-hand side, Rm[i][j][r]): h1 + h2 above the diagonal, the
// norm on it; inv[r] = 1 / norm (0 for a zero column). One thread per right-hand side.
__global__ void diis_rcol_kernel(const double2* __restrict__ h1, const double2* __restrict__ h2,
                                 const double* __restrict__ nrm, int j, int mm, int nb,
                                 double2* __restrict__ Rm, double* __restrict__ inv) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb) return;
  for (int i = 0; i < j; ++i) {
    const double2 a = h1[(int64_t)i * nb + r], b = h2[(int64_t)i * nb + r];
    Rm[((int64_t)i * mm + j) * nb + r] = make_double2(a.x + b.x, a.y + b.y);
  }
  const double nu = nrm[r];
  Rm[((int64_t)j * mm + j) * nb + r] = make_double2(nu, 0.0);
  inv[r] = nu > 0.0 ? 1.0 / nu : 0.0;
}

// V[d][r] *= inv[r]
__global__ void diis_scale_kernel(double2* __restrict__ V, const double* __restrict__ inv,
                                  int64_t D, int nb) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const double s = inv[idx % nb];
    V[idx] = make_double2(V[idx].x * s, V[idx].y * s);
  }
}

// partial[blk][i][r] = sum conj(Q_i) V over the block's rows, i < nq (same grid as above)
__global__ __launch_bounds__(CW) void diis_proj_kernel(const double2* __restrict__ Q, int64_t vs,
                                                       int nq, const double2* __restrict__ V,
                                                       int64_t D, int nb,
                                                       double2* __restrict__ partial) {
  const int r = blockIdx.y * CW + threadIdx.x;
  if (r >= nb) return;
  double2 acc[JG];
#pragma unroll
  for (int i = 0; i < JG; ++i) acc[i] = make_double2(0.0, 0.0);
  const int64_t rows = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows;
  const int64_t d1 = min(D, d0 + rows);
#pragma unroll 2
  for (int64_t d = d0; d < d1; ++d) {
    const int64_t idx = d * nb + r;
    const double2 v = V[idx];
#pragma unroll
    for (int i = 0; i < JG; ++i) {
      if (i < nq) {
        const double2 p = cconjmul(Q[(int64_t)i * vs + idx], v);
        acc[i].x += p.x;
        acc[i].y += p.y;
      }
    }
  }
  double2* out = partial + (int64_t)blockIdx.x * JG * nb + r;
#pragma unroll
  for (int i = 0; i < JG; ++i)
    if (i < nq) out[(int64_t)i * nb] = acc[i];
}

// gamma = R^{-1} g by back substitution (a zero diagonal entry drops its direction), then
// coef[0] = 0 and coef[k + 1] = -gamma_k, so that X += sum_j coef_j E_j turns the latest
// iterate into the DIIS combination. Inactive columns get coef = 0. One thread per column;
// gam is scratch [mm][nb].
__global__ void diis_gamma_kernel(const double2* __restrict__ Rm, const double2* __restrict__ g,
                                  int mm, int nb, const int* __restrict__ active,
                                  double2* __restrict__ gam, double2* __restrict__ coef) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb) return;
  const bool act = active[r] != 0;
  for (int i = mm - 1; i >= 0; --i) {
    double2 t = g[(int64_t)i * nb + r];
    for (int l = i + 1; l < mm; ++l) {
      const double2 p = cmul(Rm[((int64_t)i * mm + l) * nb + r], gam[(int64_t)l * nb + r]);
      t.x -= p.x;
      t.y -= p.y;
    }
    const double2 dg = Rm[((int64_t)i * mm + i) * nb + r];
    gam[(int64_t)i * nb + r] =
        (act && (dg.x != 0.0 || dg.y != 0.0)) ? cdiv(t, dg) : make_double2(0.0, 0.0);
  }
  coef[r] = make_double2(0.0, 0.0);
  for (int k = 0; k < mm; ++k) {
    const double2 v = gam[(int64_t)k * nb + r];
    coef[(int64_t)(k + 1) * nb + r] = make_double2(-v.x, -v.y);
  }
}

// X[d][r] += sum_{j=1}^{m-1} coef[j][r] E_j[d][r]   (coef_0 is zero)
__global__ void diis_extrap_kernel(const double2* __restrict__ E, int64_t estride, int m,
                                   const double2* __restrict__ coef, int64_t D, int nb,
                                   double2* __restrict__ X) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    double2 x = X[idx];
    for (int j = 1; j < m; ++j) {
      const double2 p = cmul(coef[(int64_t)j * nb + r], E[(int64_t)j * estride + idx]);
      x.x += p.x;
      x.y += p.y;
    }
    X[idx] = x;
  }
}

}  // namespace

const void* diis_block(gfcc_ctx* ctx, DiisWork& wk, int nb, int m, const double* omega,
                       const int* pset, int np, int nrhs, int r0, double eta, double tol,
                       int maxit, bool transpose, int* its_out, double* res_out, double* hist,
                       const void* X0) {
  GFCC_REQUIRE(m >= 1 && m <= JG, GFCC_EINVAL, "diis: iterates per extrapolation in [1, 16]");
  const int64_t D = ctx->op.D;
  const int64_t vec = D * nb;
  hipStream_t st = ctx->stream;
  const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, vec / 4096));
  const int ncb = (nb + CW - 1) / CW;
  const int mm = std::max(m - 1, 1);  // columns of Q and R
  int64_t bytes = 0;
  auto add = [&](int64_t cnt, int64_t sz) { bytes += ((cnt * sz + 255) / 256) * 256; };
  add(vec * m, 16);                          // E
  add(vec * mm, 16);                         // Q
  for (int i = 0; i < 3; ++i) add(vec, 16);  // X B S
  add((int64_t)nblk * JG * nb, 16);          // part_h
  add((int64_t)nblk * nb, 8);                // part_n
  for (int i = 0; i < 3; ++i) add((int64_t)JG * nb, 16);  // h1 h2 g
  add((int64_t)mm * mm * nb, 16);            // Rm
  add((int64_t)mm * nb, 16);                 // gam
  add((int64_t)m * nb, 16);                  // coef
  add(nb, 16);                               // z
  add(nb, 8); add(nb, 8);                    // nrm inv
  add(nb, 4); add(nb, 4);                    // prow act
  ws_ensure(ctx, wk.mem, (size_t)bytes);
  char* cur = wk.mem.as<char>();
  double2* E = carve<double2>(cur, vec * m);
  double2* Q = carve<double2>(cur, vec * mm);
  double2* X = carve<double2>(cur, vec);
  double2* B = carve<double2>(cur, vec);
  double2* S = carve<double2>(cur, vec);
  double2* part_h = carve<double2>(cur, (int64_t)nblk * JG * nb);
  double* part_n = carve<double>(cur, (int64_t)nblk * nb);
  double2* h1 = carve<double2>(cur, (int64_t)JG * nb);
  double2* h2 = carve<double2>(cur, (int64_t)JG * nb);
  double2* g = carve<double2>(cur, (int64_t)JG * nb);
  double2* Rm = carve<double2>(cur, (int64_t)mm * mm * nb);
  double2* gam = carve<double2>(cur, (int64_t)mm * nb);
  double2* coef = carve<double2>(cur, (int64_t)m * nb);
  double2* z = carve<double2>(cur, nb);
  double* nrm = carve<double>(cur, nb);
  double* inv = carve<double>(cur, nb);
  int* prow = carve<int>(cur, nb);
  int* actd = carve<int>(cur, nb);

  std::vector<double2> hz(nb);
  std::vector<int> hp(nb);
  for (int r = 0; r < nb; ++r) {
    const int gr = r0 + r;
    if (gr < nrhs) {
      hz[r] = make_double2(omega[gr / np], -eta);
      hp[r] = pset[gr % np];
    } else {
      hz[r] = make_double2(1.0, -eta);  // padding column: b = 0, done at once
      hp[r] = -1;
    }
  }
  GFCC_HIP(hipMemcpyAsync(z, hz.data(), sizeof(double2) * nb, hipMemcpyHostToDevice, st));
  GFCC_HIP(hipMemcpyAsync(prow, hp.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
  solve_rhs(ctx, prow, transpose, D, nb, B);
  const dim3 rgrid(nblk, ncb);
  const dim3 cgrid(blocks_for(nb, 64));
  // ||b|| per column (slot 0 of E serves as scratch)
  hipLaunchKernelGGL(diis_resid_kernel, rgrid, dim3(CW), 0, st, B, X, S, z, 0, D, nb, E, part_n);
  GFCC_LAUNCH_CHECK();
  hipLaunchKernelGGL(norm_reduce, dim3(ncb), dim3(256), 0, st, part_n, nblk, nb, nrm);
  GFCC_LAUNCH_CHECK();
  std::vector<double> bnorm(nb), rn(nb);
  GFCC_HIP(hipMemcpyAsync(bnorm.data(), nrm, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  fill(ctx, reinterpret_cast<double*>(X), vec * 2, 0.0);
  if (X0) {
    const int cnt = std::min(nb, nrhs - r0);
    ctranspose(ctx, static_cast<const double2*>(X0) + (int64_t)r0 * D, cnt, D, D, X, nb);
  }
  GFCC_HIP(hipStreamSynchronize(st));

  const int64_t hs = (int64_t)maxit + 1;
  std::vector<int> its(nb, 0), done(nb, 0), act(nb, 0);
  std::vector<double> rel(nb, 0.0);
  for (int r = 0; r < nb; ++r) {
    const int gr = r0 + r;
    if (hist && gr < nrhs) std::fill(hist + gr * hs, hist + (gr + 1) * hs, -1.0);
    if (bnorm[r] == 0.0) {
      done[r] = 1;
      if (hist && gr < nrhs) hist[gr * hs] = 0.0;
    }
  }
  bool xzero = X0 == nullptr;
  // forward from x = 0: the first step gives x = e_p / P_pp, whose product is a column of Hbar_N
  bool xunit = false;
  int k = 0;
  for (;;) {
    // ---- residual of the current iterate, into slot k
    if (xunit)
      unit_sigma(ctx, prow, z, nb, S);
    else if (!xzero)
      sigma_block_f64(ctx, 2 * nb, reinterpret_cast<const double*>(X),
                      reinterpret_cast<double*>(S), transpose);
    xunit = xzero && !transpose;
    hipLaunchKernelGGL(diis_resid_kernel, rgrid, dim3(CW), 0, st, B, X, S, z, xzero ? 0 : 1, D,
                       nb, E + (int64_t)k * vec, part_n);
    GFCC_LAUNCH_CHECK();
    hipLaunchKernelGGL(norm_reduce, dim3(ncb), dim3(256), 0, st, part_n, nblk, nb, nrm);
    GFCC_LAUNCH_CHECK();
    GFCC_HIP(hipMemcpyAsync(rn.data(), nrm, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    GFCC_HIP(hipStreamSynchronize(st));
    int nact = 0;
    for (int r = 0; r < nb; ++r) {
      act[r] = 0;
      if (done[r]) continue;
      const int gr = r0 + r;
      const double rl = rn[r] / bnorm[r];
      if (hist && gr < nrhs) hist[gr * hs + its[r]] = rl;
      if (rl <= tol || its[r] >= maxit || !std::isfinite(rl)) {
        done[r] = 1;
        rel[r] = rl;
      } else {
        act[r] = 1;
        ++nact;
      }
    }
    if (nact == 0) break;
    // ---- Jacobi step; the new difference of error vectors becomes column j of Q (CGS2)
    GFCC_HIP(hipMemcpyAsync(actd, act.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(diis_step_kernel, rgrid, dim3(CW), 0, st, E, Q, vec, k,
                       ctx->op.diag.as<double>(), z, actd, D, nb, X, part_h);
    GFCC_LAUNCH_CHECK();
    const int j = k - 1;
    if (j >= 0) {
      if (j > 0) {
        hipLaunchKernelGGL(dots_reduce_s<JG>, dim3(ncb, j), dim3(256), 0, st, part_h, nblk, 0, j, nb,
                           h1);
        GFCC_LAUNCH_CHECK();
        hipLaunchKernelGGL(diis_orth_kernel, rgrid, dim3(CW), 0, st, Q, vec, j, h1, 1, D, nb,
                           part_h, part_n);
        GFCC_LAUNCH_CHECK();
        hipLaunchKernelGGL(dots_reduce_s<JG>, dim3(ncb, j), dim3(256), 0, st, part_h, nblk, 0, j, nb,
                           h2);
        GFCC_LAUNCH_CHECK();
      }
      hipLaunchKernelGGL(diis_orth_kernel, rgrid, dim3(CW), 0, st, Q, vec, j, h2, 0, D, nb,
                         part_h, part_n);
      GFCC_LAUNCH_CHECK();
      hipLaunchKernelGGL(norm_reduce, dim3(ncb), dim3(256), 0, st, part_n, nblk, nb, nrm);
      GFCC_LAUNCH_CHECK();
      hipLaunchKernelGGL(diis_rcol_kernel, cgrid, dim3(64), 0, st, h1, h2, nrm, j, mm, nb, Rm,
                         inv);
      GFCC_LAUNCH_CHECK();
      hipLaunchKernelGGL(diis_scale_kernel, dim3(gridn(vec)), dim3(256), 0, st,
                         Q + (int64_t)j * vec, inv, D, nb);
      GFCC_LAUNCH_CHECK();
    }
    for (int r = 0; r < nb; ++r) its[r] += act[r];
    xzero = false;
    if (++k == m) {
      // ---- extrapolation: gamma = R^{-1} Q^H e_{m-1}, X = x_m - sum_k gamma_k e_{k+1}
      if (m > 1) {
        hipLaunchKernelGGL(diis_proj_kernel, rgrid, dim3(CW), 0, st, Q, vec, m - 1,
                           E + (int64_t)(m - 1) * vec, D, nb, part_h);
        GFCC_LAUNCH_CHECK();
        hipLaunchKernelGGL(dots_reduce_s<JG>, dim3(ncb, m - 1), dim3(256), 0, st, part_h, nblk, 0,
                           m - 1, nb, g);
        GFCC_LAUNCH_CHECK();
        hipLaunchKernelGGL(diis_gamma_kernel, cgrid, dim3(64), 0, st, Rm, g, m - 1, nb, actd,
                           gam, coef);
        GFCC_LAUNCH_CHECK();
        hipLaunchKernelGGL(diis_extrap_kernel, dim3(gridn(vec)), dim3(256), 0, st, E, vec, m,
                           coef, D, nb, X);
        GFCC_LAUNCH_CHECK();
      }
      k = 0;
    }
  }
  for (int r = 0; r < nb; ++r) {
    const int gr = r0 + r;
    if (gr >= nrhs) continue;
    its_out[gr] = its[r];
    res_out[gr] = rel[r];
  }
  return X;
}

}  // namespace gfcc
