// Shifted linear solves of the GFCC method (Eq. xplin) for many (omega, p) at once.
//
// Right-hand sides are processed in blocks of nb; a block's vectors are stored D-major as
// complex128 [D][nb], so the sigma product of the whole block is one set of matrix products
// (sigma.hip). Each right-hand side runs its own restarted GMRES on
//   M(omega) x = b,  M(omega) = (omega - i eta) I + Hbar_N,
// right-preconditioned by the Jacobi matrix diag(M(omega)). Arnoldi uses classical
// Gram-Schmidt with one full re-orthogonalisation pass (CGS2). Givens rotations, the
// convergence test and the triangular solve run on the device, one thread per right-hand side.
// A cycle ends with the residual of the updated iterate. In FP64 it is formed from the Arnoldi
// relation M Z = V H (Z = P^-1 V, the sigma products of the cycle): r = V (beta e1 - H y),
// which equals b - M x to rounding whether or not V stays orthogonal, and costs one pass over
// the basis, fused with the update of x, instead of another sigma product. It is the stopping
// test. A cycle started from a given x0 begins with the explicit b - M x0. With a
// reduced-precision sigma inside the cycle the relation holds for that operator only, so every
// cycle ends with the explicit FP64 residual: FP64 iterative refinement around a low-precision
// GMRES (GMRES-IR).
#include <algorithm>
#include <cmath>

#include "blockvec.h"

namespace gfcc {
namespace {

// basis vectors covered by one sweep of the fused Arnoldi kernels; restart lengths up to 2 FJ
// run every step with delayed reorthogonalisation, in two sweeps per pass beyond FJ vectors,
// and longer ones on the CGS2 kernels (fused up to FJ vectors, then dots_kernel and
// update_kernel)
constexpr int FJ = 32;
constexpr int FD = 2 * FJ;


// partial[blk][jj][r] = sum over this block's rows of conj(V_j[d][r]) * W[d][r], j = j0 + jj.
// Grid (nblk, ceil(nb / 64)), one wavefront per block; every lane owns one right-hand side
// and walks the block's rows, so each row of V_j and W is one contiguous 1 KB read per wave.
__global__ __launch_bounds__(CW) void dots_kernel(const double2* __restrict__ V, int64_t vstride,
                                                  int j0, int nj, const double2* __restrict__ W,
                                                  int64_t D, int nb, double2* __restrict__ partial) {
  const int r = blockIdx.y * CW + threadIdx.x;
  if (r >= nb) return;
  double2 acc[JG];
#pragma unroll
  for (int jj = 0; jj < JG; ++jj) acc[jj] = make_double2(0.0, 0.0);
  const int64_t rows_per_blk = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t d1 = min(D, d0 + rows_per_blk);
  const double2* __restrict__ Vj = V + (int64_t)j0 * vstride + r;
#pragma unroll 2
  for (int64_t d = d0; d < d1; ++d) {
    const double2 w = W[d * nb + r];
#pragma unroll
    for (int jj = 0; jj < JG; ++jj) {
      if (jj < nj) {
        const double2 p = cconjmul(Vj[(int64_t)jj * vstride + d * nb], w);
        acc[jj].x += p.x;
        acc[jj].y += p.y;
      }
    }
  }
#pragma unroll
  for (int jj = 0; jj < JG; ++jj)
    if (jj < nj) partial[((int64_t)blockIdx.x * JG + jj) * nb + r] = acc[jj];
}

// ---- fused Arnoldi passes over NJ <= FJ basis vectors (the grid of dots_kernel; partial rows are
// FJ apart per block). NJ is a template parameter so that every load of a row is issued before
// the arithmetic that consumes it.

// W += z U (the shift of M(omega) after the sigma product), then the first Gram-Schmidt
// pass's dots with V_0 .. V_{NJ-1}
template <int NJ>
__global__ __launch_bounds__(CW) void shift_dots_kernel(const double2* __restrict__ V,
                                                        int64_t vstride,
                                                        const double2* __restrict__ U,
                                                        const double2* __restrict__ z,
                                                        double2* __restrict__ W, int64_t D, int nb,
                                                        double2* __restrict__ partial) {
  const int r = blockIdx.y * CW + threadIdx.x;
  if (r >= nb) return;
  const double2 zz = z[r];
  double2 acc[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) acc[jj] = make_double2(0.0, 0.0);
  const int64_t rows_per_blk = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t d1 = min(D, d0 + rows_per_blk);
  for (int64_t d = d0; d < d1; ++d) {
    const int64_t idx = d * nb + r;
    double2 vj[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) vj[jj] = V[(int64_t)jj * vstride + idx];
    double2 w = W[idx];
    const double2 p = cmul(zz, U[idx]);
    w.x += p.x;
    w.y += p.y;
    W[idx] = w;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const double2 q = cconjmul(vj[jj], w);
      acc[jj].x += q.x;
      acc[jj].y += q.y;
    }
  }
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) partial[((int64_t)blockIdx.x * FJ + jj) * nb + r] = acc[jj];
}

// W -= sum_j V_j h[j]; then, with the same V_j in registers, the dots of the next pass
template <int NJ>
__global__ __launch_bounds__(CW) void update_dots_kernel(const double2* __restrict__ V,
                                                         int64_t vstride,
                                                         const double2* __restrict__ h,
                                                         double2* __restrict__ W, int64_t D,
                                                         int nb, double2* __restrict__ partial) {
  const int r = blockIdx.y * CW + threadIdx.x;
  if (r >= nb) return;
  double2 hr[NJ], acc[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) {
    hr[jj] = h[(int64_t)jj * nb + r];
    acc[jj] = make_double2(0.0, 0.0);
  }
  const int64_t rows_per_blk = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t d1 = min(D, d0 + rows_per_blk);
  for (int64_t d = d0; d < d1; ++d) {
    const int64_t idx = d * nb + r;
    double2 vj[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) vj[jj] = V[(int64_t)jj * vstride + idx];
    double2 w = W[idx];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const double2 p = cmul(vj[jj], hr[jj]);
      w.x -= p.x;
      w.y -= p.y;
    }
    W[idx] = w;
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const double2 q = cconjmul(vj[jj], w);
      acc[jj].x += q.x;
      acc[jj].y += q.y;
    }
  }
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) partial[((int64_t)blockIdx.x * FJ + jj) * nb + r] = acc[jj];
}

// W -= sum_j V_j h[j]; partial |W|^2 (the norm_kernel layout)
template <int NJ>
__global__ __launch_bounds__(CW) void update_norm_kernel(const double2* __restrict__ V,
                                                         int64_t vstride,
                                                         const double2* __restrict__ h,
                                                         double2* __restrict__ W, int64_t D,
                                                         int nb, double* __restrict__ partial) {
  const int r = blockIdx.y * CW + threadIdx.x;
  if (r >= nb) return;
  double2 hr[NJ];
#pragma unroll
  for (int jj = 0; jj < NJ; ++jj) hr[jj] = h[(int64_t)jj * nb + r];
  double acc = 0.0;
  const int64_t rows_per_blk = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t d1 = min(D, d0 + rows_per_blk);
  for (int64_t d = d0; d < d1; ++d) {
    const int64_t idx = d * nb + r;
    double2 vj[NJ];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) vj[jj] = V[(int64_t)jj * vstride + idx];
    double2 w = W[idx];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const double2 p = cmul(vj[jj], hr[jj]);
      w.x -= p.x;
      w.y -= p.y;
    }
    W[idx] = w;
    acc += w.x * w.x + w.y * w.y;
  }
  partial[(int64_t)blockIdx.x * nb + r] = acc;
}

// launch tables over NJ = 1 .. FJ
typedef void (*ShiftDotsFn)(const double2*, int64_t, const double2*, const double2*, double2*,
                            int64_t, int, double2*);
typedef void (*UpdateDotsFn)(const double2*, int64_t, const double2*, double2*, int64_t, int,
                             double2*);
typedef void (*UpdateNormFn)(const double2*, int64_t, const double2*, double2*, int64_t, int,
                             double*);
template <int... I> struct FusedTables {
  static constexpr ShiftDotsFn shift_dots[] = {shift_dots_kernel<I + 1>...};
  static constexpr UpdateDotsFn update_dots[] = {update_dots_kernel<I + 1>...};
  static constexpr UpdateNormFn update_norm[] = {update_norm_kernel<I + 1>...};
};
using Fused = FusedTables<0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20,
                          21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31>;
static_assert(FJ == 32, "the launch tables cover NJ = 1 .. 32");

// ---- Arnoldi with delayed reorthogonalisation (restart lengths up to FD).
// Step j applies the operator to the pending vector vt_j (orthogonalised once against the
// final basis Q_0 .. Q_{j-1}, not yet normalised). One sweep over the basis (pass A) gives
// t = Q^H w and beta = vt_j^H w for w = M(omega) P^{-1} vt_j; one reduction also completes
// s = Q^H vt_j and alpha = |vt_j|^2, which the previous step's update sweep accumulated.
// Then rho = sqrt(alpha - |s|^2) is the norm of the reorthogonalised vector, column j-1 of
// the Hessenberg matrix is c_{j-1} + s with subdiagonal rho, and the second sweep (pass B)
// writes q_j = (vt_j - Q s) / rho, the next pending vector vt_{j+1} = (w - Q t - g_j q_j) /
// rho with g_j = (beta - s^H t) / rho, its preconditioned copy, and the dots s, alpha of
// vt_{j+1}. The first-pass coefficients of column j are c_j = (g - Hbar s) / rho with
// g = (t, g_j); Hbar s is formed by the next step's reduction. Two sweeps over the basis per
// step instead of three, one reduction instead of three. The pending vector is stored only as
// its preconditioned copy U = vt / (diag + z), which the operator product needs anyway; both
// sweeps read U for the shift and recover vt = U (diag + z) from it, so a step moves the basis
// twice plus 6 vectors (W and U read by each sweep; q_j and U written) instead of 9.
// A register file holds the rows of at most FJ basis vectors; beyond that (j > FJ) each pass is
// split at c = j - FJ. Pass A: one sweep over Q_0 .. Q_{c-1}, one over Q_c .. Q_{j-1} and the
// pending vector (W and U read twice). Pass B: Q_0 .. Q_{c-1} form their shares of
// vt_j - Q s and w - Q t (dcgs_lincomb_kernel; the first in the slot of q_j, the second in a
// scratch vector), the sweep over Q_c .. Q_{j-1} completes both as above, and a last sweep forms
// the dots of Q_0 .. Q_{c-1} with the new pending vector (dcgs_dots_kernel, VN): 3j - 19 vector
// passes per step instead of 2j + 6.
constexpr int PB = FD + 1;       // first partial row of pass B (pass A uses rows 0 .. j)
constexpr int PSTR = PB + FD + 2;  // partial rows per block

// The four wavefronts of a sweep workgroup take every fourth row of its range; their partial
// sums are added in LDS, in a fixed order, C rows at a time (buf holds 4 C rows of CW values),
// and the workgroup writes one partial row per sum: dst[c][r] for c < NA. Every thread of the
// workgroup calls this (it holds barriers); lanes past nb carry zero sums and store nothing.
template <int NA, int C>
__device__ __forceinline__ void combine_partials(const double2 (&acc)[NA], double2 (*buf)[CW],
                                                 double2* __restrict__ dst, int64_t NB, int nb) {
  const int lane = threadIdx.x & (CW - 1), wave = threadIdx.x / CW;
  const int r0 = blockIdx.y * CW;
#pragma unroll
  for (int c0 = 0; c0 < NA; c0 += C) {
    __syncthreads();  // the buffer's previous contents have been read
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (c0 + c < NA) buf[wave * C + c][lane] = acc[c0 + c];
    __syncthreads();
    for (int e = threadIdx.x; e < C * CW; e += 256) {
      const int c = e / CW, l = e % CW;
      if (c0 + c >= NA || r0 + l >= nb) continue;
      double2 t = buf[c][l];
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        t.x += buf[q * C + c][l].x;
        t.y += buf[q * C + c][l].y;
      }
      dst[(int64_t)(c0 + c) * NB + r0 + l] = t;
    }
  }
}

// pass A: partial[blk][jj][r] = sum_d conj(Q_jj[d][r]) w[d][r] (jj < NJ) and row NJ with the
// pending vector vt = U (diag + z), w = W + z U; one workgroup of four wavefronts per block of
// rows. VN: rows jj < NJ only, of the pending vector itself (w = U (diag + z); W is not read).
template <int NJ, bool VN = false>
__global__ __launch_bounds__(256) void dcgs_dots_kernel(const double2* __restrict__ V,
                                                        int64_t vstride,
                                                        const double2* __restrict__ Wv,
                                                        const double2* __restrict__ U,
                                                        const double2* __restrict__ z,
                                                        const double* __restrict__ diag,
                                                        int64_t D, int nb,
                                                        double2* __restrict__ partial) {
  constexpr int C = 8;
  __shared__ double2 buf[4 * C][CW];
  const int lane = threadIdx.x & (CW - 1), wave = threadIdx.x / CW;
  const int r = blockIdx.y * CW + lane;
  const bool live = r < nb;
  const double2 zz = live ? z[r] : make_double2(0.0, 0.0);
  constexpr int NA = VN ? NJ : NJ + 1;
  double2 acc[NA];
#pragma unroll
  for (int jj = 0; jj < NA; ++jj) acc[jj] = make_double2(0.0, 0.0);
  const int64_t rows_per_blk = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t d1 = live ? min(D, d0 + rows_per_blk) : d0;
  for (int64_t d = d0 + wave; d < d1; d += 4) {
    const int64_t idx = d * nb + r;
    double2 vj[NJ + 1];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) vj[jj] = V[(int64_t)jj * vstride + idx];
    const double2 u = U[idx];
    const double2 vt = cmul(u, make_double2(diag[d] + zz.x, zz.y));
    double2 w = vt;
    if (!VN) {
      w = Wv[idx];
      vj[NJ] = vt;
      const double2 p = cmul(zz, u);
      w.x += p.x;
      w.y += p.y;
    }
#pragma unroll
    for (int jj = 0; jj < NA; ++jj) {
      const double2 q = cconjmul(vj[jj], w);
      acc[jj].x += q.x;
      acc[jj].y += q.y;
    }
  }
  combine_partials<NA, C>(acc, buf, partial + (int64_t)blockIdx.x * PSTR * nb, nb, nb);
}

// pass B over Q_0 .. Q_{NJ-1} and the pending vector vt = U (diag + z):
//   q = (vt - sum_i Q_i s_i) qscale          -> V slot NJ
//   vn = (w - sum_i Q_i t_i - g q) vscale    (not when FINAL)
//   U = vn / (diag + z), the next pending vector's only copy (the next sweeps recover
//   vt' = U (diag + z) = vn to rounding); partial rows PB + i = conj(Q_i) vn,
//   PB + NJ = conj(q) vn, PB + NJ + 1 = |vn|^2
// s, t: [NJ][nb] (t row NJ holds g). FINAL (end of a cycle) only writes q. Four wavefronts
// share the coefficients of their 64 RHS in LDS (registers hold the basis rows and the dots)
// and take every fourth row of the workgroup's range; the workgroup writes one partial row per
// sum (combine_partials). PRE (the later sweep of a split pass): the slot of q holds
// sum_i Q_i s_i over the earlier basis vectors and T1 their sum_i Q_i t_i, which start the
// two combinations.
template <int NJ, bool FINAL, bool PRE = false>
__global__ __launch_bounds__(256, NJ <= 24 ? 2 : 1) void dcgs_update_kernel(
    double2* __restrict__ V, int64_t vstride, const double2* __restrict__ Wv,
    double2* __restrict__ U, const double2* __restrict__ z, const double* __restrict__ diag,
    const double2* __restrict__ sc, const double2* __restrict__ tc,
    const double* __restrict__ qscale, const double* __restrict__ vscale, int64_t D, int nb,
    double2* __restrict__ partial, const double2* __restrict__ T1) {
  constexpr int NS = NJ > 0 ? NJ : 1;
  // the coefficients s (rows 0 .. NS-1) and t (rows NS ..) of the workgroup's 64 RHS; after the
  // sweep the same buffer adds the four wavefronts' partial sums, C rows at a time
  constexpr int NL = FINAL ? NS : 2 * NS;
  constexpr int NBUF = NL > 16 ? NL : 16;
  constexpr int C = NBUF / 4;
  __shared__ double2 buf[NBUF][CW];
  double2 (*s_l)[CW] = buf;
  double2 (*t_l)[CW] = buf + NS;
  const int lane = threadIdx.x & (CW - 1), wave = threadIdx.x / CW;
  const int r = blockIdx.y * CW + lane;
  const int64_t NB = nb;
  for (int e = threadIdx.x; e < NJ * CW; e += 256) {
    const int jj = e / CW, l = e % CW;
    const int rr = blockIdx.y * CW + l;
    s_l[jj][l] = rr < nb ? sc[jj * NB + rr] : make_double2(0.0, 0.0);
    if (!FINAL) t_l[jj][l] = rr < nb ? tc[jj * NB + rr] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const bool live = r < nb;
  if (FINAL && !live) return;  // the final sweep has no barrier after this point
  const double2 gq = (FINAL || !live) ? make_double2(0.0, 0.0) : tc[(int64_t)NJ * NB + r];
  const double qs = live ? qscale[r] : 0.0;
  const double vs = (FINAL || !live) ? 0.0 : vscale[r];
  const double2 zz = live ? z[r] : make_double2(0.0, 0.0);
  constexpr int NA = FINAL ? 1 : NJ + 2;
  double2 acc[NA];
#pragma unroll
  for (int jj = 0; jj < NA; ++jj) acc[jj] = make_double2(0.0, 0.0);
  const int64_t rows_per_blk = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t d1 = live ? min(D, d0 + rows_per_blk) : d0;
  for (int64_t d = d0 + wave; d < d1; d += 4) {
    const int64_t idx = d * nb + r;
    // an opaque zero keeps the coefficient reads inside the loop (hoisted, they would take
    // the registers that LDS is there to spare)
    int opq;
    asm volatile("v_mov_b32 %0, 0" : "=v"(opq));
    const int li = lane + opq;
    double2 vj[NS];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) vj[jj] = V[(int64_t)jj * vstride + idx];
    const double2 u = U[idx];
    const double2 dz = make_double2(diag[d] + zz.x, zz.y);
    double2 q = cmul(u, dz);
    double2 w = make_double2(0.0, 0.0);
    if (!FINAL) w = Wv[idx];
    if (PRE) {
      const double2 s1 = V[(int64_t)NJ * vstride + idx];
      q.x -= s1.x;
      q.y -= s1.y;
      if (!FINAL) {
        const double2 t1 = T1[idx];
        w.x -= t1.x;
        w.y -= t1.y;
      }
    }
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const double2 a = cmul(vj[jj], s_l[jj][li]);
      q.x -= a.x;
      q.y -= a.y;
    }
    q.x *= qs;
    q.y *= qs;
    V[(int64_t)NJ * vstride + idx] = q;
    if (FINAL) continue;
    {
      const double2 p = cmul(zz, u);
      w.x += p.x;
      w.y += p.y;
    }
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const double2 a = cmul(vj[jj], t_l[jj][li]);
      w.x -= a.x;
      w.y -= a.y;
    }
    {
      const double2 a = cmul(q, gq);
      w.x = (w.x - a.x) * vs;
      w.y = (w.y - a.y) * vs;
    }
    U[idx] = cdiv(w, dz);
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const double2 a = cconjmul(vj[jj], w);
      acc[jj].x += a.x;
      acc[jj].y += a.y;
    }
    {
      const double2 a = cconjmul(q, w);
      acc[NJ].x += a.x;
      acc[NJ].y += a.y;
      acc[NA - 1].x += w.x * w.x + w.y * w.y;
    }
  }
  if (FINAL) return;
  combine_partials<NA, C>(acc, buf, partial + ((int64_t)blockIdx.x * PSTR + PB) * NB, NB, nb);
}

// The earlier NC basis vectors' share of pass B when the pass is split (see above):
// S = sum_{i<NC} Q_i s_i and, unless FINAL, T = sum_{i<NC} Q_i t_i, with the coefficients of
// the workgroup's 64 RHS in LDS and the rows taken as in dcgs_update_kernel.
template <int NC, bool FINAL>
__global__ __launch_bounds__(256) void dcgs_lincomb_kernel(const double2* __restrict__ V,
                                                           int64_t vstride,
                                                           const double2* __restrict__ sc,
                                                           const double2* __restrict__ tc,
                                                           int64_t D, int nb,
                                                           double2* __restrict__ S,
                                                           double2* __restrict__ T) {
  __shared__ double2 s_l[NC][CW];
  __shared__ double2 t_l[FINAL ? 1 : NC][CW];
  const int lane = threadIdx.x & (CW - 1), wave = threadIdx.x / CW;
  const int r = blockIdx.y * CW + lane;
  const int64_t NB = nb;
  for (int e = threadIdx.x; e < NC * CW; e += 256) {
    const int jj = e / CW, l = e % CW;
    const int rr = blockIdx.y * CW + l;
    s_l[jj][l] = rr < nb ? sc[jj * NB + rr] : make_double2(0.0, 0.0);
    if (!FINAL) t_l[jj][l] = rr < nb ? tc[jj * NB + rr] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  if (r >= nb) return;
  const int64_t rows_per_blk = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t d1 = min(D, d0 + rows_per_blk);
  for (int64_t d = d0 + wave; d < d1; d += 4) {
    const int64_t idx = d * nb + r;
    int opq;  // an opaque zero, as in dcgs_update_kernel
    asm volatile("v_mov_b32 %0, 0" : "=v"(opq));
    const int li = lane + opq;
    double2 vj[NC];
#pragma unroll
    for (int jj = 0; jj < NC; ++jj) vj[jj] = V[(int64_t)jj * vstride + idx];
    double2 a = make_double2(0.0, 0.0), b = make_double2(0.0, 0.0);
#pragma unroll
    for (int jj = 0; jj < NC; ++jj) {
      const double2 p = cmul(vj[jj], s_l[jj][li]);
      a.x += p.x;
      a.y += p.y;
      if (!FINAL) {
        const double2 q = cmul(vj[jj], t_l[jj][li]);
        b.x += q.x;
        b.y += q.y;
      }
    }
    S[idx] = a;
    if (!FINAL) T[idx] = b;
  }
}

// The step's reduction, grid (ceil(nb/64), nA + nB + nH), 256 threads:
//   y < nA:            red[y] = sum_blk partial[blk][y]            (pass A rows)
//   nA <= y < nA + nB: red[PB + i] = sum_blk partial[blk][PB + i]  (pass B rows, i = y - nA)
//   y >= nA + nB:      hs[l] = sum_{i = max(l-1, 0)}^{nh_s - 1} Hraw[col i][row l] s_i with
//                      s = sc (the previous step's s), l = y - nA - nB (one wavefront)
// The block sums run as in dots_reduce_s.
__global__ __launch_bounds__(256) void dcgs_reduce_kernel(
    const double2* __restrict__ partial, int nblk, int nA, int nB, int nh_s, int nb, int m,
    const double2* __restrict__ Hraw, const double2* __restrict__ sc,
    double2* __restrict__ red, double2* __restrict__ hs) {
  __shared__ double2 sum4[4][CW];
  const int lane = threadIdx.x % CW, w = threadIdx.x / CW;
  const int r = blockIdx.x * CW + lane;
  const int y = blockIdx.y;
  const int64_t NB = nb;
  if (y >= nA + nB) {
    if (w != 0 || r >= nb) return;
    const int l = y - nA - nB;
    double2 acc = make_double2(0.0, 0.0);
    for (int i = l > 0 ? l - 1 : 0; i < nh_s; ++i) {
      const double2 a = cmul(Hraw[((int64_t)i * (m + 1) + l) * NB + r], sc[(int64_t)i * NB + r]);
      acc.x += a.x;
      acc.y += a.y;
    }
    hs[(int64_t)l * NB + r] = acc;
    return;
  }
  const int row = y < nA ? y : PB + (y - nA);
  // wavefront w sums blocks w, w + 4, ...: eight loads in flight, then a fixed-order sum
  double2 sacc = make_double2(0.0, 0.0);
  if (r < nb) {
    for (int b0 = w; b0 < nblk; b0 += 32) {
      double2 x[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int b = b0 + 4 * t;
        x[t] = b < nblk ? partial[((int64_t)b * PSTR + row) * NB + r] : make_double2(0.0, 0.0);
      }
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        sacc.x += x[t].x;
        sacc.y += x[t].y;
      }
    }
  }
  sum4[w][lane] = sacc;
  __syncthreads();
  if (w == 0 && r < nb) {
    double2 t = sum4[0][lane];
    for (int q = 1; q < 4; ++q) {
      t.x += sum4[q][lane].x;
      t.y += sum4[q][lane].y;
    }
    red[(int64_t)row * NB + r] = t;
  }
}

typedef void (*DcgsDotsFn)(const double2*, int64_t, const double2*, const double2*,
                           const double2*, const double*, int64_t, int, double2*);
typedef void (*DcgsUpdateFn)(double2*, int64_t, const double2*, double2*, const double2*,
                             const double*, const double2*, const double2*, const double*,
                             const double*, int64_t, int, double2*, const double2*);
typedef void (*DcgsLincombFn)(const double2*, int64_t, const double2*, const double2*, int64_t,
                              int, double2*, double2*);
template <int... I> struct DcgsTables {  // I = 1 .. FJ
  static constexpr DcgsDotsFn dots[] = {dcgs_dots_kernel<0>, dcgs_dots_kernel<I>...};  // NJ = 0 .. FJ
  static constexpr DcgsUpdateFn update[] = {dcgs_update_kernel<0, false>,
                                            dcgs_update_kernel<I, false>...};  // NJ = 0 .. FJ
  static constexpr DcgsUpdateFn final_[] = {dcgs_update_kernel<I, true>...};  // NJ - 1, NJ = 1 .. FJ
  static constexpr DcgsDotsFn vdots[] = {dcgs_dots_kernel<I, true>...};           // NC - 1
  static constexpr DcgsLincombFn lin[] = {dcgs_lincomb_kernel<I, false>...};      // NC - 1
  static constexpr DcgsLincombFn lin_final[] = {dcgs_lincomb_kernel<I, true>...};  // NC - 1
};
using Dcgs = DcgsTables<1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 15, 16, 17, 18, 19, 20,
                        21, 22, 23, 24, 25, 26, 27, 28, 29, 30, 31, 32>;


// W[d][r] -= sum_{j<=k} V_j[d][r] * h[j][r]
__global__ void update_kernel(const double2* __restrict__ V, int64_t vstride, int nj,
                              const double2* __restrict__ h, int64_t D, int nb,
                              double2* __restrict__ W) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    double2 w = W[idx];
    for (int j = 0; j < nj; ++j) {
      double2 p = cmul(V[(int64_t)j * vstride + idx], h[(int64_t)j * nb + r]);
      w.x -= p.x;
      w.y -= p.y;
    }
    W[idx] = w;
  }
}

// nrm partial: sum |W[d][r]|^2 (same grid as dots_kernel)
__global__ __launch_bounds__(CW) void norm_kernel(const double2* __restrict__ W, int64_t D, int nb,
                                                  double* __restrict__ partial) {
  const int r = blockIdx.y * CW + threadIdx.x;
  if (r >= nb) return;
  double acc = 0.0;
  const int64_t rows_per_blk = (D + gridDim.x - 1) / gridDim.x;
  const int64_t d0 = (int64_t)blockIdx.x * rows_per_blk;
  const int64_t d1 = min(D, d0 + rows_per_blk);
#pragma unroll 4
  for (int64_t d = d0; d < d1; ++d) {
    const double2 w = W[d * nb + r];
    acc += w.x * w.x + w.y * w.y;
  }
  partial[(int64_t)blockIdx.x * nb + r] = acc;
}


// U[d][r] = V[d][r] / (diag[d] + z[r])
__global__ void precond_kernel(const double2* __restrict__ V, const double* __restrict__ diag,
                               const double2* __restrict__ z, int64_t D, int nb,
                               double2* __restrict__ U) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    const int64_t d = idx / nb;
    double2 zz = z[r];
    U[idx] = cdiv(V[idx], make_double2(diag[d] + zz.x, zz.y));
  }
}

// W[d][r] = S[d][r] + z[r] * U[d][r]   (S may alias W)
__global__ void shift_kernel(const double2* S, const double2* __restrict__ U,
                             const double2* __restrict__ z, int64_t D, int nb, double2* W) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    double2 p = cmul(z[r], U[idx]);
    double2 s = S[idx];
    W[idx] = make_double2(s.x + p.x, s.y + p.y);
  }
}

// R = B - S  (S = M X, shift included)
__global__ void residual_kernel(const double2* __restrict__ B, const double2* __restrict__ S,
                                int64_t n, double2* __restrict__ R) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double2 b = B[idx], s = S[idx];
    R[idx] = make_double2(b.x - s.x, b.y - s.y);
  }
}

// V0 = R / beta (zero for inactive)
__global__ void scale_kernel(const double2* __restrict__ W, const double* __restrict__ inv,
                             int64_t D, int nb, double2* __restrict__ V) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    double s = inv[r];
    double2 w = W[idx];
    V[idx] = make_double2(w.x * s, w.y * s);
  }
}

// Vn[d][r] = W[d][r] inv[r] and U[d][r] = Vn[d][r] / (diag[d] + z[r]) (the next basis vector
// and its preconditioned copy in one pass)
__global__ void scale_precond_kernel(const double2* __restrict__ W, const double* __restrict__ inv,
                                     const double* __restrict__ diag, const double2* __restrict__ z,
                                     int64_t D, int nb, double2* __restrict__ Vn,
                                     double2* __restrict__ U) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    const int64_t d = idx / nb;
    const double s = inv[r];
    const double2 w = W[idx];
    const double2 x = make_double2(w.x * s, w.y * s);
    Vn[idx] = x;
    const double2 zz = z[r];
    U[idx] = cdiv(x, make_double2(diag[d] + zz.x, zz.y));
  }
}

struct BlockState {
  // Per-RHS arrays are stored with the RHS index fastest, so that the one-thread-per-RHS
  // kernels below read and write consecutive addresses across a wavefront.
  double2* H;      // [m][m+1][nb]  row i of column k of RHS r at H[(k*(m+1) + i)*nb + r]
  double2* Hraw;   // [m][m+1][nb]  the same columns before the Givens rotations
  double* beta;    // [nb] norm of the residual the cycle started from (0: not in the cycle)
  double2* cs;     // [m][nb]
  double2* sn;     // [m][nb]
  double2* g;      // [m+1][nb]
  int* active;     // [nb]
  int* kend;       // [nb] steps taken this cycle
  int* its;        // [nb] total iterations
  int* brk;        // [nb] singular least-squares flag
  double* resest;  // [nb]
  double* thresh;  // [nb] inner stopping threshold (absolute)
  double* inv;     // [nb] 1/||w|| for the new basis vector
};

// Column k of the Hessenberg matrix of one RHS (thread r): entries i <= k from get(i),
// subdiagonal nrm. Stores the raw column, applies the previous Givens rotations (their
// operands loaded eight rows at a time ahead of the serial chain), forms rotation k, updates g
// and the residual estimate, counts the iteration and returns 0 when the RHS continues, 1 when
// it stops, 2 when the column is singular (the active flag is cleared for 1 and 2; a singular
// column is excluded from the least-squares problem).
template <typename Get>
__device__ __forceinline__ int givens_column(const BlockState& s, int r, int k, int m, int nb,
                                              int maxit, double nrm, Get get) {
  const int64_t NB = nb;
  double2* col = s.H + (int64_t)k * (m + 1) * NB + r;
  double2* raw = s.Hraw + (int64_t)k * (m + 1) * NB + r;
  const double2* cs = s.cs + r;
  const double2* sn = s.sn + r;
  double2 a = get(0);
  raw[0] = a;
  for (int i0 = 0; i0 < k; i0 += 8) {
    double2 hb[8], cb[8], sb[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (i0 + t < k) {
        hb[t] = get(i0 + t + 1);
        cb[t] = cs[(int64_t)(i0 + t) * NB];
        sb[t] = sn[(int64_t)(i0 + t) * NB];
      }
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      if (i0 + t < k) {
        const int i = i0 + t;
        const double2 b = hb[t];
        raw[(int64_t)(i + 1) * NB] = b;
        const double2 t1 = cconjmul(cb[t], a), t2 = cconjmul(sb[t], b);
        const double2 u1 = cmul(sb[t], a), u2 = cmul(cb[t], b);
        col[(int64_t)i * NB] = make_double2(t1.x + t2.x, t1.y + t2.y);
        a = make_double2(u2.x - u1.x, u2.y - u1.y);
      }
    }
  }
  const double2 b = make_double2(nrm, 0.0);
  raw[(int64_t)(k + 1) * NB] = b;
  const double den = hypot(hypot(a.x, a.y), nrm);
  s.its[r] += 1;
  s.kend[r] = k + 1;
  if (den == 0.0) {  // singular least-squares problem
    col[(int64_t)k * NB] = a;
    col[(int64_t)(k + 1) * NB] = b;
    s.brk[r] = 1;
    s.active[r] = 0;
    s.kend[r] = k;  // exclude the singular column
    return 2;
  }
  const double2 c = make_double2(a.x / den, a.y / den), sv = make_double2(nrm / den, 0.0);
  s.cs[(int64_t)k * NB + r] = c;
  s.sn[(int64_t)k * NB + r] = sv;
  col[(int64_t)k * NB] = make_double2(den, 0.0);
  col[(int64_t)(k + 1) * NB] = make_double2(0.0, 0.0);
  double2* g = s.g + r;
  const double2 gk = g[(int64_t)k * NB];
  const double2 ng = cmul(sv, gk);
  const double2 gk1 = make_double2(-ng.x, -ng.y);
  g[(int64_t)(k + 1) * NB] = gk1;
  g[(int64_t)k * NB] = cconjmul(c, gk);
  const double est = hypot(gk1.x, gk1.y);
  s.resest[r] = est;
  const bool stop = est <= s.thresh[r] || nrm == 0.0 || s.its[r] >= maxit || k + 1 == m;
  if (stop) s.active[r] = 0;
  return stop ? 1 : 0;
}

// flag_out (optional, host-visible): one word per 64 RHS, nonzero while any of them is active
__device__ __forceinline__ void write_flag(int* flag_out, bool act) {
  if (!flag_out) return;
  const unsigned long long any = __ballot(act);
  if (threadIdx.x == 0) flag_out[blockIdx.x] = any != 0ull ? 1 : 0;
}

// Classical Gram-Schmidt step: column k = h1 + h2 (the two passes), subdiagonal hn; inv = the
// scale of the new basis vector (also for a RHS that stops here: its residual uses that
// vector; zero for a singular column and for a RHS that had stopped before).
__global__ __launch_bounds__(64) void arnoldi_finish_kernel(
    const double2* __restrict__ h1, const double2* __restrict__ h2,
    const double* __restrict__ hn, int k, int m, int nb, int maxit, BlockState s,
    int* __restrict__ flag_out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  bool act = false;
  if (r < nb && s.active[r]) {
    const int64_t NB = nb;
    const double nrm = hn[r];
    const int res = givens_column(s, r, k, m, nb, maxit, nrm, [&](int i) {
      const double2 x = h1[(int64_t)i * NB + r], y = h2[(int64_t)i * NB + r];
      return make_double2(x.x + y.x, x.y + y.y);
    });
    s.inv[r] = (res != 2 && nrm > 0.0) ? 1.0 / nrm : 0.0;
    act = res == 0;
  } else if (r < nb) {
    s.inv[r] = 0.0;
  }
  write_flag(flag_out, act);
}

// Delayed-reorthogonalisation step j (see dcgs_dots_kernel), one thread per RHS, in two parts.
// Column part (j >= 1): rho = sqrt(alpha - |s|^2) and column j-1 = (g_prev - Hbar s_prev) /
// rho_prev + s with subdiagonal rho (g_prev in tc, 1/rho_prev in vscale, Hbar s_prev in hs for
// j >= 2), stored raw and rotated; rotation j-1 and the residual estimate as in givens_column;
// s goes to sc and 1/rho to qscale (the pending vector is finalised with them). Coefficient
// part, for a RHS that continues: t and g_j = (beta - s^H t) / rho to tc, vscale = 1/rho; a RHS
// that stopped gets vscale = 0. mode 0 runs both parts (s, alpha, t and beta all reduced), mode
// 1 the column part only (also the end of a cycle), mode 2 the coefficient part only (after
// mode 1 and the operator product of the step). Every per-row quantity comes from one pass
// whose loads are issued a few rows at a time.
__global__ __launch_bounds__(64) void dcgs_finish_kernel(
    int j, int m, int nb, int maxit, int mode, BlockState s, const double2* __restrict__ red,
    const double2* __restrict__ hs, double2* __restrict__ sc, double2* __restrict__ tc,
    double* __restrict__ qscale, double* __restrict__ vscale, int* __restrict__ flag_out) {
  constexpr int FB = 8;  // rows per batch of loads
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const bool colpart = mode != 2, coefpart = mode != 1;
  bool act = false;
  if (r < nb) {
    const int64_t NB = nb;
    const double2 zero = make_double2(0.0, 0.0);
    bool live = s.active[r] != 0;
    double2 st = zero;  // s^H t (merged mode: accumulated with the column)
    if (colpart) {
      if (!live) {
        qscale[r] = 0.0;
      } else if (j == 0) {  // the pending vector is the normalised start vector: no column yet
        qscale[r] = 1.0;
      } else {
        const int k = j - 1;
        const double ip = vscale[r];
        const bool lag = j >= 2;
        const double alpha = red[(int64_t)(PB + j) * NB + r].x;
        double2* col = s.H + (int64_t)k * (m + 1) * NB + r;
        double2* raw = s.Hraw + (int64_t)k * (m + 1) * NB + r;
        double ss = 0.0;
        double2 a = zero;
        for (int i0 = 0; i0 < j; i0 += FB) {
          double2 sb[FB], tb[FB], gb[FB], hb[FB], cb[FB], qb[FB];
#pragma unroll
          for (int t = 0; t < FB; ++t) {
            // unconditional loads at clamped rows (every buffer has them), values selected
            const int i = i0 + t;
            const int ic = i < j ? i : j - 1, ir = ic > 0 ? ic - 1 : 0;
            const bool on = i < j, rot = on && i >= 1;
            const double2 s_ = red[(int64_t)(PB + ic) * NB + r], t_ = red[(int64_t)ic * NB + r];
            const double2 g_ = tc[(int64_t)ic * NB + r], h_ = hs[(int64_t)ic * NB + r];
            const double2 c_ = s.cs[(int64_t)ir * NB + r], q_ = s.sn[(int64_t)ir * NB + r];
            sb[t] = on ? s_ : zero;
            tb[t] = on && coefpart ? t_ : zero;
            gb[t] = on ? g_ : zero;
            hb[t] = on && lag ? h_ : zero;
            cb[t] = rot ? c_ : zero;
            qb[t] = rot ? q_ : zero;
          }
#pragma unroll
          for (int t = 0; t < FB; ++t) {
            const int i = i0 + t;
            if (i >= j) continue;
            ss += sb[t].x * sb[t].x + sb[t].y * sb[t].y;
            const double2 ci = make_double2((gb[t].x - hb[t].x) * ip + sb[t].x,
                                            (gb[t].y - hb[t].y) * ip + sb[t].y);
            raw[(int64_t)i * NB] = ci;
            sc[(int64_t)i * NB + r] = sb[t];
            if (coefpart) {
              const double2 p = cconjmul(sb[t], tb[t]);
              st.x += p.x;
              st.y += p.y;
              tc[(int64_t)i * NB + r] = tb[t];
            }
            if (i == 0) {
              a = ci;
            } else {  // rotation i-1 on the entries (i-1, i)
              const double2 t1 = cconjmul(cb[t], a), t2 = cconjmul(qb[t], ci);
              const double2 u1 = cmul(qb[t], a), u2 = cmul(cb[t], ci);
              col[(int64_t)(i - 1) * NB] = make_double2(t1.x + t2.x, t1.y + t2.y);
              a = make_double2(u2.x - u1.x, u2.y - u1.y);
            }
          }
        }
        const double rho2 = alpha - ss;
        const double rho = rho2 > 0.0 ? sqrt(rho2) : 0.0;
        const double2 b = make_double2(rho, 0.0);
        raw[(int64_t)j * NB] = b;
        const double den = hypot(hypot(a.x, a.y), rho);
        s.its[r] += 1;
        s.kend[r] = j;
        if (den == 0.0) {  // singular least-squares problem: the column is excluded
          col[(int64_t)k * NB] = a;
          col[(int64_t)j * NB] = b;
          s.brk[r] = 1;
          s.active[r] = 0;
          s.kend[r] = k;
          live = false;
        } else {
          const double2 c = make_double2(a.x / den, a.y / den), sv = make_double2(rho / den, 0.0);
          s.cs[(int64_t)k * NB + r] = c;
          s.sn[(int64_t)k * NB + r] = sv;
          col[(int64_t)k * NB] = make_double2(den, 0.0);
          col[(int64_t)j * NB] = zero;
          double2* g = s.g + r;
          const double2 gk = g[(int64_t)k * NB];
          const double2 ng = cmul(sv, gk);
          const double2 gk1 = make_double2(-ng.x, -ng.y);
          g[(int64_t)j * NB] = gk1;
          g[(int64_t)k * NB] = cconjmul(c, gk);
          const double est = hypot(gk1.x, gk1.y);
          s.resest[r] = est;
          const bool stop = est <= s.thresh[r] || rho == 0.0 || s.its[r] >= maxit || j == m;
          if (stop) s.active[r] = 0;
          live = !stop;
        }
        qscale[r] = rho > 0.0 ? 1.0 / rho : 0.0;
      }
      if (!coefpart) act = live;
    }
    if (coefpart) {
      if (!live) {
        vscale[r] = 0.0;
      } else {
        const double ir = qscale[r];
        if (!colpart) {  // s from sc (column part of this step), t from the reduction
          for (int i0 = 0; i0 < j; i0 += FB) {
            double2 sb[FB], tb[FB];
#pragma unroll
            for (int t = 0; t < FB; ++t) {
              const int i = i0 + t;
              const int ic = i < j ? i : j - 1;
              const double2 s_ = sc[(int64_t)ic * NB + r], t_ = red[(int64_t)ic * NB + r];
              sb[t] = i < j ? s_ : zero;
              tb[t] = i < j ? t_ : zero;
            }
#pragma unroll
            for (int t = 0; t < FB; ++t) {
              const int i = i0 + t;
              if (i >= j) continue;
              const double2 p = cconjmul(sb[t], tb[t]);
              st.x += p.x;
              st.y += p.y;
              tc[(int64_t)i * NB + r] = tb[t];
            }
          }
        }
        const double2 beta = red[(int64_t)j * NB + r];
        tc[(int64_t)j * NB + r] = make_double2((beta.x - st.x) * ir, (beta.y - st.y) * ir);
        vscale[r] = ir;
        act = true;
      }
    }
  }
  write_flag(flag_out, act);
}

// y = H(0:kend,0:kend)^{-1} g(0:kend), written to yout[j][r] (zero beyond kend)
__global__ void ysolve_kernel(int m, int nb, BlockState s, const int* __restrict__ used,
                              double2* __restrict__ yout) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb) return;
  int ke = used[r] ? s.kend[r] : 0;
  const int64_t NB = nb;
  const double2* H = s.H + r;  // H[(j*(m+1) + i)*nb]: row i of column j
  const double2* g = s.g + r;
  for (int j = ke; j < m; ++j) yout[(int64_t)j * NB + r] = make_double2(0.0, 0.0);
  for (int i = ke - 1; i >= 0; --i) {
    double2 acc = g[(int64_t)i * NB];
    for (int j = i + 1; j < ke; ++j) {
      double2 p = cmul(H[((int64_t)j * (m + 1) + i) * NB], yout[(int64_t)j * NB + r]);
      acc.x -= p.x;
      acc.y -= p.y;
    }
    yout[(int64_t)i * NB + r] = cdiv(acc, H[((int64_t)i * (m + 1) + i) * NB]);
  }
}

// The same back substitution for m <= 32, 32 lanes per RHS (two per wavefront): lane l holds
// row l of the rotated (upper triangular) H, loaded at once, and g_l; step i (from kend - 1
// down) takes y_i from lane i and updates the rows above it.
__global__ __launch_bounds__(64) void ysolve32_kernel(int m, int nb, BlockState s,
                                                      const int* __restrict__ used,
                                                      double2* __restrict__ yout) {
  const int half = threadIdx.x >> 5, l = threadIdx.x & 31;
  const int r = blockIdx.x * 2 + half;
  const bool ok = r < nb;
  const int ke = ok && used[r] ? s.kend[r] : 0;
  const int64_t NB = nb;
  double2 row[32];
#pragma unroll
  for (int i = 0; i < 32; ++i)
    row[i] = (i < ke && l <= i) ? s.H[((int64_t)i * (m + 1) + l) * NB + r] : make_double2(0.0, 0.0);
  double2 g = l < ke ? s.g[(int64_t)l * NB + r] : make_double2(0.0, 0.0);
  double2 y = make_double2(0.0, 0.0);
#pragma unroll
  for (int i = 31; i >= 0; --i) {
    const double2 mine = l == i && i < ke ? cdiv(g, row[i]) : make_double2(0.0, 0.0);
    const double2 yi = make_double2(__shfl(mine.x, half * 32 + i), __shfl(mine.y, half * 32 + i));
    if (i < ke) {
      if (l == i) y = yi;
      if (l < i) {
        const double2 a = cmul(row[i], yi);
        g.x -= a.x;
        g.y -= a.y;
      }
    }
  }
  if (ok && l < m) yout[(int64_t)l * NB + r] = y;
}

// Residual coefficients for m <= 32, one wavefront per RHS, lane i = row i (i <= m): the
// row's Hessenberg entries and the y_j it needs are loaded at once.
__global__ __launch_bounds__(64) void rescoef64_kernel(int m, int nb, BlockState s,
                                                       const int* __restrict__ used,
                                                       const double2* __restrict__ y,
                                                       double2* __restrict__ c) {
  const int r = blockIdx.x, i = threadIdx.x;
  if (i > m) return;
  const int ke = used[r] ? s.kend[r] : -1;
  const int64_t NB = nb;
  double2 acc = make_double2(i == 0 && ke >= 0 ? s.beta[r] : 0.0, 0.0);
  if (i <= ke) {
    double2 hv[32], yv[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const bool on = j < ke && j >= i - 1;  // H is upper Hessenberg
      hv[j] = on ? s.Hraw[((int64_t)j * (m + 1) + i) * NB + r] : make_double2(0.0, 0.0);
      yv[j] = on ? y[(int64_t)j * NB + r] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) {
      const double2 a = cmul(hv[j], yv[j]);
      acc.x -= a.x;
      acc.y -= a.y;
    }
  } else {
    acc = make_double2(0.0, 0.0);
  }
  c[(int64_t)i * NB + r] = acc;
}

// X[d][r] += (sum_j V_j[d][r] y[j][r]) / (diag[d] + z[r])
__global__ void xupdate_kernel(const double2* __restrict__ V, int64_t vstride, int nj,
                               const double2* __restrict__ y, const double* __restrict__ diag,
                               const double2* __restrict__ z, int64_t D, int nb,
                               double2* __restrict__ X) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    const int64_t d = idx / nb;
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < nj; ++j) {
      double2 p = cmul(V[(int64_t)j * vstride + idx], y[(int64_t)j * nb + r]);
      acc.x += p.x;
      acc.y += p.y;
    }
    double2 zz = z[r];
    double2 u = cdiv(acc, make_double2(diag[d] + zz.x, zz.y));
    double2 x = X[idx];
    X[idx] = make_double2(x.x + u.x, x.y + u.y);
  }
}

// Residual coefficients of the cycle, one thread per RHS: c = beta e1 - Hraw y over rows
// 0..kend (zero beyond, and for a RHS not in the cycle); c[i][r].
__global__ void rescoef_kernel(int m, int nb, BlockState s, const int* __restrict__ used,
                               const double2* __restrict__ y, double2* __restrict__ c) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nb) return;
  const int ke = used[r] ? s.kend[r] : -1;
  const double2* H = s.Hraw + r;  // H[(j*(m+1) + i)*nb]
  for (int i = 0; i <= m; ++i) {
    double2 acc = make_double2(i == 0 && ke >= 0 ? s.beta[r] : 0.0, 0.0);
    if (i <= ke) {
      for (int j = (i > 0 ? i - 1 : 0); j < ke; ++j) {  // H is upper Hessenberg
        const double2 p = cmul(H[((int64_t)j * (m + 1) + i) * nb], y[(int64_t)j * nb + r]);
        acc.x -= p.x;
        acc.y -= p.y;
      }
    } else {
      acc = make_double2(0.0, 0.0);
    }
    c[(int64_t)i * nb + r] = acc;
  }
}

// The end of a cycle in one pass over the basis: X += (sum_{j<nj} V_j y_j) / (diag + z) and,
// for the RHS in the cycle, R = sum_{i<=nj} V_i c_i (the residual of the updated X by the
// Arnoldi relation); R of the others is left as it is.
__global__ void xupdate_res_kernel(const double2* __restrict__ V, int64_t vstride, int nj,
                                   const double2* __restrict__ y, const double2* __restrict__ c,
                                   const int* __restrict__ used,
                                   const double* __restrict__ diag,
                                   const double2* __restrict__ z, int64_t D, int nb,
                                   double2* __restrict__ X, double2* __restrict__ R) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    const int64_t d = idx / nb;
    double2 acc = make_double2(0.0, 0.0), res = make_double2(0.0, 0.0);
    for (int j = 0; j <= nj; ++j) {
      const double2 vj = V[(int64_t)j * vstride + idx];
      const double2 q = cmul(vj, c[(int64_t)j * nb + r]);
      res.x += q.x;
      res.y += q.y;
      if (j < nj) {
        const double2 p = cmul(vj, y[(int64_t)j * nb + r]);
        acc.x += p.x;
        acc.y += p.y;
      }
    }
    const double2 zz = z[r];
    const double2 u = cdiv(acc, make_double2(diag[d] + zz.x, zz.y));
    const double2 x = X[idx];
    X[idx] = make_double2(x.x + u.x, x.y + u.y);
    if (used[r]) R[idx] = res;
  }
}

// The first sigma product of a forward cycle started from x = 0: there U = e_p / P_pp for
// column r (p = prow[r], P_pp = diag[p] + z[r]), and Hbar_N e_p is column p of Hbar_N, i.e.
// column p of W1 in the 1h rows and of W4c in the 2h1p rows (the three-body, Woo and ovvo
// terms act on the zero 2h1p part). W[d][r] = Hbar_N[d][p] / P_pp, zero for padding columns.
__global__ void unit_sigma_kernel(const int* __restrict__ prow, const double* __restrict__ W1,
                                  const double* __restrict__ W4c, int64_t ldw4,
                                  const double* __restrict__ diag, const double2* __restrict__ z,
                                  int o, int64_t D, int nb, double2* __restrict__ W) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    const int64_t d = idx / nb;
    const int p = prow[r];
    if (p < 0) {
      W[idx] = make_double2(0.0, 0.0);
      continue;
    }
    const double h = d < o ? W1[d * D + p] : W4c[(d - o) * ldw4 + p];
    const double2 zz = z[r];
    const double2 u = cdiv(make_double2(1.0, 0.0), make_double2(diag[p] + zz.x, zz.y));
    W[idx] = make_double2(h * u.x, h * u.y);
  }
}

// right-hand sides: forward b = e_p, transpose b = c_p (row p of Crows)
__global__ void rhs_kernel(const int* __restrict__ prow, const double* __restrict__ Crows,
                           int transpose, int64_t D, int nb, double2* __restrict__ B) {
  const int64_t n = D * nb;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % nb);
    const int64_t d = idx / nb;
    const int p = prow[r];
    double val = 0.0;
    if (p >= 0) val = transpose ? Crows[(int64_t)p * D + d] : (d == p ? 1.0 : 0.0);
    B[idx] = make_double2(val, 0.0);
  }
}

// Column compaction of a block ([D][ns] -> [D][nd]): dst[d][j] = src[d][map[j]] (zero where
// map[j] < 0), and back: dst[d][map[j]] = src[d][j] where map[j] >= 0
__global__ void pick_cols_kernel(const double2* __restrict__ src, int ns,
                                 const int* __restrict__ map, int nd, int64_t D,
                                 double2* __restrict__ dst) {
  const int64_t n = D * nd;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = i / nd;
    const int c = map[i % nd];
    dst[i] = c >= 0 ? src[d * ns + c] : make_double2(0.0, 0.0);
  }
}
__global__ void put_cols_kernel(const double2* __restrict__ src, int nd,
                                const int* __restrict__ map, int ns, int64_t D,
                                double2* __restrict__ dst) {
  const int64_t n = D * nd;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = i / nd;
    const int c = map[i % nd];
    if (c >= 0) dst[d * ns + c] = src[i];
  }
}

// Gq[k][r] = sum_d Crows[q_k][d] X[d][r]  computed by gemm; here the transpose variant:
// Gq[k][r] = X[q_k][r]
__global__ void gather_rows_kernel(const double2* __restrict__ X, const int* __restrict__ q, int nq,
                                   int nb, double2* __restrict__ out) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nq * nb) return;
  int k = idx / nb, r = idx % nb;
  out[idx] = X[(int64_t)q[k] * nb + r];
}

// G_out[w][qk][pk] = Gq[qk][r] for the block's right-hand sides r -> (w, pk). The adjoint
// systems give b_q^T Y_p = G_pq, stored transposed so both directions fill G in one layout.
__global__ void scatter_G_kernel(const double2* __restrict__ Gq, int nq, int nb, int r0,
                                 int nrhs_total, int np, int transpose, double2* __restrict__ G) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nq * nb) return;
  int k = idx / nb, r = idx % nb;
  int gr = r0 + r;
  if (gr >= nrhs_total) return;
  int w = gr / np, pk = gr % np;
  if (transpose) G[((int64_t)w * np + pk) * np + k] = Gq[idx];
  else G[((int64_t)w * np + k) * np + pk] = Gq[idx];
}

__global__ void copy_rows_kernel(const double* __restrict__ C, const int* __restrict__ q, int nq,
                                 int64_t D, double* __restrict__ out) {
  const int64_t n = (int64_t)nq * D;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int k = (int)(idx / D);
    int64_t d = idx - (int64_t)k * D;
    out[idx] = C[(int64_t)q[k] * D + d];
  }
}

__global__ void f64_to_f32_kernel(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (float)s[i];
}
__global__ void f32_to_f64_kernel(const float* __restrict__ s, double* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (double)s[i];
}


}  // namespace

// ------------------------------------------------------------------------------------------
// Block GMRES driver
struct GmresBlock {
  gfcc_ctx* ctx = nullptr;
  int64_t D = 0;
  int nb = 0, m = 0;
  int precision = GFCC_FP64;
  bool transpose = false;
  // work arrays live in the context (ws_solve, ws_solve_f32), so that consecutive solves
  // reuse them instead of allocating and freeing the Krylov basis every call
  double2 *V, *W, *U, *X, *B, *R, *Hh, *Hh2, *Y, *Cc, *z;
  // delayed-reorthogonalisation state: reduced dots, Hbar s, pass-B coefficients and scales
  double2 *red = nullptr, *hsb = nullptr, *scb = nullptr, *tcb = nullptr;
  double *qsc = nullptr, *vsc = nullptr;
  double *nrm, *part_n;
  double2* part_h;
  int *used, *prow;
  float *Uf = nullptr, *Sf = nullptr;
  BlockState s;
  int nblk_rows = 1, nbrows_y = 1;
  // convergence flags written by the finishing kernels straight into host-visible memory (one
  // word per 64 RHS, two slots by step parity; owned by the context, so that captured steps
  // stay valid from solve to solve)
  int* hflags = nullptr;
  int* dflags = nullptr;  // the same memory as the kernel sees it
  hipEvent_t flag_ev[2] = {nullptr, nullptr};

  GmresBlock() = default;
  GmresBlock(const GmresBlock&) = delete;
  GmresBlock& operator=(const GmresBlock&) = delete;
  ~GmresBlock() {
    for (hipEvent_t e : flag_ev)
      if (e) (void)hipEventDestroy(e);
  }

  // a multiple of 4: the delayed-reorthogonalisation sweeps run row_blocks / 4 workgroups of
  // four wavefronts, one partial row per workgroup and sum
  static int row_blocks(int64_t D, int nb) {
    const int n = (int)std::min<int64_t>(1024, std::max<int64_t>(1, D * nb / 4096));
    return (n + 3) / 4 * 4;
  }
  // rows of nb partial dots: the fused CGS2 sweeps write FJ per block of rows, the delayed-
  // reorthogonalisation sweeps PSTR per workgroup (nblk / 4 of them)
  static int64_t part_rows(int nblk) {
    return std::max<int64_t>((int64_t)nblk * FJ, (int64_t)(nblk / 4) * PSTR);
  }
  // bytes of the work arrays of a block (each array 256-byte aligned)
  static int64_t bytes_for(int64_t D, int nb, int m) {
    const int64_t vec = D * nb;
    const int nblk = row_blocks(D, nb);
    int64_t bytes = 0;
    auto add = [&](int64_t n, int64_t sz) { bytes += ((n * sz + 255) / 256) * 256; };
    add(vec * (m + 1), 16);                                   // V
    for (int i = 0; i < 5; ++i) add(vec, 16);                 // W U X B R
    add((int64_t)(m + 1) * nb, 16); add((int64_t)(m + 1) * nb, 16);  // Hh Hh2
    add((int64_t)m * nb, 16);                                 // Y
    add((int64_t)(m + 1) * nb, 16);                           // Cc
    add(nb, 16);                                              // z
    add(nb, 8);                                               // nrm
    add((int64_t)nblk * nb, 8);                               // part_n
    add(part_rows(nblk) * nb, 16);                            // part_h
    add((int64_t)PSTR * nb, 16); add((int64_t)(FD + 1) * nb, 16);    // red hsb
    add((int64_t)(FD + 1) * nb, 16); add((int64_t)(FD + 2) * nb, 16);  // scb tcb
    add(nb, 8); add(nb, 8);                                   // qsc vsc
    add(nb, 4); add(nb, 4);                                   // used prow
    add((int64_t)nb * m * (m + 1), 16);                       // H
    add((int64_t)nb * m * (m + 1), 16);                       // Hraw
    add(nb, 8);                                               // beta
    add((int64_t)nb * m, 16); add((int64_t)nb * m, 16);       // cs sn
    add((int64_t)nb * (m + 1), 16);                           // g
    for (int i = 0; i < 4; ++i) add(nb, 4);
    for (int i = 0; i < 3; ++i) add(nb, 8);
    return bytes;
  }

  // Work arrays carved from the context's solver workspace (base null), or from base, which
  // must hold bytes_for(D, nb_, m_) bytes: a compacted block of the right-hand sides a restart
  // leaves active lives in the Krylov basis of the block it came from.
  void setup(gfcc_ctx* c, int nb_, int m_, int prec, bool tr, char* base = nullptr) {
    ctx = c;
    D = ctx->op.D;
    nb = nb_;
    m = m_;
    precision = prec;
    transpose = tr;
    const int64_t vec = D * nb;
    nblk_rows = row_blocks(D, nb);
    nbrows_y = (nb + CW - 1) / CW;
    const int64_t bytes = bytes_for(D, nb, m);
    if (!base) {
      ws_ensure(ctx, ctx->ws_solve, (size_t)bytes);
      base = ctx->ws_solve.as<char>();
    }
    char* cur = base;
    V = carve<double2>(cur, vec * (m + 1));
    W = carve<double2>(cur, vec);
    U = carve<double2>(cur, vec);
    X = carve<double2>(cur, vec);
    B = carve<double2>(cur, vec);
    R = carve<double2>(cur, vec);
    Hh = carve<double2>(cur, (int64_t)(m + 1) * nb);
    Hh2 = carve<double2>(cur, (int64_t)(m + 1) * nb);
    Y = carve<double2>(cur, (int64_t)m * nb);
    Cc = carve<double2>(cur, (int64_t)(m + 1) * nb);
    z = carve<double2>(cur, nb);
    nrm = carve<double>(cur, nb);
    part_n = carve<double>(cur, (int64_t)nblk_rows * nb);
    part_h = carve<double2>(cur, part_rows(nblk_rows) * nb);
    red = carve<double2>(cur, (int64_t)PSTR * nb);
    hsb = carve<double2>(cur, (int64_t)(FD + 1) * nb);
    scb = carve<double2>(cur, (int64_t)(FD + 1) * nb);
    tcb = carve<double2>(cur, (int64_t)(FD + 2) * nb);
    qsc = carve<double>(cur, nb);
    vsc = carve<double>(cur, nb);
    used = carve<int>(cur, nb);
    prow = carve<int>(cur, nb);
    s.H = carve<double2>(cur, (int64_t)nb * m * (m + 1));
    s.Hraw = carve<double2>(cur, (int64_t)nb * m * (m + 1));
    s.beta = carve<double>(cur, nb);
    s.cs = carve<double2>(cur, (int64_t)nb * m);
    s.sn = carve<double2>(cur, (int64_t)nb * m);
    s.g = carve<double2>(cur, (int64_t)nb * (m + 1));
    s.active = carve<int>(cur, nb);
    s.kend = carve<int>(cur, nb);
    s.its = carve<int>(cur, nb);
    s.brk = carve<int>(cur, nb);
    s.resest = carve<double>(cur, nb);
    s.thresh = carve<double>(cur, nb);
    s.inv = carve<double>(cur, nb);
    if (precision != GFCC_FP64) {
      ws_ensure(ctx, ctx->ws_solve_f32, sizeof(float) * (size_t)vec * 2 * 2);
      Uf = ctx->ws_solve_f32.as<float>();
      Sf = Uf + vec * 2;
    }
    if (nb > ctx->hflags_n) {
      drop_step_graphs(ctx);
      if (ctx->hflags) GFCC_HIP(hipHostFree(ctx->hflags));
      ctx->hflags = nullptr;
      ctx->dflags = nullptr;
      ctx->hflags_n = 0;
      GFCC_HIP(hipHostMalloc(reinterpret_cast<void**>(&ctx->hflags), sizeof(int) * 2 * (size_t)nb,
                             hipHostMallocMapped | hipHostMallocCoherent));
      GFCC_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&ctx->dflags), ctx->hflags, 0));
      ctx->hflags_n = nb;
    }
    hflags = ctx->hflags;
    dflags = ctx->dflags;
    for (hipEvent_t& e : flag_ev)
      if (!e) GFCC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }

  hipStream_t st() const { return ctx->stream; }

  // out[r] = ||Wv[:, r]||
  void norms(const double2* Wv, double* out) {
    hipLaunchKernelGGL(norm_kernel, dim3(nblk_rows, nbrows_y), dim3(CW), 0, st(), Wv, D, nb, part_n);
    GFCC_LAUNCH_CHECK();
    hipLaunchKernelGGL(norm_reduce, dim3(nbrows_y), dim3(256), 0, st(), part_n, nblk_rows, nb,
                       out);
    GFCC_LAUNCH_CHECK();
  }

  // h[j][r] = V_j^H W for j in [0, nj)
  void dots(int nj, double2* h) {
    for (int j0 = 0; j0 < nj; j0 += JG) {
      int cnt = std::min(JG, nj - j0);
      hipLaunchKernelGGL(dots_kernel, dim3(nblk_rows, nbrows_y), dim3(CW), 0, st(), V, D * nb,
                         j0, cnt, W, D, nb, part_h);
      GFCC_LAUNCH_CHECK();
      hipLaunchKernelGGL(dots_reduce_s<JG>, dim3(nbrows_y, cnt), dim3(256), 0, st(), part_h, nblk_rows,
                         j0, cnt, nb, h);
      GFCC_LAUNCH_CHECK();
    }
  }

  // Wv = M(omega) Uv = sigma(Uv) + z Uv ; sigma in FP64 when fp64 is set, else in the
  // block's precision
  // With shift false, only the sigma product is formed (the caller adds z U itself).
  void apply_M(const double2* Uv, double2* Wv, bool fp64, bool shift = true) {
    const int nc = 2 * nb;
    if (fp64 || precision == GFCC_FP64) {
      sigma_block_f64(ctx, nc, reinterpret_cast<const double*>(Uv), reinterpret_cast<double*>(Wv),
                      transpose);
    } else {
      const int64_t n = D * nc;
      hipLaunchKernelGGL(f64_to_f32_kernel, dim3(gridn(n)), dim3(256), 0, st(),
                         reinterpret_cast<const double*>(Uv), Uf, n);
      GFCC_LAUNCH_CHECK();
      sigma_block_f32(ctx, nc, Uf, Sf, precision);
      hipLaunchKernelGGL(f32_to_f64_kernel, dim3(gridn(n)), dim3(256), 0, st(), Sf,
                         reinterpret_cast<double*>(Wv), n);
      GFCC_LAUNCH_CHECK();
    }
    if (!shift) return;
    hipLaunchKernelGGL(shift_kernel, dim3(gridn(D * nb)), dim3(256), 0, st(), Wv, Uv, z, D, nb, Wv);
    GFCC_LAUNCH_CHECK();
  }

  // h[j][r] = sum over blocks of the partial dots of the fused kernels (nj <= FJ)
  void reduce_dots(int nj, double2* h) {
    hipLaunchKernelGGL(dots_reduce_s<FJ>, dim3(nbrows_y, nj), dim3(256), 0, st(), part_h, nblk_rows, 0,
                       nj, nb, h);
    GFCC_LAUNCH_CHECK();
  }
  // the delayed-reorthogonalisation reduction: nA pass-A rows, nB pass-B rows, nH rows of
  // Hbar s over the previous step's nh_s coefficients
  void dcgs_reduce(int nA, int nB, int nH, int nh_s) {
    hipLaunchKernelGGL(dcgs_reduce_kernel, dim3(nbrows_y, nA + nB + nH), dim3(256), 0, st(),
                       part_h, nblk_rows / 4, nA, nB, nh_s, nb, m, s.Hraw, scb, red, hsb);
    GFCC_LAUNCH_CHECK();
  }
  void reduce_norms(double* out) {
    hipLaunchKernelGGL(norm_reduce, dim3(nbrows_y), dim3(256), 0, st(), part_n, nblk_rows, nb,
                       out);
    GFCC_LAUNCH_CHECK();
  }
};

// Solve the systems of right-hand sides [r0, r0+nb) (global index r = w*np + k). On return
// gb.X holds the solutions (D-major block).
// X0: optional initial guesses [nrhs][D] (device); the first cycle then starts from the
// explicit residual b - M X0.
// Solves the right-hand sides r0 .. r0 + nb - 1 (or, with cols, the right-hand sides cols[r]
// of columns r, -1 for padding) of the block. X0: start iterates [nrhs][D]; x_ready: the
// block's X already holds them (a compacted block). its0: iterations already done per column.
static void solve_block(GmresBlock& gb, const double* omega, const int* pset, int np, int nrhs,
                        int r0, double eta, double tol, int maxit, std::vector<int>& its_out,
                        std::vector<double>& res_out, std::vector<int>& brk_out,
                        const double2* X0, const int* cols = nullptr, const int* its0 = nullptr,
                        bool x_ready = false) {
  gfcc_ctx* ctx = gb.ctx;
  const int nb = gb.nb, m = gb.m;
  const int64_t D = gb.D;
  hipStream_t st = ctx->stream;
  auto gidx = [&](int r) { return cols ? cols[r] : (r0 + r < nrhs ? r0 + r : -1); };
  std::vector<double2> hz(nb);
  std::vector<int> hp(nb);
  for (int r = 0; r < nb; ++r) {
    const int gr = gidx(r);
    if (gr >= 0) {
      hz[r] = make_double2(omega[gr / np], -eta);
      hp[r] = pset[gr % np];
    } else {
      hz[r] = make_double2(1.0, -eta);  // padding column: b = 0, done at once
      hp[r] = -1;
    }
  }
  GFCC_HIP(hipMemcpyAsync(gb.z, hz.data(), sizeof(double2) * nb, hipMemcpyHostToDevice, st));
  GFCC_HIP(hipMemcpyAsync(gb.prow, hp.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
  solve_rhs(ctx, gb.prow, gb.transpose, D, nb, gb.B);
  std::vector<double> bnorm(nb), rn(nb);
  gb.norms(gb.B, gb.nrm);
  GFCC_HIP(hipMemcpyAsync(bnorm.data(), gb.nrm, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
  if (!x_ready) {
    fill(ctx, reinterpret_cast<double*>(gb.X), D * nb * 2, 0.0);
    if (X0) {
      const int cnt = std::min(nb, nrhs - r0);
      ctranspose(ctx, X0 + (int64_t)r0 * D, cnt, D, D, gb.X, nb);
    }
  }
  std::vector<int> zeros(nb, 0);
  GFCC_HIP(hipMemcpyAsync(gb.s.brk, zeros.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
  GFCC_HIP(hipStreamSynchronize(st));

  std::vector<int> its(nb, 0), act(nb), brk(nb, 0);
  if (its0) std::copy(its0, its0 + nb, its.begin());
  std::vector<double> thr(nb), inv0(nb), rel(nb, 0.0);
  std::vector<double2> g0((size_t)nb * (m + 1));
  bool first = X0 == nullptr && !x_ready;
  bool handed = false;  // the active right-hand sides went on in a compacted block
  const bool mixed = gb.precision != GFCC_FP64;
  // small blocks (sigma work of a step below about 0.3 ms at 70 TF/s: 4 (ov)^2 o flops per
  // complex right-hand side in the ovvo product) read the convergence flags one step late
  const double ov = (double)ctx->op.OV;
  const bool late = (double)nb * 4.0 * ov * ov * (double)ctx->op.o < 2e10;
  const double inner_rel = 1e-4;  // relative tolerance of a reduced-precision cycle
  bool have_res = false;  // R holds the residual of X from the Arnoldi relation of the last cycle
  bool unit_start = false;  // this cycle starts from V0 = e_p (forward, x = 0)
  std::vector<double> hbeta(nb);
  std::vector<char> fin(nb, 0);  // stopped: its residual and iteration count are final
  auto explicit_residual = [&]() {
    gb.apply_M(gb.X, gb.U, true);
    hipLaunchKernelGGL(residual_kernel, dim3(gridn(D * nb)), dim3(256), 0, st, gb.B, gb.U,
                       D * nb, gb.R);
    GFCC_LAUNCH_CHECK();
  };
  auto stops = [&](int r, double rl) {
    return bnorm[r] == 0.0 || rl <= tol || its[r] >= maxit || brk[r];
  };
  for (;;) {
    // ---- residual R of the current X and its norm: b at the start, the explicit FP64
    // b - M X after a given x0 or a reduced-precision cycle, else the relation residual
    unit_start = first && !gb.transpose;
    if (first) {
      GFCC_HIP(hipMemcpyAsync(gb.R, gb.B, sizeof(double2) * D * nb, hipMemcpyDeviceToDevice, st));
    } else if (!have_res) {
      explicit_residual();
    }
    first = false;
    gb.norms(gb.R, gb.nrm);
    GFCC_HIP(hipMemcpyAsync(rn.data(), gb.nrm, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    GFCC_HIP(hipStreamSynchronize(st));
    if (have_res) {
      // The relation residual of a cycle equals b - M X up to the rounding of that cycle only
      // when the cycle started from an explicit (or exact) residual: carried from cycle to
      // cycle, its rounding accumulates, and next to a pole, after tens of short cycles, it
      // fell 30 times below the true residual. So it decides only for the right-hand sides it
      // stops; if another cycle is needed, every other one restarts from the explicit FP64
      // residual of its iterate (one sigma product per extra cycle; none when one cycle
      // suffices, as far from the poles).
      int more = 0;
      for (int r = 0; r < nb; ++r) {
        if (fin[r]) continue;
        const double rl = bnorm[r] > 0 ? rn[r] / bnorm[r] : 0.0;
        if (stops(r, rl)) {
          fin[r] = 1;
          rel[r] = rl;
        } else {
          ++more;
        }
      }
      // When at most half the block's columns (in 64-column groups) go on, they go on in a
      // compacted block carved from this block's Krylov basis: the next cycles sweep and
      // multiply only their columns. The compacted block starts from their iterates with the
      // explicit residual, as the restart here would.
      const int nb2 = std::max(CW, (more + CW - 1) / CW * CW);
      if (more && ctx->compact && 2 * nb2 <= nb &&
          GmresBlock::bytes_for(D, nb2, m) <= D * nb * (int64_t)(m + 1) * 16) {
        std::vector<int> cols2(nb2, -1), its2(nb2, 0), map(nb2, -1);
        int j = 0;
        for (int r = 0; r < nb; ++r) {
          if (fin[r]) continue;
          cols2[j] = gidx(r);
          its2[j] = its[r];
          map[j] = r;
          ++j;
        }
        GmresBlock gb2;
        gb2.setup(ctx, nb2, m, gb.precision, gb.transpose, reinterpret_cast<char*>(gb.V));
        GFCC_HIP(hipMemcpyAsync(gb.used, map.data(), sizeof(int) * nb2, hipMemcpyHostToDevice,
                                st));
        hipLaunchKernelGGL(pick_cols_kernel, dim3(gridn(D * nb2)), dim3(256), 0, st, gb.X, nb,
                           gb.used, nb2, D, gb2.X);
        GFCC_LAUNCH_CHECK();
        solve_block(gb2, omega, pset, np, nrhs, r0, eta, tol, maxit, its_out, res_out, brk_out,
                    nullptr, cols2.data(), its2.data(), true);
        hipLaunchKernelGGL(put_cols_kernel, dim3(gridn(D * nb2)), dim3(256), 0, st, gb2.X, nb2,
                           gb.used, nb, D, gb.X);
        GFCC_LAUNCH_CHECK();
        handed = true;
        break;
      }
      if (more) {
        explicit_residual();
        gb.norms(gb.R, gb.nrm);
        GFCC_HIP(hipMemcpyAsync(rn.data(), gb.nrm, sizeof(double) * nb, hipMemcpyDeviceToHost,
                                st));
        GFCC_HIP(hipStreamSynchronize(st));
      }
    }
    have_res = false;
    int nact = 0;
    for (int r = 0; r < nb; ++r) {
      if (!fin[r]) rel[r] = bnorm[r] > 0 ? rn[r] / bnorm[r] : 0.0;
      const bool done = fin[r] || stops(r, rel[r]);
      fin[r] = done ? 1 : 0;
      act[r] = done ? 0 : 1;
      nact += act[r];
      inv0[r] = act[r] ? 1.0 / rn[r] : 0.0;
      const double t_abs = 0.5 * tol * bnorm[r];
      thr[r] = mixed ? std::max(t_abs, inner_rel * rn[r]) : t_abs;
      for (int i = 0; i <= m; ++i) g0[(size_t)i * nb + r] = make_double2(0.0, 0.0);
      g0[r] = make_double2(act[r] ? rn[r] : 0.0, 0.0);
      hbeta[r] = act[r] ? rn[r] : 0.0;
    }
    if (nact == 0) break;
    // ---- cycle start: V0 = R / ||R||, g = (||R||, 0, ...)
    GFCC_HIP(hipMemcpyAsync(gb.s.active, act.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
    GFCC_HIP(hipMemcpyAsync(gb.used, act.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
    GFCC_HIP(hipMemcpyAsync(gb.s.thresh, thr.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
    GFCC_HIP(hipMemcpyAsync(gb.s.inv, inv0.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
    GFCC_HIP(hipMemcpyAsync(gb.s.g, g0.data(), sizeof(double2) * g0.size(), hipMemcpyHostToDevice, st));
    GFCC_HIP(hipMemcpyAsync(gb.s.beta, hbeta.data(), sizeof(double) * nb, hipMemcpyHostToDevice, st));
    GFCC_HIP(hipMemcpyAsync(gb.s.kend, zeros.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
    GFCC_HIP(hipMemcpyAsync(gb.s.its, its.data(), sizeof(int) * nb, hipMemcpyHostToDevice, st));
    // V0 = R / ||R|| and its preconditioned copy U
    hipLaunchKernelGGL(scale_precond_kernel, dim3(gridn(D * nb)), dim3(256), 0, st, gb.R, gb.s.inv,
                       ctx->op.diag.as<double>(), gb.z, D, nb, gb.V, gb.U);
    GFCC_LAUNCH_CHECK();
    int ksteps = 0;  // Arnoldi steps taken in this cycle (basis vectors that y can weight)
    const dim3 rgrid(gb.nblk_rows, gb.nbrows_y);
    const dim3 ugrid(gb.nblk_rows / 4, gb.nbrows_y);
    // flags written by the finishing kernel of step kk: is any RHS still active?
    auto any_active = [&](int kk) {
      GFCC_HIP(hipEventSynchronize(gb.flag_ev[kk & 1]));
      const volatile int* f = gb.hflags + (size_t)(kk & 1) * gb.nbrows_y;
      int any = 0;
      for (int b = 0; b < gb.nbrows_y; ++b) any |= f[b];
      return any != 0;
    };
    const bool delayed = m <= FD;
    if (delayed) {
      // Arnoldi with delayed reorthogonalisation: step k finalises column k - 1 and basis
      // vector k; the end of the cycle finalises column m - 1 and vector m
      bool stopped = false;
      const double* dg = ctx->op.diag.as<double>();
      const int64_t vs = D * nb;
      auto finish = [&](int j, int mode, int* fslot) {
        hipLaunchKernelGGL(dcgs_finish_kernel, dim3(gb.nbrows_y), dim3(CW), 0, st, j, m, nb,
                           maxit, mode, gb.s, gb.red, gb.hsb, gb.scb, gb.tcb, gb.qsc, gb.vsc,
                           fslot);
        GFCC_LAUNCH_CHECK();
      };
      // pass A of step k over Q_0 .. Q_{k-1}: beyond FJ vectors the older c = k - FJ first;
      // that sweep's pending-vector row c is then rewritten by the second one
      auto dots_sweep = [&](int k) {
        if (k <= FJ) {
          hipLaunchKernelGGL(Dcgs::dots[k], ugrid, dim3(256), 0, st, gb.V, vs, gb.W, gb.U, gb.z,
                             dg, D, nb, gb.part_h);
          GFCC_LAUNCH_CHECK();
          return;
        }
        const int c = k - FJ;
        hipLaunchKernelGGL(Dcgs::dots[c], ugrid, dim3(256), 0, st, gb.V, vs, gb.W, gb.U, gb.z,
                           dg, D, nb, gb.part_h);
        GFCC_LAUNCH_CHECK();
        hipLaunchKernelGGL(Dcgs::dots[FJ], ugrid, dim3(256), 0, st, gb.V + c * vs, vs, gb.W,
                           gb.U, gb.z, dg, D, nb, gb.part_h + (int64_t)c * nb);
        GFCC_LAUNCH_CHECK();
      };
      // pass B of step k (fin: the end of a cycle, q_k only). Beyond FJ vectors: the shares of
      // Q_0 .. Q_{c-1} go to the slot of q_k and to R (free between the start of a cycle and
      // its solution update), the sweep over the last FJ vectors completes q_k and the next
      // pending vector, and the dots of Q_0 .. Q_{c-1} with that vector follow
      auto update_sweep = [&](int k, bool fin) {
        if (k <= FJ) {
          hipLaunchKernelGGL(fin ? Dcgs::final_[k - 1] : Dcgs::update[k], ugrid, dim3(256), 0, st,
                             gb.V, vs, gb.W, gb.U, gb.z, dg, gb.scb, gb.tcb, gb.qsc, gb.vsc, D,
                             nb, gb.part_h, nullptr);
          GFCC_LAUNCH_CHECK();
          return;
        }
        const int c = k - FJ;
        hipLaunchKernelGGL(fin ? Dcgs::lin_final[c - 1] : Dcgs::lin[c - 1], ugrid, dim3(256), 0,
                           st, gb.V, vs, gb.scb, gb.tcb, D, nb, gb.V + k * vs, gb.R);
        GFCC_LAUNCH_CHECK();
        const DcgsUpdateFn later = fin ? dcgs_update_kernel<FJ, true, true>
                                       : dcgs_update_kernel<FJ, false, true>;
        hipLaunchKernelGGL(later, ugrid, dim3(256), 0, st, gb.V + c * vs, vs, gb.W, gb.U, gb.z, dg,
                           gb.scb + (int64_t)c * nb, gb.tcb + (int64_t)c * nb, gb.qsc, gb.vsc, D,
                           nb, gb.part_h + (int64_t)c * nb, gb.R);
        GFCC_LAUNCH_CHECK();
        if (fin) return;
        hipLaunchKernelGGL(Dcgs::vdots[c - 1], ugrid, dim3(256), 0, st, gb.V, vs, nullptr, gb.U,
                           gb.z, dg, D, nb, gb.part_h + (int64_t)PB * nb);
        GFCC_LAUNCH_CHECK();
      };
      auto final_vector = [&](int j) { update_sweep(j, true); };  // q_j = (vt_j - Q s) / rho
      // one step of a small block (flags read one step late): the operator product, pass A,
      // the reduction, the finishing kernel and pass B
      auto late_step = [&](int k) {
        int* fslot = gb.dflags + (size_t)(k & 1) * gb.nbrows_y;
        if (k == 0 && unit_start) {
          unit_sigma(ctx, gb.prow, gb.z, nb, gb.W);
        } else {
          gb.apply_M(gb.U, gb.W, false, false);
        }
        dots_sweep(k);
        gb.dcgs_reduce(k + 1, k >= 1 ? k + 1 : 0, k >= 2 ? k : 0, k - 1);
        finish(k, 0, fslot);
        update_sweep(k, false);
      };
      // The same step as a HIP graph, one per step shape, kept by the context: the first
      // sighting of a shape runs eagerly (it tunes products and sizes workspaces), the second
      // captures and launches, later ones launch. Not while a timer records launches (its
      // host-side bookkeeping runs per call).
      bool timing = false;
      for (const auto& t : ctx->timers) timing |= t.enabled;
      auto run_late_step = [&](int k) {
        if (!ctx->graphs || timing) {
          late_step(k);
          return;
        }
        const std::array<int64_t, 10> key{(int64_t)ctx->generation, ctx->op.o, ctx->op.v, nb, m,
                                          k, (k == 0 && unit_start) ? 1 : 0, gb.precision,
                                          gb.transpose ? 1 : 0, maxit};
        auto it = ctx->step_graphs.find(key);
        if (it != ctx->step_graphs.end()) {
          GFCC_HIP(hipGraphLaunch(it->second, st));
          return;
        }
        if (ctx->step_seen[key]++ == 0) {
          late_step(k);
          return;
        }
        // captured on a stream of the context's own (the library's stream may be the null
        // stream, on which capture is not permitted), launched on the library's stream
        if (!ctx->capture_stream)
          GFCC_HIP(hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking));
        const hipStream_t home = st;
        hipGraph_t g = nullptr;
        GFCC_HIP(hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeThreadLocal));
        ctx->stream = st = ctx->capture_stream;
        try {
          late_step(k);
        } catch (...) {
          ctx->stream = st = home;
          if (hipStreamEndCapture(ctx->capture_stream, &g) == hipSuccess && g)
            (void)hipGraphDestroy(g);
          throw;
        }
        ctx->stream = st = home;
        GFCC_HIP(hipStreamEndCapture(ctx->capture_stream, &g));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        GFCC_HIP(e);
        ctx->step_graphs[key] = ex;
        GFCC_HIP(hipGraphLaunch(ex, st));
      };
      for (int k = 0; k < m; ++k) {
        if (late) {
          // step k is queued before the flags of step k - 1 are read; when step k - 1 has
          // stopped every RHS (its columns reach k - 2), step k met only inactive ones
          run_late_step(k);
          GFCC_HIP(hipEventRecord(gb.flag_ev[k & 1], st));
          if (k > 0 && !any_active(k - 1)) {
            ksteps = k - 1;
            stopped = true;
            break;
          }
          continue;
        }
        int* fslot = gb.dflags + (size_t)(k & 1) * gb.nbrows_y;
        if (k > 0) {
          // large blocks: column k - 1 is finalised before the operator product of step k,
          // so a block whose right-hand sides have all stopped ends the cycle with one sweep
          // over the basis instead of another product
          gb.dcgs_reduce(0, k + 1, k >= 2 ? k : 0, k - 1);
          finish(k, 1, fslot);
          GFCC_HIP(hipEventRecord(gb.flag_ev[k & 1], st));
          if (!any_active(k)) {
            final_vector(k);
            ksteps = k;
            stopped = true;
            break;
          }
        }
        if (k == 0 && unit_start) {
          unit_sigma(ctx, gb.prow, gb.z, nb, gb.W);
        } else {
          gb.apply_M(gb.U, gb.W, false, false);
        }
        dots_sweep(k);
        gb.dcgs_reduce(k + 1, 0, 0, 0);
        finish(k, k == 0 ? 0 : 2, nullptr);
        update_sweep(k, false);
      }
      if (!stopped) {  // the end of the cycle: column m - 1 and basis vector m
        gb.dcgs_reduce(0, m + 1, m >= 2 ? m : 0, m - 1);
        finish(m, 1, nullptr);
        final_vector(m);
        ksteps = m;
      }
    }
    for (int k = 0; k < m && !delayed; ++k) {
      const int nj = k + 1;
      if (nj <= FJ) {
        // W = sigma(U); the shift, both Gram-Schmidt passes (CGS2) and the norm in three
        // fused sweeps over the basis; Hessenberg column = sum of both passes. The first
        // product of a cycle started from b = e_p is a column of Hbar_N.
        if (k == 0 && unit_start) {
          unit_sigma(ctx, gb.prow, gb.z, nb, gb.W);
        } else {
          gb.apply_M(gb.U, gb.W, false, false);
        }
        hipLaunchKernelGGL(Fused::shift_dots[nj - 1], rgrid, dim3(CW), 0, st, gb.V, D * nb, gb.U,
                           gb.z, gb.W, D, nb, gb.part_h);
        GFCC_LAUNCH_CHECK();
        gb.reduce_dots(nj, gb.Hh);
        hipLaunchKernelGGL(Fused::update_dots[nj - 1], rgrid, dim3(CW), 0, st, gb.V, D * nb,
                           gb.Hh, gb.W, D, nb, gb.part_h);
        GFCC_LAUNCH_CHECK();
        gb.reduce_dots(nj, gb.Hh2);
        hipLaunchKernelGGL(Fused::update_norm[nj - 1], rgrid, dim3(CW), 0, st, gb.V, D * nb,
                           gb.Hh2, gb.W, D, nb, gb.part_n);
        GFCC_LAUNCH_CHECK();
        gb.reduce_norms(gb.nrm);
      } else {
        gb.apply_M(gb.U, gb.W, false);
        gb.dots(nj, gb.Hh);
        hipLaunchKernelGGL(update_kernel, dim3(gridn(D * nb)), dim3(256), 0, st, gb.V, D * nb,
                           nj, gb.Hh, D, nb, gb.W);
        GFCC_LAUNCH_CHECK();
        gb.dots(nj, gb.Hh2);
        hipLaunchKernelGGL(update_kernel, dim3(gridn(D * nb)), dim3(256), 0, st, gb.V, D * nb,
                           nj, gb.Hh2, D, nb, gb.W);
        GFCC_LAUNCH_CHECK();
        gb.norms(gb.W, gb.nrm);
      }
      int* fslot = late ? gb.dflags + (size_t)(k & 1) * gb.nbrows_y : nullptr;
      hipLaunchKernelGGL(arnoldi_finish_kernel, dim3(gb.nbrows_y), dim3(CW), 0, st, gb.Hh,
                         gb.Hh2, gb.nrm, k, m, nb, maxit, gb.s, fslot);
      GFCC_LAUNCH_CHECK();
      // V_{k+1} and the preconditioned input of the next step
      hipLaunchKernelGGL(scale_precond_kernel, dim3(gridn(D * nb)), dim3(256), 0, st, gb.W,
                         gb.s.inv, ctx->op.diag.as<double>(), gb.z, D, nb,
                         gb.V + (int64_t)(k + 1) * D * nb, gb.U);
      GFCC_LAUNCH_CHECK();
      if (late) {
        // Step k is queued before the flags of step k - 1 are read, so the GPU does not wait
        // for the host. When step k - 1 has stopped every right-hand side, step k only met
        // inactive ones (their next basis vectors and inputs are zero, their state is left
        // alone) and does not count.
        GFCC_HIP(hipEventRecord(gb.flag_ev[k & 1], st));
        if (k > 0 && !any_active(k - 1)) break;
        ksteps = k + 1;
        continue;
      }
      ksteps = k + 1;
      GFCC_HIP(hipMemcpyAsync(act.data(), gb.s.active, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
      GFCC_HIP(hipStreamSynchronize(st));
      int any = 0;
      for (int r = 0; r < nb; ++r) any |= act[r];
      if (!any) break;
    }
    // ---- solution update x += P^{-1} V y (y is zero beyond each right-hand side's kend,
    // and kend <= ksteps)
    if (m <= 32) {
      hipLaunchKernelGGL(ysolve32_kernel, dim3((nb + 1) / 2), dim3(64), 0, st, m, nb, gb.s,
                         gb.used, gb.Y);
    } else {
      hipLaunchKernelGGL(ysolve_kernel, dim3(blocks_for(nb, 64)), dim3(64), 0, st, m, nb, gb.s,
                         gb.used, gb.Y);
    }
    GFCC_LAUNCH_CHECK();
    if (!mixed) {
      // FP64: the update and the residual of the updated X (Arnoldi relation) in one pass
      if (m <= 32) {
        hipLaunchKernelGGL(rescoef64_kernel, dim3(nb), dim3(64), 0, st, m, nb, gb.s, gb.used,
                           gb.Y, gb.Cc);
      } else {
        hipLaunchKernelGGL(rescoef_kernel, dim3(blocks_for(nb, 64)), dim3(64), 0, st, m, nb, gb.s,
                           gb.used, gb.Y, gb.Cc);
      }
      GFCC_LAUNCH_CHECK();
      hipLaunchKernelGGL(xupdate_res_kernel, dim3(gridn(D * nb)), dim3(256), 0, st, gb.V, D * nb,
                         ksteps, gb.Y, gb.Cc, gb.used, ctx->op.diag.as<double>(), gb.z, D, nb,
                         gb.X, gb.R);
      GFCC_LAUNCH_CHECK();
      have_res = true;
    } else {
      hipLaunchKernelGGL(xupdate_kernel, dim3(gridn(D * nb)), dim3(256), 0, st, gb.V, D * nb,
                         ksteps, gb.Y, ctx->op.diag.as<double>(), gb.z, D, nb, gb.X);
      GFCC_LAUNCH_CHECK();
    }
    GFCC_HIP(hipMemcpyAsync(its.data(), gb.s.its, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
    GFCC_HIP(hipMemcpyAsync(brk.data(), gb.s.brk, sizeof(int) * nb, hipMemcpyDeviceToHost, st));
    GFCC_HIP(hipStreamSynchronize(st));
  }
  for (int r = 0; r < nb; ++r) {
    const int gr = gidx(r);
    if (gr < 0 || (handed && !fin[r])) continue;  // padding, or finished in the compacted block
    its_out[gr] = its[r];
    res_out[gr] = rel[r];
    brk_out[gr] = brk[r];
  }
}

// Full driver shared by gfcc_solve and the reduced-order model: solves every (omega, p),
// writes G (device, [nw][np][np]) and optionally X ([nw][np][D] device).
void unit_sigma(gfcc_ctx* ctx, const int* prow, const void* z, int nb, void* W) {
  const Operator& op = ctx->op;
  hipLaunchKernelGGL(unit_sigma_kernel, dim3(gridn(op.D * nb)), dim3(256), 0, ctx->stream, prow,
                     op.f64.W1.as<double>(), op.f64.W4c.as<double>(), (int64_t)(op.o + op.v),
                     op.diag.as<double>(), static_cast<const double2*>(z), op.o, op.D, nb,
                     static_cast<double2*>(W));
  GFCC_LAUNCH_CHECK();
}

void solve_rhs(gfcc_ctx* ctx, const int* prow, bool transpose, int64_t D, int nb, void* B) {
  hipLaunchKernelGGL(rhs_kernel, dim3(gridn(D * nb)), dim3(256), 0, ctx->stream, prow,
                     ctx->op.Crows.as<double>(), transpose ? 1 : 0, D, nb,
                     static_cast<double2*>(B));
  GFCC_LAUNCH_CHECK();
}

gfcc_status solve_all(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                      double eta, double tol, int maxit, int restart, int block, int precision,
                      int transpose, void* X_out, void* G_out, int* iters_out, double* resid_out,
                      const void* X0, int ndiis, double* hist) {
  Operator& op = ctx->op;
  const int64_t D = op.D;
  const int nrhs = nw * np;
  int nb = block > 0 ? block : std::min(nrhs, 128);
  nb = std::max(1, std::min(nb, nrhs));
  // a block holding every right-hand side is padded to a multiple of 64 (zero right-hand
  // sides) when that adds at most a quarter, which keeps the column-block ovvo loader
  if (nb == nrhs) {
    const int r = (nrhs + 63) / 64 * 64;
    if (r != nrhs && (int64_t)r * 4 <= (int64_t)nrhs * 5) nb = r;
  }
  GFCC_REQUIRE(nb <= 2048, GFCC_EINVAL, "gfcc_solve: block too large");
  const bool diis = ndiis > 0;
  GmresBlock gb;
  DiisWork dw;
  if (!diis) gb.setup(ctx, nb, restart, precision, transpose != 0);
  std::vector<int> its(nrhs, 0), brk(nrhs, 0);
  std::vector<double> res(nrhs, 0.0);
  // rows used for G: c_q rows (forward) or the 1h entries q (transpose)
  DevBuf bq, bC, bG;
  bq.alloc(sizeof(int) * np);
  GFCC_HIP(hipMemcpyAsync(bq.p, p, sizeof(int) * np, hipMemcpyHostToDevice, ctx->stream));
  if (!transpose) {
    bC.alloc(sizeof(double) * (size_t)np * D);
    hipLaunchKernelGGL(copy_rows_kernel, dim3(gridn((int64_t)np * D)), dim3(256), 0, ctx->stream,
                       op.Crows.as<double>(), bq.as<int>(), np, D, bC.as<double>());
    GFCC_LAUNCH_CHECK();
  }
  bG.alloc(sizeof(double2) * (size_t)np * nb);
  for (int r0 = 0; r0 < nrhs;) {
    // the last block is only as wide as the right-hand sides left, rounded up to a multiple
    // of 64 (which keeps the column-block ovvo kernel); padding columns have b = 0
    const int left = nrhs - r0;
    if (left < nb) {
      const int nbl = std::min(nb, (left + 63) / 64 * 64);
      if (nbl != nb) {
        nb = nbl;
        if (!diis) gb.setup(ctx, nb, restart, precision, transpose != 0);
      }
    }
    const int nbb = nb;
    const double2* Xb;
    if (diis) {
      Xb = static_cast<const double2*>(diis_block(ctx, dw, nbb, ndiis, omega, p, np, nrhs, r0,
                                                  eta, tol, maxit, transpose != 0, its.data(),
                                                  res.data(), hist, X0));
    } else {
      solve_block(gb, omega, p, np, nrhs, r0, eta, tol, maxit, its, res, brk,
                  static_cast<const double2*>(X0));
      Xb = gb.X;
    }
    // G rows for this block
    if (!transpose) {
      gemm<double>(ctx, false, false, np, 2 * nbb, (int)D, 1.0, bC.as<double>(), D,
                   reinterpret_cast<const double*>(Xb), 2 * nbb, 0.0, bG.as<double>(), 2 * nbb);
    } else {
      hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for((int64_t)np * nbb, 256)), dim3(256),
                         0, ctx->stream, Xb, bq.as<int>(), np, nbb, bG.as<double2>());
      GFCC_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(scatter_G_kernel, dim3(blocks_for((int64_t)np * nbb, 256)), dim3(256), 0,
                       ctx->stream, bG.as<double2>(), np, nbb, r0, nrhs, np, transpose,
                       static_cast<double2*>(G_out));
    GFCC_LAUNCH_CHECK();
    if (X_out) {
      int cnt = std::min(nbb, nrhs - r0);
      ctranspose(ctx, Xb, D, cnt, nbb, static_cast<double2*>(X_out) + (int64_t)r0 * D, D);
    }
    r0 += nbb;
  }
  GFCC_HIP(hipStreamSynchronize(ctx->stream));
  timers_collect(ctx);
  bool noconv = false, anybrk = false;
  for (int r = 0; r < nrhs; ++r) {
    if (iters_out) iters_out[r] = its[r];
    if (resid_out) resid_out[r] = res[r];
    if (brk[r]) anybrk = true;
    if (!(res[r] <= tol)) noconv = true;
  }
  if (anybrk) {
    ctx->last_error = "gfcc_solve: singular shifted operator on a Krylov space";
    return GFCC_EBREAKDOWN;
  }
  if (noconv) {
    ctx->last_error = "gfcc_solve: some right-hand sides did not reach the tolerance";
    return GFCC_ENOCONV;
  }
  return GFCC_OK;
}

namespace {

// S[d] = sum_r weight_{w(r)} Im(Y[r][d] X[r][d])
__global__ void grad_rows_kernel(const double2* __restrict__ X, const double2* __restrict__ Y,
                                 const double* __restrict__ wt, int nw, int np, int64_t D,
                                 double* __restrict__ S) {
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < D;
       d += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int w = 0; w < nw; ++w) {
      double aw = 0.0;
      for (int k = 0; k < np; ++k) {
        int64_t off = ((int64_t)w * np + k) * D + d;
        double2 y = Y[off], x = X[off];
        aw += y.x * x.y + y.y * x.x;
      }
      acc += wt[w] * aw;
    }
    S[d] = acc;
  }
}

// grad[m] for occupied m: (1/pi) (S[m] + sum_{pairs with m} sum_a S[...]);
// grad[o+a] for virtual a: -(1/pi) sum_pairs S[o + pr v + a]
__global__ void grad_bins_kernel(const double* __restrict__ S, int o, int v,
                                 double* __restrict__ grad) {
  __shared__ double red[256];
  const int orb = blockIdx.x;
  const int64_t P = (int64_t)o * (o - 1) / 2;
  double acc = 0.0;
  if (orb < o) {
    const int mm = orb;
    const int64_t nterm = (int64_t)(o - 1) * v;
    for (int64_t t = threadIdx.x; t < nterm; t += blockDim.x) {
      int kk = (int)(t / v), a = (int)(t % v);
      int k = kk < mm ? kk : kk + 1;
      int64_t pr = k < mm ? pair_of(k, mm, o) : pair_of(mm, k, o);
      acc += S[o + pr * v + a];
    }
    if (threadIdx.x == 0) acc += S[mm];
  } else {
    const int a = orb - o;
    for (int64_t pr = threadIdx.x; pr < P; pr += blockDim.x) acc += S[o + pr * v + a];
    acc = -acc;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) grad[orb] = red[0] / 3.14159265358979323846;
}

__global__ void spectral_kernel(const double2* __restrict__ G, int nw, int np, double* __restrict__ A) {
  int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nw) return;
  double s = 0.0;
  for (int k = 0; k < np; ++k) s += G[((int64_t)w * np + k) * np + k].y;
  A[w] = s / 3.14159265358979323846;
}

// J = (1/pi) sum_w wt[w] sum_k Im G[w][k][k]: one workgroup, a fixed order of summation
__global__ void weighted_spectral_kernel(const double2* __restrict__ G, int nw, int np,
                                         const double* __restrict__ wt, double* __restrict__ J) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int w = threadIdx.x; w < nw; w += blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < np; ++k) s += G[((int64_t)w * np + k) * np + k].y;
    acc += wt[w] * s;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *J = red[0] / 3.14159265358979323846;
}

}  // namespace
}  // namespace gfcc

namespace gfcc {
// argument checks shared by gfcc_solve and gfcc_solve_x0 (throws Error)
static void check_solve_args(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                             double eta, double tol, int maxit, int restart, int precision,
                             int transpose, const void* G_out) {
  GFCC_REQUIRE(ctx->op.built, GFCC_ESTATE, "gfcc_solve: no operator built");
  GFCC_REQUIRE(nw >= 0 && np >= 0, GFCC_EINVAL, "gfcc_solve: negative sizes");
  if (nw == 0 || np == 0) return;
  GFCC_REQUIRE(omega && p && G_out, GFCC_EINVAL, "gfcc_solve: null pointer");
  GFCC_REQUIRE((int64_t)nw * np < (1LL << 30), GFCC_EINVAL, "gfcc_solve: too many right-hand sides");
  GFCC_REQUIRE(eta >= 0.0 && std::isfinite(eta), GFCC_EINVAL, "gfcc_solve: eta must be >= 0");
  GFCC_REQUIRE(tol > 0.0 && tol < 1.0, GFCC_EINVAL, "gfcc_solve: tol must be in (0, 1)");
  GFCC_REQUIRE(maxit >= 1, GFCC_EINVAL, "gfcc_solve: maxit must be >= 1");
  GFCC_REQUIRE(restart >= 1 && restart <= 200, GFCC_EINVAL, "gfcc_solve: restart in [1, 200]");
  GFCC_REQUIRE(precision >= GFCC_FP64 && precision <= GFCC_BF16_PAIRS, GFCC_EINVAL,
               "gfcc_solve: unknown precision");
  GFCC_REQUIRE(precision == GFCC_FP64 || (ctx->op.keep & GFCC_KEEP_FP32), GFCC_ESTATE,
               "gfcc_solve: reduced precision needs GFCC_KEEP_FP32 at build time");
  GFCC_REQUIRE(!(transpose && precision != GFCC_FP64), GFCC_EINVAL,
               "gfcc_solve: the transpose solve is FP64 only");
  for (int w = 0; w < nw; ++w)
    GFCC_REQUIRE(std::isfinite(omega[w]), GFCC_EINVAL, "gfcc_solve: non-finite omega");
  std::vector<char> seen(ctx->op.o, 0);
  for (int k = 0; k < np; ++k) {
    GFCC_REQUIRE(p[k] >= 0 && p[k] < ctx->op.o, GFCC_EINVAL,
                 "gfcc_solve: p must be occupied orbitals 0 <= p < o");
    GFCC_REQUIRE(!seen[p[k]], GFCC_EINVAL, "gfcc_solve: repeated orbital in p");
    seen[p[k]] = 1;
  }
  if (eta == 0.0) {
    // Without broadening the shifted operator is real, and omega + diag(Hbar_N) can vanish
    // (for T = V = 0 exactly at omega = eps_i, a pole): the Jacobi preconditioner diag(M) does
    // not exist there, and for a diagonal operator M itself is singular. Checked before any
    // solve; the outputs are left untouched.
    const Operator& op = ctx->op;
    std::vector<double> dg((size_t)op.D);
    GFCC_HIP(hipMemcpyAsync(dg.data(), op.diag.p, sizeof(double) * (size_t)op.D,
                            hipMemcpyDeviceToHost, ctx->stream));
    GFCC_HIP(hipStreamSynchronize(ctx->stream));
    std::sort(dg.begin(), dg.end());
    for (int w = 0; w < nw; ++w)
      if (std::binary_search(dg.begin(), dg.end(), -omega[w]))
        throw Error(GFCC_EBREAKDOWN, "gfcc_solve: eta = 0 and a diagonal entry of the shifted "
                                     "operator is zero at omega = " + std::to_string(omega[w]));
  }
}
}  // namespace gfcc

extern "C" {

gfcc_status gfcc_solve(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                       double eta, double tol, int maxit, int restart, int block, int precision,
                       int transpose, void* X_out, void* G_out, int* iters_out,
                       double* resid_out) {
  if (!ctx) return GFCC_EINVAL;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_HIP(hipSetDevice(ctx->device));
  check_solve_args(ctx, nw, omega, np, p, eta, tol, maxit, restart, precision, transpose, G_out);
  if (nw == 0 || np == 0) return GFCC_OK;
  return solve_all(ctx, nw, omega, np, p, eta, tol, maxit, restart, block, precision, transpose,
                   X_out, G_out, iters_out, resid_out, nullptr);
  GFCC_API_END(ctx)
}

gfcc_status gfcc_solve_x0(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                          double eta, double tol, int maxit, int restart, int block,
                          int precision, int transpose, const void* X0, void* X_out,
                          void* G_out, int* iters_out, double* resid_out) {
  if (!ctx) return GFCC_EINVAL;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_HIP(hipSetDevice(ctx->device));
  check_solve_args(ctx, nw, omega, np, p, eta, tol, maxit, restart, precision, transpose, G_out);
  if (nw == 0 || np == 0) return GFCC_OK;
  GFCC_REQUIRE(X0 != nullptr, GFCC_EINVAL, "gfcc_solve_x0: null X0");
  if (X_out) {
    const size_t bytes = sizeof(double2) * (size_t)nw * np * (size_t)ctx->op.D;
    const char* a = static_cast<const char*>(X0);
    const char* b = static_cast<const char*>(X_out);
    GFCC_REQUIRE(a + bytes <= b || b + bytes <= a, GFCC_EINVAL,
                 "gfcc_solve_x0: X0 and X_out overlap");
  }
  return solve_all(ctx, nw, omega, np, p, eta, tol, maxit, restart, block, precision, transpose,
                   X_out, G_out, iters_out, resid_out, X0);
  GFCC_API_END(ctx)
}

gfcc_status gfcc_solve_diis(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                            double eta, double tol, int maxit, int ndiis, int block,
                            int transpose, const void* X0, void* X_out, void* G_out,
                            int* iters_out, double* resid_out, double* hist_out) {
  if (!ctx) return GFCC_EINVAL;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_HIP(hipSetDevice(ctx->device));
  check_solve_args(ctx, nw, omega, np, p, eta, tol, maxit, 1, GFCC_FP64, transpose, G_out);
  if (nw == 0 || np == 0) return GFCC_OK;
  GFCC_REQUIRE(ndiis >= 1 && ndiis <= 16, GFCC_EINVAL,
               "gfcc_solve_diis: ndiis must be in [1, 16]");
  if (X0 && X_out) {
    const size_t bytes = sizeof(double2) * (size_t)nw * np * (size_t)ctx->op.D;
    const char* a = static_cast<const char*>(X0);
    const char* b = static_cast<const char*>(X_out);
    GFCC_REQUIRE(a + bytes <= b || b + bytes <= a, GFCC_EINVAL,
                 "gfcc_solve_diis: X0 and X_out overlap");
  }
  return solve_all(ctx, nw, omega, np, p, eta, tol, maxit, 1, block, GFCC_FP64, transpose, X_out,
                   G_out, iters_out, resid_out, X0, ndiis, hist_out);
  GFCC_API_END(ctx)
}

gfcc_status gfcc_grad_eps(gfcc_ctx* ctx, int nw, const double* weight, int np, const void* X,
                          const void* Y, double* grad_out) {
  if (!ctx) return GFCC_EINVAL;
  GFCC_API_BEGIN(ctx)
  using namespace gfcc;
  GFCC_REQUIRE(ctx->op.built, GFCC_ESTATE, "gfcc_grad_eps: no operator built");
  GFCC_REQUIRE(nw >= 1 && np >= 1 && weight && X && Y && grad_out, GFCC_EINVAL,
               "gfcc_grad_eps: bad arguments");
  const int o = ctx->op.o, v = ctx->op.v;
  const int64_t D = ctx->op.D;
  DevBuf bw, bS, bg;
  bw.alloc(sizeof(double) * nw);
  bS.alloc(sizeof(double) * D);
  bg.alloc(sizeof(double) * (o + v));
  GFCC_HIP(hipMemcpyAsync(bw.p, weight, sizeof(double) * nw, hipMemcpyHostToDevice, ctx->stream));
  hipLaunchKernelGGL(grad_rows_kernel, dim3(gridn(D)), dim3(256), 0, ctx->stream,
                     static_cast<const double2*>(X), static_cast<const double2*>(Y), bw.as<double>(),
                     nw, np, D, bS.as<double>());
  GFCC_LAUNCH_CHECK();
  hipLaunchKernelGGL(grad_bins_kernel, dim3(o + v), dim3(256), 0, ctx->stream, bS.as<double>(),
                     o, v, bg.as<double>());
  GFCC_LAUNCH_CHECK();
  GFCC_HIP(hipMemcpyAsync(grad_out, bg.p, sizeof(double) * (o + v), hipMemcpyDeviceToHost,
                          ctx->stream));
  GFCC_HIP(hipStreamSynchronize(ctx->stream));
  GFCC_API_END(ctx)
}

gfcc_status spectral_weight(int nw, int np, const void* G, int is_device, const double* weight,
                            double* J_out) {
  if (nw < 0 || np < 0 || !J_out || (nw > 0 && (!weight || (np > 0 && !G)))) return GFCC_EINVAL;
  *J_out = 0.0;
  if (nw == 0 || np == 0) return GFCC_OK;
  const size_t gbytes = sizeof(double2) * (size_t)nw * np * np;
  double* dw = nullptr;   // [nw] weights, then J
  void* dG = nullptr;
  if (hipMalloc(&dw, sizeof(double) * ((size_t)nw + 1)) != hipSuccess) return GFCC_ENOMEM;
  hipError_t e = hipMemcpy(dw, weight, sizeof(double) * nw, hipMemcpyHostToDevice);
  if (e == hipSuccess && !is_device) {
    e = hipMalloc(&dG, gbytes);
    if (e == hipSuccess) e = hipMemcpy(dG, G, gbytes, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(gfcc::weighted_spectral_kernel, dim3(1), dim3(256), 0, nullptr,
                       static_cast<const double2*>(is_device ? G : dG), nw, np, dw, dw + nw);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(J_out, dw + nw, sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(dw);
  if (dG) (void)hipFree(dG);
  if (e == hipErrorOutOfMemory) return GFCC_ENOMEM;
  return e == hipSuccess ? GFCC_OK : GFCC_EHIP;
}

gfcc_status spectral_function(int nw, int np, const void* G, int is_device, double* A_out) {
  if (nw < 0 || np < 0 || (nw > 0 && (!A_out || (np > 0 && !G)))) return GFCC_EINVAL;
  if (nw == 0) return GFCC_OK;
  // a host G is copied to the device: the sum runs in the same kernel either way
  const size_t gbytes = sizeof(double2) * (size_t)nw * np * np;
  double* dA = nullptr;
  void* dG = nullptr;
  if (hipMalloc(&dA, sizeof(double) * nw) != hipSuccess) return GFCC_ENOMEM;
  hipError_t e = hipSuccess;
  if (!is_device && gbytes > 0) {
    e = hipMalloc(&dG, gbytes);
    if (e == hipSuccess) e = hipMemcpy(dG, G, gbytes, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(gfcc::spectral_kernel, dim3((nw + 255) / 256), dim3(256), 0, nullptr,
                       static_cast<const double2*>(is_device ? G : dG), nw, np, dA);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpy(A_out, dA, sizeof(double) * nw, hipMemcpyDeviceToHost);
  (void)hipFree(dA);
  if (dG) (void)hipFree(dG);
  if (e == hipErrorOutOfMemory) return GFCC_ENOMEM;
  return e == hipSuccess ? GFCC_OK : GFCC_EHIP;
}

}  // extern "C"
