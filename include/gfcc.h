/*
 * gfcc.h -- C ABI of the MI355X IP-GFCC solver library (libgfcc.so).
 *
 * The library computes the retarded coupled-cluster Green's function in the ionisation
 * (N-1 electron) sector by solving the shifted linear systems of the GFCC method
 *   ( omega - i*eta + Hbar_N ) X_p(omega) = b_p                  (Peng et al., Eq. xplin)
 *   G_qp(omega) = c_q^T X_p(omega)                                (Eq. gfcclineqn)
 *   A(omega)    = (1/pi) sum_p Im G_pp(omega)                     (spectral function)
 * and by projecting them onto a reduced-order model (Eq. model, Methodology section).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Orbitals: spin orbitals; o occupied (indices i,j,k,l,m,n < o), v virtual (a..f < v).
 * Vector space of X_p (Eq. xp): D = o + o(o-1)/2 * v. Packed layout of one vector:
 *   x[i]                           one-hole amplitude x^i, 0 <= i < o
 *   x[o + pi(i,j)*v + a]           two-hole-one-particle amplitude x^{ij}_a, i < j,
 *   pi(i,j) = i*o - i*(i+1)/2 + (j - i - 1)   (lexicographic pairs, a fastest).
 * Complex vectors are interleaved complex128 (re, im), as torch.complex128 stores them.
 * Integral blocks: full antisymmetrised spin-orbital blocks <pq||rs>, row-major, named by
 *   occupancy; e.g. ovvo[m][b][e][j] = <m b || e j>. They must satisfy
 *   <pq||rs> = -<qp||rs> = -<pq||sr> = <rs||pq>.
 * Amplitudes: t1[i][a], t2[i][j][a][b] (antisymmetric in ij and in ab), l1, l2 likewise
 *   (Lambda stored in the same index order as T).
 * Pointers: unless marked "host", every array argument is a DEVICE pointer on the context's
 *   device. The caller owns all buffers passed in; the context owns the operator it builds.
 * Streams: all work is enqueued on the stream given to gfcc_create. Entry points that
 *   return host results synchronise that stream before returning.
 * Errors: no exception crosses the ABI. Every call returns a gfcc_status; on failure
 *   gfcc_last_error(ctx) holds a message. Inputs are validated before any kernel launch.
 * Threads: a context must not be used from two host threads at once.
 */
#ifndef GFCC_H
#define GFCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gfcc_ctx gfcc_ctx;
typedef struct gfcc_mor gfcc_mor;

typedef enum {
  GFCC_OK = 0,
  GFCC_EINVAL = 1,      /* bad argument (sizes, indices, null pointers, non-finite data) */
  GFCC_ENOMEM = 2,      /* device allocation failed or a size limit was exceeded */
  GFCC_EHIP = 3,        /* a HIP runtime call failed */
  GFCC_ENOCONV = 4,     /* an iterative solve stopped at maxit above its tolerance */
  GFCC_EBREAKDOWN = 5,  /* a shifted operator is exactly singular for some right-hand side */
  GFCC_ESTATE = 6       /* called in the wrong state (e.g. no operator built yet) */
} gfcc_status;

/* Arithmetic of the sigma product (H-bar times a block of vectors). */
enum {
  GFCC_FP64 = 0,            /* all terms in FP64 (MFMA f64) */
  GFCC_FP32 = 1,            /* all terms in FP32 (MFMA f32, FP32 accumulation) */
  GFCC_FP32_BF16_3BODY = 2, /* FP32, with the three-body T2*<kl||cd> term on BF16 MFMA */
  GFCC_BF16_PAIRS = 3       /* FP32, with the ovvo contraction (T5, T6, T8 through Weff, most
                               of the flops) on BF16 MFMA with two-term operands x = hi + lo
                               (hi.hi + hi.lo + lo.hi, FP32 accumulation, about 16 bits) when
                               2 * nrhs of a block is a multiple of 128 and v >= 32, on FP32
                               MFMA otherwise */
};

/* Bit mask for build_hbar_operands: which operator copies to keep on the device. */
enum {
  GFCC_KEEP_FP64 = 1,       /* always kept */
  GFCC_KEEP_FP32 = 2,       /* FP32 copies and BF16 pairs (three-body, Weff) for mixed solves */
  GFCC_KEEP_TRANSPOSE = 4   /* transposed copies for fast H-bar^T products (adjoint) */
};

/* Dimension D of the packed IP vector space for o occupied and v virtual spin orbitals. */
int64_t gfcc_dim(int o, int v);

/* Create a context on HIP device `device` that enqueues on `hip_stream` (a hipStream_t; NULL
 * means the device's null stream). */
gfcc_status gfcc_create(gfcc_ctx** ctx, int device, void* hip_stream);

/* Free the context, its operator and all device memory it owns. NULL is accepted. */
gfcc_status gfcc_destroy(gfcc_ctx* ctx);

/* Message of the last failed call on ctx ("" if none). Valid until the next call on ctx. */
const char* gfcc_last_error(const gfcc_ctx* ctx);

/*
 * build_hbar_operands -- form the similarity-transformed Hamiltonian blocks that the sigma
 * product needs (the transform Hbar = e^{-T} H e^{T} defined under Eq. gfxn1) and keep them
 * on the device.
 *
 * eps [o+v] orbital energies (the Fock matrix is diag(eps)); t1 [o][v]; t2 [o][o][v][v];
 * l1 [o][v]; l2 [o][o][v][v]; oooo [o][o][o][o]; ooov [o][o][o][v]; oovv [o][o][v][v];
 * ovvo [o][v][v][o]; ovvv [o][v][v][v]. All FP64, device pointers, read only during the
 * call. precision_mask: GFCC_KEEP_* bits. Replaces any operator built before; a rebuild
 * reuses the previous operator's device buffers where the sizes match, and the context keeps
 * the build's work arrays (about 6 o^2 v^2 doubles) for the next build while they total at
 * most 8 GiB (gfcc_destroy frees them).
 * Errors: EINVAL for o < 2, v < 1, null pointers or non-finite entries (checked on the
 * device); ENOMEM if the operator does not fit.
 */
gfcc_status build_hbar_operands(gfcc_ctx* ctx, int o, int v, const double* eps,
                                const double* t1, const double* t2, const double* l1,
                                const double* l2, const double* oooo, const double* ooov,
                                const double* oovv, const double* ovvo, const double* ovvv,
                                int precision_mask);

/*
 * build_hbar_first_order -- build_hbar_operands with T and Lambda replaced by their
 * first-order perturbative terms (the variant of the Conclusions, after Nooijen and Snijders,
 * which skips the CC ground state): t1 = l1 = 0 and
 * t2[i][j][a][b] = l2[i][j][a][b] = oovv[i][j][a][b] / (eps_i + eps_j - eps_a - eps_b), formed
 * on the device from the Moller-Plesset partitioning of the diagonal Fock matrix diag(eps).
 * Arguments as build_hbar_operands (no amplitudes). The amplitudes are temporary (o^2 v^2
 * doubles during the call). Errors: as build_hbar_operands, and EINVAL unless every occupied
 * energy lies below every virtual one (no vanishing denominator).
 */
gfcc_status build_hbar_first_order(gfcc_ctx* ctx, int o, int v, const double* eps,
                                   const double* oooo, const double* ooov, const double* oovv,
                                   const double* ovvo, const double* ovvv, int precision_mask);

/*
 * sigma_apply -- y = Hbar_N x (transpose = 0) or y = Hbar_N^T x (transpose = 1) for nrhs
 * complex vectors: x, y are complex128 [nrhs][D] (device). This is the connected part of
 * Hbar_N acting on X_p (Eq. xplin), the product every Krylov iteration needs.
 * precision: GFCC_FP64, GFCC_FP32, GFCC_FP32_BF16_3BODY or GFCC_BF16_PAIRS (the reduced
 * ones need GFCC_KEEP_FP32 at build time; transpose needs GFCC_KEEP_TRANSPOSE for speed but works
 * without it). x and y must not overlap. ESTATE if no operator is built. Any nrhs >= 0;
 * the products run in chunks of at most 2048 vectors.
 */
gfcc_status sigma_apply(gfcc_ctx* ctx, int nrhs, const void* x, void* y, int transpose,
                        int precision);

/*
 * gfcc_autotune -- switch the GEMM autotuner of ctx on (1, the default) or off (0) and forget
 * its choices. Products whose 128 x 128 tiles cannot fill the GPU but whose K is long (the
 * skinny products of the sigma) run split-K; with the tuner on, the first call in each product
 * class (tile counts, binary magnitude of K, 16-byte loads possible) times the generic kernel
 * and the pipelined kernel at three split counts, synchronising the context stream, and keeps
 * the fastest for the context. Products of 256 to 4095 tiles with a long K (the operator
 * build's largest products) are timed as the plain pipelined kernel and with 2 to 6 k ranges,
 * which moves the partly filled last round of workgroups. The forward FP64 sigma's two linear
 * products ([W1 ; 0 | Vp^T] . x, and the 2h1p products W4c . [x_1h ; tau] + (Woo (x) I_v) .
 * x_2h1p summed in one pass as a product batched over the virtual index) are timed as their
 * unfused route and as a segmented product on every candidate tile (32, 64 or 128 rows by 64
 * or 128 columns) and split count. Small row-major products (fewer than 64 tiles of 128 x 128
 * and 128 <= K < 512 doubles or 1024 floats, chiefly the operator build's at small shapes; a
 * transposed B is transposed first) are timed, into a scratch output, as their route above and
 * as a segmented product on every candidate tile and split count. The forward FP64 sigma's ovvo
 * product, when its operand written out takes at most 64 MiB (small operators and blocks), is
 * timed as the ovvo kernel and as the written-out operand on every segmented tile and split.
 * Off: the generic kernel with its heuristic split count for the first kind, the plain
 * pipelined kernel for the second, the unfused route for the sigma's products, the route above
 * for small products, the ovvo kernel for small ovvo products. enable = 2 skips the timing and
 * takes the most split candidate of every class (the segmented product for the sigma's, the
 * small and the small ovvo products), so that tests reach the split-K and segmented paths. Results agree to
 * rounding in every mode. EINVAL for another value of enable.
 */
gfcc_status gfcc_autotune(gfcc_ctx* ctx, int enable);

/*
 * gfcc_autotune_entry -- the tuner's choice number `index` (0-based, ordered by class):
 * desc[8] (host) receives {element bytes, kind, M, N, K, splits, tile rows, tile columns}.
 * kind: 0 or 1 a plain product (transA); 20 the sigma's [W1 ; 0 | Vp^T] . x; 21 the sigma's
 * linear 2h1p products; 22 a small product; 23 a small ovvo product. M, N, K: the shape it was measured on (for kind 21 the fused
 * product's: M = P pairs, N = columns, K = o + v + P, batched over the v virtual orbitals). splits: 0 for the generic kernel and,
 * for plain products of 256 tiles or more, 1 for the plain pipelined kernel. The tile is 0 x 0
 * for a plain product, for a sigma product that runs unfused and for a small product that
 * keeps its route. us[2] (host, may be NULL):
 * the measured time of the choice and of the reference variant (the generic kernel, the plain
 * pipelined kernel for products of 256 tiles or more, the unfused route of a sigma product,
 * the route of a small product when it is not segmented) in
 * microseconds. EINVAL past the last entry.
 */
gfcc_status gfcc_autotune_entry(const gfcc_ctx* ctx, int index, int64_t* desc, double* us);

/*
 * gfcc_autotune_pin -- fix the choice of every later sigma product of one kind on ctx,
 * bypassing the timing (until the next gfcc_autotune call): kind 20 or 21 (see
 * gfcc_autotune_entry). tile_m in {32, 64, 128}, tile_n in {64, 128}, splits >= 1 (split-K
 * applies to the unbatched kind 20 only); tile 0 x 0 selects the unfused route. For
 * measurements and tests of each variant. EINVAL for another kind or tile.
 */
gfcc_status gfcc_autotune_pin(gfcc_ctx* ctx, int kind, int tile_m, int tile_n, int splits);

/*
 * gfcc_graphs -- capture the Arnoldi steps of small GMRES blocks (those whose convergence flags
 * are read one step late: sigma work per step below about 0.3 ms) as HIP graphs (1, the
 * default) or launch them kernel by kernel (0). The first time a step shape is met on ctx it
 * runs eagerly, the second time it is captured, after that its graph is launched; graphs are
 * kept by the context and dropped whenever a workspace grows, the operator is rebuilt or the
 * tuner changes. No capture while a gfcc_timer records. Results are bitwise identical either
 * way. EINVAL for another value of enable.
 */
gfcc_status gfcc_graphs(gfcc_ctx* ctx, int enable);

/*
 * gfcc_compact -- restart compaction of GMRES blocks (1, the default) or none (0). At an FP64
 * restart where the right-hand sides that go on fill at most half the block's columns (counted
 * in groups of 64), they go on in a block of only their columns, whose work arrays take part
 * of the Krylov basis of the block they came from; its cycles start from their iterates with
 * the explicit FP64 residual, as the restart would. Results agree with the uncompacted solve
 * to rounding (the products of a narrower block may sum in another order); iteration counts
 * and residuals are reported per right-hand side as before. EINVAL for another value.
 */
gfcc_status gfcc_compact(gfcc_ctx* ctx, int enable);

/*
 * gfcc_solve -- solve Eq. xplin at every (omega_w, p_k) and form G (Eq. gfcclineqn).
 *
 * omega [nw] (host), p [np] (host; occupied orbitals 0 <= p < o, distinct), eta >= 0 (the
 *   broadening; eta = 0 is the undamped limit, whose real shifted operator is singular at
 *   its poles).
 * transpose = 0: (omega - i eta + Hbar_N) X = b_p with b_p = e_p (the occupied-orbital
 *   right-hand side), and G_out[w][q][p] = c_q^T X_p for q, p in the p set.
 * transpose = 1: (omega - i eta + Hbar_N^T) Y = c_p (the adjoint systems); since
 *   b_p^T Y_q = c_q^T X_p, G_out[w][q][p] is filled from b_p^T Y_q: the same G as the
 *   forward solve, up to the solve tolerance.
 * precision: GFCC_FP64 (right-preconditioned restarted GMRES with CGS2 Arnoldi, Jacobi
 *   preconditioner) or GFCC_FP32 / GFCC_FP32_BF16_3BODY / GFCC_BF16_PAIRS (FP64 iterative
 *   refinement around
 *   an inner GMRES whose sigma product runs in that precision; the stopping test is always
 *   the FP64 true relative residual).
 * tol: relative residual ||b - M x|| / ||b||. maxit: max iterations per right-hand side
 *   (inner+outer). restart: Krylov restart length (1..200; up to 64 the second Gram-Schmidt
 *   pass is delayed by one step, so the basis is swept twice per step instead of four times,
 *   which is the faster choice for long cycles). block: number of right-hand
 *   sides solved together (0 = library default, at most 2048). Multiples of 64 keep the
 *   fastest ovvo loader; a block that holds every right-hand side is padded with zero
 *   right-hand sides up to the next multiple of 64 when that adds at most a quarter; the last
 *   of several blocks is padded up to a multiple of 64 (at most the block size).
 * X_out: optional complex128 [nw][np][D] (device) or NULL. G_out: complex128 [nw][np][np]
 *   (device). iters_out, resid_out: host arrays [nw*np] or NULL.
 * Returns ENOCONV (after filling every output with the best iterate) if some right-hand side
 * did not reach tol; EBREAKDOWN (outputs filled as for ENOCONV) if a shifted operator is
 * exactly singular on a Krylov space (the Hessenberg least-squares problem of GMRES has a
 * zero pivot), and, for eta = 0, EBREAKDOWN before any solve (outputs untouched) when
 * omega_w + diag(Hbar_N) has a zero entry, where the Jacobi preconditioner does not exist
 * (for T = V = 0 exactly the poles omega = eps_i).
 * Memory: the context keeps the solver's work arrays (chiefly the Krylov basis,
 * (restart + 1) D block complex128 entries) for later solves; gfcc_destroy frees them.
 */
gfcc_status gfcc_solve(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                       double eta, double tol, int maxit, int restart, int block,
                       int precision, int transpose, void* X_out, void* G_out,
                       int* iters_out, double* resid_out);

/*
 * gfcc_solve_x0 -- gfcc_solve started from the initial guesses X0 (complex128 [nw][np][D],
 * device, the layout of X_out; for transpose = 1 the guesses of the adjoint solutions). The
 * first restart cycle begins with the explicit FP64 residual b - M X0, so a guess that already
 * meets tol costs one sigma product and no iteration. X0 may come from mor_lift (the reduced
 * model's approximate solutions, the initial guesses the paper names as a by-product of the
 * model described with Eq. model). X0 must not overlap X_out. Other arguments, outputs and
 * status codes as gfcc_solve.
 */
gfcc_status gfcc_solve_x0(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                          double eta, double tol, int maxit, int restart, int block,
                          int precision, int transpose, const void* X0, void* X_out,
                          void* G_out, int* iters_out, double* resid_out);

/*
 * gfcc_solve_diis -- Eq. xplin at every (omega_w, p_k) by complex DIIS, the linear solver of the
 * paper's convergence study (Results, Fig. 3, which keeps 10 micro-iteration iterates), in
 * FP64. A micro-iteration is one Jacobi step x <- x + e, e = P^{-1} (b - M x), P = diag(M),
 * M = (omega - i eta) I + Hbar_N (or Hbar_N^T for transpose = 1); after ndiis steps the kept
 * iterates are combined with the complex coefficients that minimise ||sum_k c_k e_k|| under
 * sum_k c_k = 1, and the subspace starts afresh. Each micro-iteration costs one sigma product.
 * The stopping test is the true relative residual, formed before every micro-iteration; a
 * right-hand side stops at tol, at maxit micro-iterations or at a non-finite residual.
 * ndiis: iterates per extrapolation, 1..16 (1 is the plain Jacobi iteration).
 * X0: initial guesses complex128 [nw][np][D] (device, e.g. from mor_lift) or NULL (zero);
 *   must not overlap X_out.
 * hist_out: host [nw*np][maxit+1] or NULL: relative residual of every evaluated iterate of each
 *   right-hand side (entry 0: the initial guess), -1 after the last one -- the convergence
 *   profile of Fig. 3.
 * iters_out receives micro-iterations. Other arguments, outputs and status codes as
 * gfcc_solve (ENOCONV if some right-hand side did not reach tol).
 */
gfcc_status gfcc_solve_diis(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                            double eta, double tol, int maxit, int ndiis, int block,
                            int transpose, const void* X0, void* X_out, void* G_out,
                            int* iters_out, double* resid_out, double* hist_out);

/*
 * gfcc_grad_eps -- adjoint gradient of J = sum_w weight_w A(omega_w) with respect to the
 * orbital energies eps (amplitudes held fixed):
 *   dJ/deps_r = (1/pi) sum_w weight_w sum_k Im( - Y_k^T D_r X_k ),
 * where X are forward solutions, Y adjoint solutions (both complex128 [nw][np][D] device, as
 * written by gfcc_solve) and D_r = dHbar_N/deps_r is diagonal in the packed basis.
 * weight [nw] (host). grad_out [o+v] (host).
 */
gfcc_status gfcc_grad_eps(gfcc_ctx* ctx, int nw, const double* weight, int np, const void* X,
                          const void* Y, double* grad_out);

/*
 * mor_build -- first reduced-order model (Eq. model): full solves at omega_k [nk] (host)
 * for orbitals p [np] (host), then a real orthonormal basis S of span{Re X_p(omega_k),
 * Im X_p(omega_k)} (CGS2, columns whose norm falls below defl_tol times their original norm
 * are dropped), Hbar S, and the projected Hhat = S^T Hbar S, bhat = S^T b, chat = S^T c.
 * The model owns its device memory; it stays valid while ctx lives.
 */
gfcc_status mor_build(gfcc_ctx* ctx, int nk, const double* omega_k, int np, const int* p,
                      double eta, double solve_tol, double defl_tol, gfcc_mor** model);

/*
 * mor_build_diag -- one reduced-order model per diagonal Green's function curve (the variant
 * the paper proposes in its outlook: separate models for every G_pp, whose sum gives A): the
 * full solves at omega_k [nk] (host) for all orbitals p [np] (host) run once, then model k is
 * built from the solutions of p[k] alone (basis from Re and Im X_{p[k]}(omega_k), as
 * mor_build with the single orbital p[k]). models [np] (host array) receives the np models;
 * on failure none is returned. Each model is refined, evaluated, lifted and destroyed like
 * one from mor_build; its G is the 1 x 1 block G_{p[k] p[k]}.
 */
gfcc_status mor_build_diag(gfcc_ctx* ctx, int nk, const double* omega_k, int np, const int* p,
                           double eta, double solve_tol, double defl_tol, gfcc_mor** models);

/*
 * mor_refine -- adaptive refinement (the strategy described after Eq. model): evaluate the
 * relative full-space residual of the reduced solutions on grid [nw] (host) restricted to
 * [wmin, wmax]; while its maximum exceeds resid_tol, add up to per_round midpoints of the
 * sampled-frequency intervals with the largest residual, solve there in full and extend S.
 * Stops at resid_tol, at max_order basis columns or after max_rounds. rounds_out (host)
 * receives the rounds run, max_resid_out (host) the final maximum residual.
 */
gfcc_status mor_refine(gfcc_mor* model, int nw, const double* grid, double wmin, double wmax,
                       int per_round, double resid_tol, int max_order, int max_rounds,
                       int* rounds_out, double* max_resid_out);

/*
 * mor_eval -- reduced Green's function at omega [nw] (host): Ghat_qp = chat_q^T xhat_p with
 * ((omega - i eta) I + Hhat) xhat_p = bhat_p. G_out complex128 [nw][np][np] (device);
 * resid_out [nw] (host, may be NULL): max over p of the relative full-space residual.
 */
gfcc_status mor_eval(gfcc_mor* model, int nw, const double* omega, void* G_out,
                     double* resid_out);

/*
 * mor_eval_noalloc -- mor_eval that allocates no device memory, for callers that cannot
 * allocate (code under HIP graph capture, serving loops that query a built model for new
 * frequencies, harnesses that forbid hipMalloc). The caller passes G_out (device) and
 * resid_out (host, may be NULL) as for mor_eval and gets the same values (the same kernels).
 * The per-frequency work space lives in a 32 MiB device array that the library holds on each
 * device until the process ends (its address is taken when the first context on that device
 * is created); frequencies run in chunks of as many as fit (a model of order m and np
 * orbitals takes 16 (m^2 + np m) + 16 bytes per frequency). ENOMEM if one frequency does not
 * fit (m of about 1440 at np = 8), ESTATE for an empty model. Every call on a device uses the
 * same array: calls that overlap in time on one device (other contexts, other host threads)
 * race and must be serialised by the caller. Synchronises the context stream.
 */
gfcc_status mor_eval_noalloc(gfcc_mor* model, int nw, const double* omega, void* G_out,
                             double* resid_out);

/*
 * mor_lift -- the reduced model's full-space approximate solutions X_out[w][k] = S xhat_{p_k}
 * (omega_w) for omega [nw] (host), the p set of the model: complex128 [nw][np][D] (device).
 * At a sampled frequency this is the full solution (up to the solve tolerance); elsewhere its
 * relative residual is the one mor_eval reports. Used as initial guesses by gfcc_solve_x0.
 */
gfcc_status mor_lift(gfcc_mor* model, int nw, const double* omega, void* X_out);

/* Model facts: order m (columns of S), sampled frequencies (host array of cap entries). */
gfcc_status mor_info(const gfcc_mor* model, int* m_out, int* nk_out, double* omega_k_out,
                     int cap);

/* Free a model. NULL is accepted. */
gfcc_status mor_destroy(gfcc_mor* model);

/*
 * spectral_function -- A(omega_w) = (1/pi) sum_p Im G[w][p][p] for G complex128
 * [nw][np][np] (device if is_device, else host: copied to the device first; the sum runs on
 * the device either way, on the null stream). A_out [nw] (host). The sign makes the peaks
 * positive for the operator (omega - i eta + Hbar_N). nw = 0 or np = 0 is accepted (A = 0
 * for np = 0); EINVAL for negative sizes or a null pointer that is needed.
 */
gfcc_status spectral_function(int nw, int np, const void* G, int is_device, double* A_out);

/*
 * spectral_weight -- the windowed spectral weight J = sum_w weight_w A(omega_w), with A as in
 * spectral_function (the objective whose orbital-energy gradient gfcc_grad_eps returns; with
 * trapezoid weights it is the integral of A over the window). G complex128 [nw][np][np]
 * (device if is_device, else host: copied to the device first); weight [nw] (host); J_out
 * (host). The sum runs on the device in a fixed order, on the null stream, and synchronises.
 * J = 0 for nw = 0 or np = 0; EINVAL for negative sizes or a null pointer that is needed.
 */
gfcc_status spectral_weight(int nw, int np, const void* G, int is_device, const double* weight,
                            double* J_out);

/*
 * Inspection (tests and profiling).
 * gfcc_export: copy a built operator block to a device buffer dst (FP64):
 *   0 Foo [o][o] (F_mi), 1 Fov [o][v] (F_me), 2 Fvv [v][v] (F_ae),
 *   3 Woooo [o][o][o][o] (W_mnij), 4 Wooov [o][o][o][v] (W_mnie),
 *   5 Wovvo [o][v][v][o] (W_mbej), 6 Wovoo [o][v][o][o] (W_mbij), 7 diag [D].
 * gfcc_timer: accumulated device time (ms, from HIP events on the context stream) and launch
 *   count of kernel family `which` since the last reset (0: the ovvo contraction of sigma,
 *   1: whole sigma products, 2: the two-term bf16 ovvo kernel of GFCC_BF16_PAIRS, which counts
 *   only the products that took it, not those on the FP32 fallback); reset = 1 clears after
 *   reading. Timing happens only while a family is enabled (enable = 1).
 */
gfcc_status gfcc_export(gfcc_ctx* ctx, int which, void* dst);
gfcc_status gfcc_timer(gfcc_ctx* ctx, int which, int enable, int reset, double* ms_out,
                       int64_t* launches_out);

#ifdef __cplusplus
}
#endif
#endif /* GFCC_H */
