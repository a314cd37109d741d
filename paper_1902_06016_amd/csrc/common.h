// Internal declarations shared by the HIP sources of libgfcc.so.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <array>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <stdexcept>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/gfcc.h"

namespace gfcc {

// ---------------------------------------------------------------------------------------
// errors: internal code throws gfcc::Error; every extern "C" entry point catches it.
struct Error : std::runtime_error {
  gfcc_status status;
  Error(gfcc_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

#define GFCC_HIP(call)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::gfcc::Error(GFCC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define GFCC_REQUIRE(cond, status, msg)                  \
  do {                                                   \
    if (!(cond)) throw ::gfcc::Error((status), (msg));   \
  } while (0)

#define GFCC_LAUNCH_CHECK() GFCC_HIP(hipGetLastError())

// ---------------------------------------------------------------------------------------
// device memory owned by the library (RAII, freed with hipFree).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw Error(GFCC_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
  }
  // grow-only reuse (scratch/workspace)
  void ensure(size_t n) {
    if (n > bytes) alloc(n);
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

// Pair index of i<j in the packed 2h1p layout (lexicographic).
__host__ __device__ inline int64_t pair_of(int i, int j, int o) {
  return (int64_t)i * o - (int64_t)i * (i + 1) / 2 + (j - i - 1);
}

// ---------------------------------------------------------------------------------------
// The device-resident operator. Row-major matrices acting on D-major vector blocks
// X[D][nc] (nc real columns; a complex right-hand side occupies two adjacent columns).
//
//   sigma_1h   = W1 . X                                (o x D)
//   sigma_2h1p = W4c . [X_1h ; tau]  +  Woo (x) I_v . X_2h1p  +  antisym( Weff . unpack(X_2h1p) )
//   tau        = Vp^T . X_2h1p                         (v x nc)
// with
//   W1[i][k]            = -F_ki,   W1[i][o+(kl)v+d] = -W_klid + d_ik F_ld - d_il F_kd
//   W4c[(ij)a][k]       = -W_kaij, W4c[(ij)a][o+d]  = -t_ij^ad
//   Woo[(ij)][(kl)]     = W_klij
//   Vp[(kl)c][d]        = <kl||cd>
//   Weff[(i,a)][(m,e)]  = W_maei - d_ae F_mi + 1/2 d_mi F_ae
// so that every sigma term is a dense contraction.
template <typename T> struct OpPieces {
  DevBuf W1, W4c, Woo, Vp, Weff;
  DevBuf W1V;              // [W1 ; 0 | Vp^T] (FP64): sigma_1h and tau in one product
  DevBuf W4;               // the first o columns of W4c (mixed precision)
};

struct Operator {
  bool built = false;
  int o = 0, v = 0;
  int64_t D = 0, P = 0, PV = 0, OV = 0;
  int64_t ldwoo = 0;            // row stride of Woo (P padded with zeros to a multiple of 4)
  int keep = 0;
  OpPieces<double> f64;
  OpPieces<float> f32;
  // bf16 pairs (x = hi + lo) of the three-body operands (mixed precision), padded row layout
  // of pairs_gemm: Vp^T [v][(ij)a] and -t2 [(ij)a][d]
  DevBuf VpT_bf16, VpT_bf16_lo, T2p_bf16, T2p_bf16_lo;
  DevBuf Weff_bf16, Weff_bf16_lo;  // Weff as bf16 pairs [o v][ldweff_bf] (pairs_split_rows)
  int64_t ldweff_bf = 0;
  DevBuf WeffT, W1T, W4cT, WooT, VpT;  // transposed copies (adjoint)
  DevBuf diag;                  // [D] diagonal of Hbar_N
  DevBuf Crows;                 // [o][D] c_q rows for all occupied q
  DevBuf pairlut;               // [o*o] int: +(pair+1) for i<j, -(pair+1) for i>j, 0 on i==j
  // blocks kept for export
  DevBuf Foo, Fov, Fvv, Woooo, Wooov, Wovvo, Wovoo;
};

// GEMM autotuner: one choice per product class {element bytes, transA, M tiles, N tiles,
// floor(log2 K), 16-byte A loads possible}; products of one class behave alike, so shapes that
// change a little (the reduced model's, round after round) are tuned once.
// The sigma's fused products are classes of their own: key[1] = one of the TUNE_SIGMA_* kinds
// below.
struct TuneChoice {
  int splits = 0;          // 0: generic split-K kernel (heuristic split count); > 0: pipelined
  double best_us = 0.0;    // measured time of the choice
  double generic_us = 0.0; // measured time of the generic kernel (or of the unfused route)
  int M = 0, N = 0, K = 0; // the shape it was measured on
  int tile_m = 0, tile_n = 0;  // segmented-product tile (0: not a segmented-product choice)
};
constexpr int64_t TUNE_SIGMA_1H = 20;      // sigma's [W1 ; Vp^T] . X: fused (tile) or unfused
constexpr int64_t TUNE_SIGMA_2H1P = 21;    // sigma's linear 2h1p products: fused or unfused
constexpr int64_t TUNE_SMALL = 22;         // small products: segmented tile and split, or generic
constexpr int64_t TUNE_OVVO = 23;          // small ovvo products: expanded operand on the segmented kernel, or the ovvo kernel
using TuneKey = std::array<int64_t, 6>;

struct TimerSlot {
  bool enabled = false;
  double ms = 0.0;
  int64_t launches = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

}  // namespace gfcc

struct gfcc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  gfcc::Operator op;
  // scratch, grow-only
  gfcc::DevBuf ws_gemm;     // split-K partials
  gfcc::DevBuf ws_a, ws_b, ws_c, ws_d, ws_e;
  gfcc::DevBuf ws_trans;    // transposed B operands of the row-major product paths
  gfcc::DevBuf ws_io;       // sigma_apply: D-major copies of its input and output blocks
  gfcc::DevBuf ws_pairs;    // the expanded bf16-pair operand of the two-term ovvo product
  gfcc::DevBuf ws_rexp;     // the expanded FP64 ovvo operand of small sigma products
  gfcc::DevBuf ws_tail;     // partial sums of the ovvo contraction's tail rows (split over m)
  gfcc::DevBuf ws_solve, ws_solve_f32;  // GMRES block work arrays (Krylov basis, state)
  std::vector<gfcc::DevBuf> build_pool;  // operator-build buffers kept for the next build
  gfcc::DevBuf zrow;        // zeros (read for structurally zero rows of the ovvo operand)
  gfcc::TimerSlot timers[3];  // ovvo contraction, whole sigma products, two-term bf16 ovvo
  int tune_mode = 1;        // 0 off, 1 timed, 2 most split variant without timing
  std::map<gfcc::TuneKey, gfcc::TuneChoice> tune;
  // choices pinned by gfcc_autotune_pin, by kind: {tile rows, tile columns, splits}
  std::map<int64_t, std::array<int, 3>> tune_pins;
  std::vector<hipEvent_t> event_pool;
  // Captured Arnoldi steps of small GMRES blocks (solve.hip), keyed by the step's shape; they
  // bake in kernel arguments (workspace and operator addresses, tuner choices), so every
  // workspace growth, operator build and tuner change bumps the generation and drops them.
  uint64_t generation = 0;
  bool graphs = true;
  bool compact = true;  // GMRES restarts continue the active right-hand sides in a compacted block
  std::vector<const void*> op_addresses;  // of the operator the captured steps were made for
  hipStream_t capture_stream = nullptr;  // the steps are captured here, launched on `stream`
  // host-visible convergence flags of the GMRES blocks (pinned, mapped; hflags_n words per slot)
  int* hflags = nullptr;
  int* dflags = nullptr;
  int hflags_n = 0;
  std::map<std::array<int64_t, 10>, hipGraphExec_t> step_graphs;
  std::map<std::array<int64_t, 10>, int> step_seen;
};

namespace gfcc {

// Grow a context-owned scratch buffer. Work already queued on the context stream may still
// read the old allocation, so the stream is drained before it is released.
// Drops the captured Arnoldi steps (their baked-in addresses or choices may be stale), after
// the stream has run every launch of them.
inline void drop_step_graphs(gfcc_ctx* ctx) {
  ++ctx->generation;
  if (!ctx->step_graphs.empty()) {
    GFCC_HIP(hipStreamSynchronize(ctx->stream));
    for (auto& kv : ctx->step_graphs) (void)hipGraphExecDestroy(kv.second);
    ctx->step_graphs.clear();
  }
  ctx->step_seen.clear();
}

inline void ws_ensure(gfcc_ctx* ctx, DevBuf& b, size_t n) {
  if (n <= b.bytes) return;
  GFCC_HIP(hipStreamSynchronize(ctx->stream));
  b.alloc(n);
  drop_step_graphs(ctx);
}

// ------------------------------------------------------------------------------ GEMM
// C[M][N] = alpha * op(A)[M][K] . op(B)[K][N] + beta * C, row-major, batched by strides.
// op(A) = A ([M][K], lda) or A^T (A stored [K][M], lda); op(B) likewise.
// beta == 0 never reads C.
template <typename T>
void gemm(gfcc_ctx* ctx, bool transA, bool transB, int M, int N, int K, T alpha, const T* A,
          int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc, int batch = 1,
          int64_t sA = 0, int64_t sB = 0, int64_t sC = 0);

// The ovvo contraction of sigma: Z[(i,a)][(j,c)] = sum_(m,e) Weff[(i,a)][(m,e)] * r_mj^e[c],
// where r is read from the packed 2h1p block X2[(pair,e)][c] (ld = ldx) through pairlut.
// transW: use Weff^T (the transpose product). Z is [o*v][o*nc].
template <typename T>
void gemm_ovvo(gfcc_ctx* ctx, bool transW, int o, int v, int nc, const T* W, const T* X2,
               int64_t ldx, const int* pairlut, T* Z);

// Specialised kernels for the same product (ovvo.hip); false if the shape is unsupported.
// W must be followed by ovvo_pad_bytes(o * v) bytes of zeros; zrow holds at least nc zeros
// (null disables the column-block variant).
template <typename T>
bool ovvo_fast(gfcc_ctx* ctx, bool transW, int o, int v, int nc, const T* W, const T* X2,
               int64_t ldx, T* Z, const T* zrow);
inline int64_t ovvo_pad_bytes(int64_t M) { return 512 * M; }

// C[M][N] = alpha op(A) B + beta C, B row-major [K][ldb], on the pipelined kernel of ovvo.hip;
// false when the product has too few 128 x 128 tiles to fill the GPU.
// a_padded: every row of A (its k dimension, or m when transposed) continues with finite
// entries up to a multiple of 16 bytes inside lda, so that 16-byte loads may cover the tail.
// Zas (with as_o, as_v, as_nc): C is the 2h1p block [P pairs][v nc] of the forward sigma and
// the epilogue adds its antisymmetrised ovvo term Z[(i,a)][(j,c)] - Z[(j,a)][(i,c)] (row
// pair(i, j), column a nc + c; Z [o v][o nc]).
template <typename T>
bool gemm_pipe(gfcc_ctx* ctx, bool transA, int M, int N, int K, T alpha, const T* A, int64_t lda,
               const T* B, int64_t ldb, T beta, T* C, int64_t ldc, bool a_padded = false,
               const T* Zas = nullptr, int as_o = 0, int as_v = 0, int as_nc = 0);

// Split-K partial products on the same kernel: part[y][M][N] = op(A) B over the k range
// [y kchunk, (y+1) kchunk) for y < splits (kchunk a multiple of 128 bytes of k); the caller
// reduces the slices.
template <typename T>
void gemm_pipe_split(gfcc_ctx* ctx, bool transA, int M, int N, int K, const T* A, int64_t lda,
                     const T* B, int64_t ldb, T* part, int splits, int kchunk);

// Segmented batched products: C_b = alpha * sum_{s < nseg} A_s,b . B_s,b + beta * C_b for
// b < batch, with A_s,b row-major [M][K_s] at A[s] + b * sA[s] (row stride lda[s]) and B_s,b
// row-major [K_s][N] at B[s] + b * sB[s] (row stride ldb[s]); C_b at C + b * sC (row stride
// ldc), except rows m >= msplit, which go to C2 + b * sC + (m - msplit) * ldc. beta == 0 never
// reads C. Row and batch strides express the Kronecker-structured 2h1p products of the sigma
// (a batch over the virtual index whose rows are v rows apart); the segments sum several such
// products in one pass over the output.
constexpr int SEG_MAX = 3;
template <typename T> struct SegSpec {
  int M = 0, N = 0, batch = 1, nseg = 1;
  int K[SEG_MAX] = {0, 0, 0};
  const T* A[SEG_MAX] = {nullptr, nullptr, nullptr};
  int64_t lda[SEG_MAX] = {0, 0, 0}, sA[SEG_MAX] = {0, 0, 0};
  const T* B[SEG_MAX] = {nullptr, nullptr, nullptr};
  int64_t ldb[SEG_MAX] = {0, 0, 0}, sB[SEG_MAX] = {0, 0, 0};
  T* C = nullptr;
  T* C2 = nullptr;
  int64_t ldc = 0, sC = 0;
  int msplit = 1 << 30;
  T alpha = T(1), beta = T(0);
  // Optional epilogue term (batch 1 per virtual index a, rows = pairs i < j, columns c): adds
  // Z[(i v + a)][j nc + c] - Z[(j v + a)][i nc + c], the antisymmetrised ovvo contraction of
  // the sigma (Z as written by gemm_ovvo, o v rows of o nc).
  const T* Zas = nullptr;
  int as_o = 0, as_v = 0, as_nc = 0;
};
// Runs the product on a given tile (tm x tn, tm in {32, 64, 128}, tn in {64, 128}) and split
// count (> 1 only for batch 1); the partials live in the context's split-K workspace.
template <typename T>
void segmm_run(gfcc_ctx* ctx, const SegSpec<T>& s, int tm, int tn, int splits);
// The tile and split candidates of a product, in the order the tuner times them.
template <typename T>
void segmm_candidates(const SegSpec<T>& s, std::vector<std::array<int, 3>>& out);

// Grows the split-K workspace to what the most split of the candidates needs, before they are
// timed (so that no candidate's time includes the allocation).
template <typename T>
void segmm_reserve(gfcc_ctx* ctx, const SegSpec<T>& s,
                   const std::vector<std::array<int, 3>>& cands);
// Times each candidate (one warm-up run, then two timed runs, on the context stream; a
// candidate whose warm-up run took more than twice the best time so far is not run again) and
// returns the index of the fastest; us[i] receives candidate i's time in microseconds.
// Synchronises the stream. Candidates must be complete, idempotent computations.
int time_candidates(gfcc_ctx* ctx, const std::vector<std::function<void()>>& cands,
                    std::vector<double>& us);

// A device buffer of at least `bytes` zero bytes, owned by the context (grown on demand).
const void* zero_row(gfcc_ctx* ctx, size_t bytes);

// Two-term bf16 products (ovvo_bf3.hip): C[M][N] (+)= A B with A held as bf16 pairs (hi, lo)
// in the padded row layout [pairs_pad_rows(M)][pairs_pad_k(K)] written by pairs_split_general
// (A[r][k] = S[r rs + k cs]), and B FP32 [K][N] (row stride ldb) split into pairs on the way;
// every block takes hi.hi + hi.lo + lo.hi with FP32 accumulation.
int64_t pairs_pad_rows(int64_t M);
int64_t pairs_pad_k(int64_t K);
void pairs_split_general(gfcc_ctx* ctx, const double* S, int64_t rs, int64_t cs, int64_t M,
                         int64_t K, void* hi, void* lo);
void pairs_gemm(gfcc_ctx* ctx, const void* Ah, const void* Al, int M, int K, const float* B,
                int64_t ldb, int N, float* C, int64_t ldc, bool accumulate);

// ------------------------------------------------------------------- tensor utilities
// dst[i0][i1][i2][i3] (contiguous, dims d[]) = alpha * src[i0*s0 + i1*s1 + i2*s2 + i3*s3]
//   + beta * dst   (beta == 0 never reads dst)
void permute4(gfcc_ctx* ctx, const double* src, const int64_t d[4], const int64_t s[4],
              double* dst, double alpha = 1.0, double beta = 0.0);
void fill(gfcc_ctx* ctx, double* p, int64_t n, double val);
void fill_f(gfcc_ctx* ctx, float* p, int64_t n, float val);
void cast_f64_f32(gfcc_ctx* ctx, const double* s, float* d, int64_t n);
void cast_f32_f64(gfcc_ctx* ctx, const float* s, double* d, int64_t n);
// ovvo contraction with two-term bf16 operands (FP32 X2 and Z; W as pairs from
// pairs_split_rows); false when nc is not a multiple of 128 (the caller then uses the FP32
// kernel)
bool ovvo_bf3(gfcc_ctx* ctx, int o, int v, int nc, const void* Wh, const void* Wl,
              const float* X2, int64_t ldx, float* Z);
// row length (bf16 elements) of the pairs of the o v x o v ovvo matrix: o segments of v rounded
// up to 8, rounded up to a 32-deep slab
int64_t pairs_ldk(int o, int v);
// rows of those pairs: o v rounded up to a multiple of 256 (the extra rows are zero)
int64_t pairs_rows(int o, int v);
// those pairs from the FP64 matrix S [o v][o v]: hi and lo are [pairs_rows][pairs_ldk] bf16
void pairs_split_rows(gfcc_ctx* ctx, const double* S, int o, int v, void* hi, void* lo);
void transpose2d(gfcc_ctx* ctx, const double* src, int64_t rows, int64_t cols, double* dst);
// complex128 transpose: dst[c*ldd + r] = src[r*lds + c] for r < rows, c < cols
void ctranspose(gfcc_ctx* ctx, const void* src, int64_t rows, int64_t cols, int64_t lds,
                void* dst, int64_t ldd);
// count of non-finite entries of a device array (synchronises)
// number of non-finite entries of each device array (one synchronisation for all)
std::vector<int64_t> count_nonfinite(gfcc_ctx* ctx,
                                     const std::vector<std::pair<const double*, int64_t>>& arrs);

// -------------------------------------------------------------------- sigma products
// Y[D][nc] = Hbar_N X[D][nc] (or Hbar_N^T). Real columns; X and Y D-major with ld = nc.
void sigma_block_f64(gfcc_ctx* ctx, int nc, const double* X, double* Y, bool transpose);
void sigma_block_f32(gfcc_ctx* ctx, int nc, const float* X, float* Y, int precision);

// -------------------------------------------------------------------- shifted solves
// Every (omega, p) of the grid, solved in blocks of right-hand sides (solve.hip). G_out is
// device [nw][np][np], X_out null or device [nw][np][D], X0 null or device initial guesses
// [nw][np][D]. ndiis > 0 selects the periodic complex DIIS of diis.hip with that many iterates
// per extrapolation (FP64; restart and precision unused) and hist its residual histories
// (null or host [nw * np][maxit + 1]).
gfcc_status solve_all(gfcc_ctx* ctx, int nw, const double* omega, int np, const int* p,
                      double eta, double tol, int maxit, int restart, int block, int precision,
                      int transpose, void* X_out, void* G_out, int* iters_out, double* resid_out,
                      const void* X0, int ndiis = 0, double* hist = nullptr);

// Right-hand-side block B[D][nb] (complex128): forward b = e_p, transpose b = c_p; a column
// with prow[r] = -1 is zero. prow is a device array.
void solve_rhs(gfcc_ctx* ctx, const int* prow, bool transpose, int64_t D, int nb, void* B);

// Hbar_N U for the block U[d][r] = e_p / (diag_p + z_r), p = prow[r] (zero columns where
// prow[r] < 0): column p of Hbar_N (of W1 in the 1h rows, of W4c in the 2h1p rows) scaled, the
// first product of a forward solve started from x = 0, without a sigma product. z is complex
// [nb], W complex [D][nb], all device.
void unit_sigma(gfcc_ctx* ctx, const int* prow, const void* z, int nb, void* W);

// DIIS workspace, grown on demand and reused across blocks.
struct DiisWork {
  DevBuf mem;
};
// Solves the right-hand sides [r0, r0 + nb) (global index w * np + k; indices >= nrhs are
// padding) by periodic DIIS with m iterates per extrapolation. Returns the device block of
// solutions [D][nb] (inside w.mem). its and res are host arrays over all right-hand sides;
// hist is null or host [nrhs][maxit + 1]; X0 is null or device [nrhs][D].
const void* diis_block(gfcc_ctx* ctx, DiisWork& w, int nb, int m, const double* omega,
                       const int* pset, int np, int nrhs, int r0, double eta, double tol,
                       int maxit, bool transpose, int* its, double* res, double* hist,
                       const void* X0);

// event-timed launch helpers
void timer_begin(gfcc_ctx* ctx, int which, hipEvent_t* ev);
void timer_end(gfcc_ctx* ctx, int which, hipEvent_t ev0);
void timers_collect(gfcc_ctx* ctx);
// an event from timer_begin whose launch did not happen (returned to the pool)
void timer_cancel(gfcc_ctx* ctx, hipEvent_t ev0);

inline unsigned blocks_for(int64_t n, int threads) {
  int64_t b = (n + threads - 1) / threads;
  if (b > (1 << 30)) b = 1 << 30;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace gfcc

// Wrap an extern "C" body: converts exceptions to status codes and records the message.
#define GFCC_API_BEGIN(ctx) try {
#define GFCC_API_END(ctx)                                              \
  }                                                                    \
  catch (const ::gfcc::Error& e) {                                     \
    if (ctx) (ctx)->last_error = e.what();                             \
    return e.status;                                                   \
  }                                                                    \
  catch (const std::exception& e) {                                    \
    if (ctx) (ctx)->last_error = e.what();                             \
    return GFCC_EINVAL;                                                \
  }                                                                    \
  return GFCC_OK;
