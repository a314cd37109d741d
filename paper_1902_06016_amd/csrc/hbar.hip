// build_hbar_operands: the similarity-transformed Hamiltonian blocks of the IP sector.
//
// The paper defines Hbar = e^{-T} H e^{T} (definition under Eq. gfxn1) and leaves its matrix
// elements to the literature. The blocks formed here are the spin-orbital CCSD Hbar elements
// with a diagonal Fock matrix; they are what the connected IP sigma product contracts with:
//   F_me, F_mi, F_ae, W_mnij, W_mnie, W_mbej, W_mbij.
// Every contraction is a dense product on the matrix cores: operands are first permuted
// into row-major [rows][contraction] form, then multiplied (gemm.hip). The two O(o^3 v^3)
// products are  sum_nf <mn||ef> t_jn^fb  (shared by W_mbej and W_mbij) and
// 1/2 sum_ef <mb||ef> tau_ij^ef.
//
// The blocks are then laid out as the row-major operator pieces that sigma multiplies by
// (common.h): W1, W4c, Woo, Vp, Weff, plus the diagonal and the c_q rows (Eq. gfxn2).
#include "common.h"

namespace gfcc {
namespace {

__global__ void tau_kernel(const double* __restrict__ t1, const double* __restrict__ t2, int o,
                           int v, double* __restrict__ tau) {
  int64_t n = (int64_t)o * o * v * v;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = idx;
    int b = t % v; t /= v;
    int a = t % v; t /= v;
    int j = t % o; t /= o;
    int i = (int)t;
    tau[idx] = t2[idx] + t1[i * v + a] * t1[j * v + b] - t1[i * v + b] * t1[j * v + a];
  }
}

__global__ void add_diag_kernel(double* __restrict__ M, int n, const double* __restrict__ e) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) M[(int64_t)i * n + i] += e[i];
}

__global__ void pairlut_kernel(int o, int* __restrict__ lut) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= o * o) return;
  int m = idx / o, j = idx % o;
  int s = 0;
  if (m < j) s = (int)pair_of(m, j, o) + 1;
  else if (m > j) s = -((int)pair_of(j, m, o) + 1);
  lut[idx] = s;
}

// pair index -> (i, j) by search over rows (o is small)
__device__ inline void unpair(int64_t pr, int o, int* pi, int* pj) {
  int i = 0;
  int64_t base = 0;
  while (i < o - 1) {
    int64_t cnt = o - 1 - i;
    if (pr < base + cnt) break;
    base += cnt;
    ++i;
  }
  *pi = i;
  *pj = (int)(i + 1 + (pr - base));
}

// W1[i][k] = -Foo[k][i];  W1[i][o+(kl)v+d] = -Wooov[k][l][i][d] + d_ik Fov[l][d] - d_il Fov[k][d]
__global__ void assemble_W1_kernel(const double* __restrict__ Foo, const double* __restrict__ Fov,
                                   const double* __restrict__ Wooov, int o, int v, int64_t D,
                                   double* __restrict__ W1) {
  int64_t n = (int64_t)o * D;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int i = (int)(idx / D);
    int64_t col = idx - (int64_t)i * D;
    double val;
    if (col < o) {
      val = -Foo[col * o + i];
    } else {
      int64_t q = col - o;
      int64_t pr = q / v;
      int d = (int)(q - pr * v);
      int k, l;
      unpair(pr, o, &k, &l);
      val = -Wooov[(((int64_t)k * o + l) * o + i) * v + d];
      if (i == k) val += Fov[(int64_t)l * v + d];
      if (i == l) val -= Fov[(int64_t)k * v + d];
    }
    W1[idx] = val;
  }
}

// W4c[(ij)a][k] = -Wovoo[k][a][i][j];  W4c[(ij)a][o+d] = -t2[i][j][a][d]
__global__ void assemble_W4c_kernel(const double* __restrict__ Wovoo, const double* __restrict__ t2,
                                    int o, int v, int64_t PV, double* __restrict__ W4c) {
  const int w = o + v;
  int64_t n = PV * w;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t row = idx / w;
    int col = (int)(idx - row * w);
    int64_t pr = row / v;
    int a = (int)(row - pr * v);
    int i, j;
    unpair(pr, o, &i, &j);
    double val;
    if (col < o) val = -Wovoo[(((int64_t)col * v + a) * o + i) * o + j];
    else val = -t2[(((int64_t)i * o + j) * v + a) * v + (col - o)];
    W4c[idx] = val;
  }
}

// Woo[(ij)][(kl)] = Woooo[k][l][i][j], rows of stride ldw (the padding is left untouched)
__global__ void assemble_Woo_kernel(const double* __restrict__ Woooo, int o, int64_t P,
                                    int64_t ldw, double* __restrict__ Woo) {
  int64_t n = P * P;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = idx / P, c = idx - (idx / P) * P;
    int i, j, k, l;
    unpair(r, o, &i, &j);
    unpair(c, o, &k, &l);
    Woo[r * ldw + c] = Woooo[(((int64_t)k * o + l) * o + i) * o + j];
  }
}

// Vp[(kl)c][d] = <kl||cd>
__global__ void assemble_Vp_kernel(const double* __restrict__ oovv, int o, int v, int64_t PV,
                                   double* __restrict__ Vp) {
  int64_t n = PV * v;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t row = idx / v;
    int d = (int)(idx - row * v);
    int64_t pr = row / v;
    int c = (int)(row - pr * v);
    int k, l;
    unpair(pr, o, &k, &l);
    Vp[idx] = oovv[(((int64_t)k * o + l) * v + c) * v + d];
  }
}

// Weff[(i,a)][(m,e)] = Wovvo[m][a][e][i] - d_ae Foo[m][i] + 1/2 d_mi Fvv[a][e]
__global__ void assemble_Weff_kernel(const double* __restrict__ Wovvo, const double* __restrict__ Foo,
                                     const double* __restrict__ Fvv, int o, int v,
                                     double* __restrict__ Weff) {
  const int64_t OV = (int64_t)o * v;
  int64_t n = OV * OV;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t r = idx / OV, c = idx - (idx / OV) * OV;
    int i = (int)(r / v), a = (int)(r % v);
    int m = (int)(c / v), e = (int)(c % v);
    double val = Wovvo[(((int64_t)m * v + a) * v + e) * o + i];
    if (a == e) val -= Foo[(int64_t)m * o + i];
    if (m == i) val += 0.5 * Fvv[(int64_t)a * v + e];
    Weff[idx] = val;
  }
}

// diagonal of Hbar_N in the packed basis
__global__ void diag_kernel(const double* __restrict__ W1, const double* __restrict__ Woo,
                            int64_t ldw, const double* __restrict__ Weff,
                            const double* __restrict__ t2, const double* __restrict__ oovv, int o,
                            int v, int64_t D, double* __restrict__ diag) {
  const int64_t OV = (int64_t)o * v;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < D;
       idx += (int64_t)gridDim.x * blockDim.x) {
    if (idx < o) {
      diag[idx] = W1[idx * D + idx];
      continue;
    }
    int64_t q = idx - o;
    int64_t pr = q / v;
    int a = (int)(q - pr * v);
    int i, j;
    unpair(pr, o, &i, &j);
    double val = Woo[pr * ldw + pr];
    int64_t ri = (int64_t)i * v + a, rj = (int64_t)j * v + a;
    val += Weff[ri * OV + ri] + Weff[rj * OV + rj];
    const double* tp = t2 + (((int64_t)i * o + j) * v + a) * v;
    const double* vp = oovv + (((int64_t)i * o + j) * v + a) * v;
    double s = 0.0;
    for (int d = 0; d < v; ++d) s += tp[d] * vp[d];
    diag[idx] = val - s;
  }
}

// c_q rows for all occupied q (Eq. gfxn2 with the GFCCSD truncation):
//   c_k    = d_qk - Y8[k][q] - 1/2 Y7[k][q]
//   c_kl^c = d_qk l1[l][c] - d_ql l1[k][c] - Y9[(kl)][q][c]
// with Y8[k][q] = sum_a l1[k][a] t1[q][a], Y7[k][q] = sum_lab l2[k][l][a][b] t2[q][l][a][b],
//      Y9[(k,l)][q][c] = sum_a t1[q][a] l2[k][l][a][c]   ((k,l) unrestricted)
__global__ void crows_kernel(const double* __restrict__ Y7, const double* __restrict__ Y8,
                             const double* __restrict__ Y9, const double* __restrict__ l1, int o,
                             int v, int64_t D, double* __restrict__ C) {
  int64_t n = (int64_t)o * D;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int q = (int)(idx / D);
    int64_t col = idx - (int64_t)q * D;
    double val;
    if (col < o) {
      int k = (int)col;
      val = (k == q ? 1.0 : 0.0) - Y8[(int64_t)k * o + q] - 0.5 * Y7[(int64_t)k * o + q];
    } else {
      int64_t t = col - o;
      int64_t pr = t / v;
      int c = (int)(t - pr * v);
      int k, l;
      unpair(pr, o, &k, &l);
      val = -Y9[(((int64_t)k * o + l) * o + q) * v + c];
      if (q == k) val += l1[(int64_t)l * v + c];
      if (q == l) val -= l1[(int64_t)k * v + c];
    }
    C[idx] = val;
  }
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

// First-order doubles: t2[i][j][a][b] = oovv[i][j][a][b] / (eps_i + eps_j - eps_a - eps_b)
// (virtual energies at eps[o + a]); the denominator is summed in that order.
__global__ void first_order_t2_kernel(const double* __restrict__ eps,
                                      const double* __restrict__ oovv, int o, int v,
                                      double* __restrict__ t2) {
  const int64_t n = (int64_t)o * o * v * v;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(idx % v);
    const int a = (int)((idx / v) % v);
    const int j = (int)((idx / ((int64_t)v * v)) % o);
    const int i = (int)(idx / ((int64_t)o * v * v));
    const double den = ((eps[i] + eps[j]) - eps[o + a]) - eps[o + b];
    t2[idx] = oovv[idx] / den;
  }
}

// small helper: dst (contiguous dims d) = alpha * src(strides s) + beta * dst
inline void perm(gfcc_ctx* ctx, const double* src, std::initializer_list<int64_t> d,
                 std::initializer_list<int64_t> s, double* dst, double alpha = 1.0,
                 double beta = 0.0) {
  int64_t dd[4], ss[4];
  int k = 0;
  for (auto x : d) dd[k++] = x;
  k = 0;
  for (auto x : s) ss[k++] = x;
  permute4(ctx, src, dd, ss, dst, alpha, beta);
}

}  // namespace

void first_order_t2(gfcc_ctx* ctx, int o, int v, const double* eps, const double* oovv,
                    double* t2) {
  hipLaunchKernelGGL(first_order_t2_kernel, dim3(grid_for((int64_t)o * o * v * v)), dim3(256), 0,
                     ctx->stream, eps, oovv, o, v, t2);
  GFCC_LAUNCH_CHECK();
}

namespace {

// Device buffers are reused from build to build: the previous operator's pieces and the work
// arrays of the previous build are taken back by size, so a rebuild of the same shape makes no
// hipMalloc or hipFree (each of which waits for the device). Buffers not taken are freed at
// the end of the build.
void collect(OpPieces<double>& f, std::vector<DevBuf>& out) {
  for (DevBuf* b : {&f.W1, &f.W4c, &f.Woo, &f.Vp, &f.Weff, &f.W1V, &f.W4})
    if (b->p) out.push_back(std::move(*b));
}
void collect(OpPieces<float>& f, std::vector<DevBuf>& out) {
  for (DevBuf* b : {&f.W1, &f.W4c, &f.Woo, &f.Vp, &f.Weff, &f.W1V, &f.W4})
    if (b->p) out.push_back(std::move(*b));
}
void collect(Operator& op, std::vector<DevBuf>& out) {
  collect(op.f64, out);
  collect(op.f32, out);
  for (DevBuf* b : {&op.VpT_bf16, &op.T2p_bf16, &op.VpT_bf16_lo, &op.T2p_bf16_lo, &op.Weff_bf16,
                    &op.Weff_bf16_lo, &op.WeffT, &op.W1T, &op.W4cT, &op.WooT, &op.VpT, &op.diag, &op.Crows, &op.pairlut, &op.Foo, &op.Fov, &op.Fvv, &op.Woooo,
                    &op.Wooov, &op.Wovvo, &op.Wovoo})
    if (b->p) out.push_back(std::move(*b));
}

// The device addresses of every operator piece, in a fixed order: captured solver steps bake
// them in, so they stay valid across a rebuild that hands back the same addresses.
std::vector<const void*> operator_addresses(const Operator& op) {
  std::vector<const void*> a;
  for (const DevBuf* b : {&op.f64.W1, &op.f64.W4c, &op.f64.Woo, &op.f64.Vp, &op.f64.Weff,
                          &op.f64.W1V, &op.f64.W4, &op.f32.W1, &op.f32.W4c, &op.f32.Woo,
                          &op.f32.Vp, &op.f32.Weff, &op.f32.W1V, &op.f32.W4, &op.VpT_bf16,
                          &op.T2p_bf16, &op.VpT_bf16_lo, &op.T2p_bf16_lo, &op.Weff_bf16,
                          &op.Weff_bf16_lo, &op.WeffT, &op.W1T, &op.W4cT, &op.WooT, &op.VpT,
                          &op.diag, &op.Crows, &op.pairlut})
    a.push_back(b->p);
  return a;
}

struct BuildBuffers {
  std::vector<DevBuf> avail;       // reusable buffers (freed when the build ends)
  std::vector<DevBuf>* keep_pool;  // receives the current operator build's work arrays
  void* take(DevBuf& b, size_t bytes) {
    for (size_t i = 0; i < avail.size(); ++i)
      if (avail[i].bytes == bytes) {
        b = std::move(avail[i]);
        avail.erase(avail.begin() + (std::ptrdiff_t)i);
        return b.p;
      }
    b.alloc(bytes);
    return b.p;
  }
};

// a work array of the build, handed to the next build when it goes out of scope
struct WorkBuf {
  std::vector<DevBuf>* pool;
  DevBuf b;
  explicit WorkBuf(BuildBuffers& bb) : pool(bb.keep_pool) {}
  WorkBuf(const WorkBuf&) = delete;
  WorkBuf& operator=(const WorkBuf&) = delete;
  ~WorkBuf() {
    if (b.p) pool->push_back(std::move(b));
  }
};

// work arrays above this total are not kept between builds
constexpr size_t BUILD_POOL_MAX = size_t(8) << 30;

}  // namespace

void build_operator(gfcc_ctx* ctx, int o, int v, const double* eps, const double* t1,
                    const double* t2, const double* l1, const double* l2, const double* oooo,
                    const double* ooov, const double* oovv, const double* ovvo,
                    const double* ovvv, int keep) {
  Operator& op = ctx->op;
  op.built = false;
  BuildBuffers bb;
  bb.avail = std::move(ctx->build_pool);
  ctx->build_pool.clear();
  bb.keep_pool = &ctx->build_pool;
  collect(op, bb.avail);
  op = Operator();
  const int64_t O = o, V = v;
  const int64_t P = O * (O - 1) / 2, PV = P * V, OV = O * V, D = O + PV;
  op.o = o; op.v = v; op.P = P; op.PV = PV; op.OV = OV; op.D = D; op.keep = keep;
  const int64_t o2 = O * O, v2 = V * V, o2v2 = o2 * v2, o3v = o2 * O * V;
  hipStream_t st = ctx->stream;
  auto B = [&bb](DevBuf& b, int64_t n) {
    return static_cast<double*>(bb.take(b, (size_t)n * sizeof(double)));
  };
  auto BW = [&bb](WorkBuf& w, int64_t n) {
    return static_cast<double*>(bb.take(w.b, (size_t)n * sizeof(double)));
  };

  double* Foo = B(op.Foo, o2);
  double* Fov = B(op.Fov, OV);
  double* Fvv = B(op.Fvv, v2);
  double* Woooo = B(op.Woooo, o2 * o2);
  double* Wooov = B(op.Wooov, o3v);
  double* Wovvo = B(op.Wovvo, o2v2);
  double* Wovoo = B(op.Wovoo, o3v);

  WorkBuf b_tau(bb), b_P1(bb), b_Q(bb), b_K6(bb), b_tmp1(bb), b_tmp2(bb);
  double* tau = BW(b_tau, o2v2);
  double* P1 = BW(b_P1, o2v2);    // <mn||ef> as [m][e][n][f]
  double* Q = BW(b_Q, o2v2);
  double* K6 = BW(b_K6, o2v2);
  double* T1 = BW(b_tmp1, std::max<int64_t>(o2v2, o3v));
  double* T2b = BW(b_tmp2, std::max<int64_t>(o2v2, o3v));

  hipLaunchKernelGGL(tau_kernel, dim3(grid_for(o2v2)), dim3(256), 0, st, t1, t2, o, v, tau);
  GFCC_LAUNCH_CHECK();
  // P1[m][e][n][f] = oovv[m][n][e][f]
  perm(ctx, oovv, {O, V, O, V}, {O * v2, V, v2, 1}, P1);

  // ---- F_me = sum_nf <mn||ef> t_n^f
  gemm<double>(ctx, false, false, (int)OV, 1, (int)OV, 1.0, P1, OV, t1, 1, 0.0, Fov, 1);

  // ---- F_mi = eps_i d_mi + sum_ne t_n^e <mn||ie> + 1/2 sum_nef tau_in^ef <mn||ef>
  gemm<double>(ctx, false, true, o, o, (int)(O * v2), 0.5, oovv, O * v2, tau, O * v2, 0.0, Foo, o);
  perm(ctx, ooov, {O, O, O, V}, {O * O * V, V, O * V, 1}, T1);  // [m][i][n][e]
  gemm<double>(ctx, false, false, (int)o2, 1, (int)OV, 1.0, T1, OV, t1, 1, 1.0, Foo, 1);
  hipLaunchKernelGGL(add_diag_kernel, dim3(1), dim3(256), 0, st, Foo, o, eps);
  GFCC_LAUNCH_CHECK();

  // ---- F_ae = eps_a d_ae - sum_mf t_m^f <ma||ef> - 1/2 sum_mnf tau_mn^af <mn||ef>
  perm(ctx, tau, {V, O, O, V}, {V, O * v2, v2, 1}, T1);   // tau as [a][m][n][f]
  perm(ctx, oovv, {V, O, O, V}, {V, O * v2, v2, 1}, T2b);  // oovv as [e][m][n][f]
  gemm<double>(ctx, false, true, v, v, (int)(o2 * V), -0.5, T1, o2 * V, T2b, o2 * V, 0.0, Fvv, v);
  {
    // Y[(ae)][m] = sum_f ovvv[m][a][e][f] t1[m][f]  (batched over m), then Fvv -= Y . 1
    WorkBuf b_y(bb), b_one(bb);
    double* Y = BW(b_y, v2 * O);
    double* ones = BW(b_one, O);
    fill(ctx, ones, O, 1.0);
    gemm<double>(ctx, false, false, (int)v2, 1, v, 1.0, ovvv, V, t1, 1, 0.0, Y, O, o,
                 V * v2, V, 1);
    gemm<double>(ctx, false, false, (int)v2, 1, o, -1.0, Y, O, ones, 1, 1.0, Fvv, 1);
    hipLaunchKernelGGL(add_diag_kernel, dim3(blocks_for(v, 256)), dim3(256), 0, st, Fvv, v,
                       eps + o);
    GFCC_LAUNCH_CHECK();
  }

  // ---- W_mnij = <mn||ij> + P(ij) t_j^e <mn||ie> + 1/2 tau_ij^ef <mn||ef>
  gemm<double>(ctx, false, true, (int)(o2 * O), o, v, 1.0, ooov, V, t1, V, 0.0, T1, O);  // Y[m][n][i][j]
  GFCC_HIP(hipMemcpyAsync(Woooo, oooo, sizeof(double) * o2 * o2, hipMemcpyDeviceToDevice, st));
  perm(ctx, T1, {O, O, O, O}, {O * O * O, O * O, O, 1}, Woooo, 1.0, 1.0);
  perm(ctx, T1, {O, O, O, O}, {O * O * O, O * O, 1, O}, Woooo, -1.0, 1.0);
  gemm<double>(ctx, false, true, (int)o2, (int)o2, (int)v2, 0.5, oovv, v2, tau, v2, 1.0, Woooo, o2);

  // ---- W_mnie = <mn||ie> + t_i^f <mn||fe>   (batched over (mn))
  GFCC_HIP(hipMemcpyAsync(Wooov, ooov, sizeof(double) * o3v, hipMemcpyDeviceToDevice, st));
  gemm<double>(ctx, false, false, o, v, v, 1.0, t1, V, oovv, V, 1.0, Wooov, V, (int)o2, 0, v2, O * V);

  // ---- K6[m][e][j][b] = sum_nf <mn||ef> t_jn^fb  (the O(o^3 v^3) product)
  perm(ctx, t2, {O, V, O, V}, {v2, V, O * v2, 1}, Q);  // Q[n][f][j][b] = t2[j][n][f][b]
  gemm<double>(ctx, false, false, (int)OV, (int)OV, (int)OV, 1.0, P1, OV, Q, OV, 0.0, K6, OV);

  // ---- W_mbej = <mb||ej> + t_j^f <mb||ef> - t_n^b <mn||ej> - (t_jn^fb + t_j^f t_n^b) <mn||ef>
  GFCC_HIP(hipMemcpyAsync(Wovvo, ovvo, sizeof(double) * o2v2, hipMemcpyDeviceToDevice, st));
  gemm<double>(ctx, false, true, (int)(O * v2), o, v, 1.0, ovvv, V, t1, V, 1.0, Wovvo, O);
  // Y2[m][b][j][e] = sum_n t1[n][b] ooov[m][n][j][e]  (batched over m); <mn||ej> = -<mn||je>
  gemm<double>(ctx, true, false, v, (int)OV, o, 1.0, t1, V, ooov, OV, 0.0, T1, OV, o,
               0, o2 * V, V * OV);
  perm(ctx, T1, {O, V, V, O}, {V * OV, OV, 1, V}, Wovvo, 1.0, 1.0);
  // - K6[m][e][j][b]  -> Wovvo[m][b][e][j]
  perm(ctx, K6, {O, V, V, O}, {V * OV, 1, OV, V}, Wovvo, -1.0, 1.0);
  // - sum_n t1[n][b] U[m][n][e][j],  U[(mne)][j] = sum_f oovv[m][n][e][f] t1[j][f]
  gemm<double>(ctx, false, true, (int)(o2 * V), o, v, 1.0, oovv, V, t1, V, 0.0, T1, O);
  gemm<double>(ctx, true, false, v, (int)(V * O), o, -1.0, t1, V, T1, V * O, 1.0, Wovvo, V * O, o,
               0, O * V * O, V * V * O);

  // ---- W_mbij
  //   = <mb||ij> - F_me t_ij^be - t_n^b W_mnij + 1/2 <mb||ef> tau_ij^ef
  //     + P(ij) <mn||ie> t_jn^be + P(ij) t_i^e ( <mb||ej> - t_nj^bf <mn||ef> )
  perm(ctx, ooov, {O, V, O, O}, {V, 1, O * O * V, O * V}, Wovoo);  // <ij||mb> -> [m][b][i][j]
  gemm<double>(ctx, false, true, o, (int)(o2 * V), v, 1.0, Fov, V, t2, V, 0.0, T1, o2 * V);  // [m][i][j][b]
  perm(ctx, T1, {O, V, O, O}, {o2 * V, 1, O * V, V}, Wovoo, -1.0, 1.0);
  gemm<double>(ctx, true, false, v, (int)o2, o, -1.0, t1, V, Woooo, o2, 1.0, Wovoo, o2, o,
               0, O * o2, V * o2);
  gemm<double>(ctx, false, true, (int)OV, (int)o2, (int)v2, 0.5, ovvv, v2, tau, v2, 1.0, Wovoo, o2);
  // Y5[m][i][j][b] = sum_ne ooov[m][n][i][e] t2[j][n][b][e]
  perm(ctx, ooov, {O, O, O, V}, {O * O * V, V, O * V, 1}, T1);      // A5[m][i][n][e]
  perm(ctx, t2, {O, V, O, V}, {v2, 1, O * v2, V}, T2b);              // B5[n][e][j][b]
  {
    WorkBuf b_y5(bb);
    double* Y5 = BW(b_y5, o3v);
    gemm<double>(ctx, false, false, (int)o2, (int)OV, (int)OV, 1.0, T1, OV, T2b, OV, 0.0, Y5, OV);
    perm(ctx, Y5, {O, V, O, O}, {O * OV, 1, OV, V}, Wovoo, 1.0, 1.0);
    perm(ctx, Y5, {O, V, O, O}, {O * OV, 1, V, OV}, Wovoo, -1.0, 1.0);
    // Z[m][b][e][j] = <mb||ej> - K6[m][e][j][b]
    GFCC_HIP(hipMemcpyAsync(T2b, ovvo, sizeof(double) * o2v2, hipMemcpyDeviceToDevice, st));
    perm(ctx, K6, {O, V, V, O}, {V * OV, 1, OV, V}, T2b, -1.0, 1.0);
    // Y6[(mb)][i][j] = sum_e t1[i][e] Z[(mb)][e][j]   (batched over (mb))
    WorkBuf b_y6(bb);
    double* Y6 = BW(b_y6, OV * o2);
    gemm<double>(ctx, false, false, o, o, v, 1.0, t1, V, T2b, O, 0.0, Y6, O, (int)OV, 0, V * O, o2);
    perm(ctx, Y6, {O, V, O, O}, {V * o2, o2, O, 1}, Wovoo, 1.0, 1.0);
    perm(ctx, Y6, {O, V, O, O}, {V * o2, o2, 1, O}, Wovoo, -1.0, 1.0);
  }

  // ---- operator pieces
  {
    bb.take(op.pairlut, sizeof(int) * o2);
    hipLaunchKernelGGL(pairlut_kernel, dim3(blocks_for(o2, 256)), dim3(256), 0, st, o,
                       op.pairlut.as<int>());
    GFCC_LAUNCH_CHECK();
    OpPieces<double>& f = op.f64;
    double* W1 = B(f.W1, O * D);
    hipLaunchKernelGGL(assemble_W1_kernel, dim3(grid_for(O * D)), dim3(256), 0, st, Foo, Fov,
                       Wooov, o, v, D, W1);
    GFCC_LAUNCH_CHECK();
    double* W4c = B(f.W4c, PV * (O + V));
    hipLaunchKernelGGL(assemble_W4c_kernel, dim3(grid_for(PV * (O + V))), dim3(256), 0, st,
                       Wovoo, t2, o, v, PV, W4c);
    GFCC_LAUNCH_CHECK();
    // rows padded with zeros to a multiple of 4 entries: 16-byte aligned rows for the
    // vector loads of the pipelined kernel in FP64 and FP32
    const int64_t ldw = op.ldwoo = (P + 3) / 4 * 4;
    double* Woo = B(f.Woo, P * ldw);
    fill(ctx, Woo, P * ldw, 0.0);
    hipLaunchKernelGGL(assemble_Woo_kernel, dim3(grid_for(P * P)), dim3(256), 0, st, Woooo, o, P,
                       ldw, Woo);
    GFCC_LAUNCH_CHECK();
    double* Vp = B(f.Vp, PV * V);
    hipLaunchKernelGGL(assemble_Vp_kernel, dim3(grid_for(PV * V)), dim3(256), 0, st, oovv, o, v, PV, Vp);
    GFCC_LAUNCH_CHECK();
    // [W1 ; 0 | Vp^T]: the forward sigma forms sigma_1h and the three-body intermediate tau
    // in one skinny product over the whole vector (X read once per 128-row tile)
    {
      double* W1V = B(f.W1V, (O + V) * D);
      GFCC_HIP(hipMemcpyAsync(W1V, W1, sizeof(double) * O * D, hipMemcpyDeviceToDevice, st));
      fill(ctx, W1V + O * D, V * D, 0.0);
      WorkBuf bt(bb);
      double* vt = BW(bt, V * PV);
      transpose2d(ctx, Vp, PV, V, vt);  // [v][PV]
      GFCC_HIP(hipMemcpy2DAsync(W1V + O * D + O, sizeof(double) * D, vt, sizeof(double) * PV,
                                sizeof(double) * PV, V, hipMemcpyDeviceToDevice, st));
    }
    // Weff is followed by zero padding read by the ovvo kernels past the last k slab
    const int64_t wpad = ovvo_pad_bytes(OV) / (int64_t)sizeof(double);
    double* Weff = B(f.Weff, OV * OV + wpad);
    fill(ctx, Weff + OV * OV, wpad, 0.0);
    hipLaunchKernelGGL(assemble_Weff_kernel, dim3(grid_for(OV * OV)), dim3(256), 0, st, Wovvo,
                       Foo, Fvv, o, v, Weff);
    GFCC_LAUNCH_CHECK();
    double* dg = B(op.diag, D);
    hipLaunchKernelGGL(diag_kernel, dim3(grid_for(D)), dim3(256), 0, st, W1, Woo, ldw, Weff, t2,
                       oovv, o, v, D, dg);
    GFCC_LAUNCH_CHECK();

    // c_q rows
    WorkBuf b7(bb), b8(bb), b9(bb);
    double* Y7 = BW(b7, o2);
    double* Y8 = BW(b8, o2);
    double* Y9 = BW(b9, o2 * O * V);
    gemm<double>(ctx, false, true, o, o, (int)(O * v2), 1.0, l2, O * v2, t2, O * v2, 0.0, Y7, O);
    gemm<double>(ctx, false, true, o, o, v, 1.0, l1, V, t1, V, 0.0, Y8, O);
    gemm<double>(ctx, false, false, o, v, v, 1.0, t1, V, l2, V, 0.0, Y9, V, (int)o2, 0, v2, O * V);
    double* C = B(op.Crows, O * D);
    hipLaunchKernelGGL(crows_kernel, dim3(grid_for(O * D)), dim3(256), 0, st, Y7, Y8, Y9, l1, o,
                       v, D, C);
    GFCC_LAUNCH_CHECK();

    if (keep & GFCC_KEEP_FP32) {
      OpPieces<float>& g = op.f32;
      auto F = [&bb](DevBuf& b, int64_t n) {
        return static_cast<float*>(bb.take(b, (size_t)n * sizeof(float)));
      };
      cast_f64_f32(ctx, W1, F(g.W1, O * D), O * D);
      cast_f64_f32(ctx, W4c, F(g.W4c, PV * (O + V)), PV * (O + V));
      cast_f64_f32(ctx, Woo, F(g.Woo, P * ldw), P * ldw);
      cast_f64_f32(ctx, Vp, F(g.Vp, PV * V), PV * V);
      const int64_t wpadf = ovvo_pad_bytes(OV) / (int64_t)sizeof(float);
      float* Wf = F(g.Weff, OV * OV + wpadf);
      cast_f64_f32(ctx, Weff, Wf, OV * OV);
      fill_f(ctx, Wf + OV * OV, wpadf, 0.0f);
      // Weff as bf16 pairs for the two-term ovvo: k segments of v padded to a multiple of 8,
      // rows padded to the 32-deep slab
      op.ldweff_bf = pairs_ldk(o, v);
      const int64_t nwb = pairs_rows(o, v) * op.ldweff_bf;
      bb.take(op.Weff_bf16, (size_t)nwb * sizeof(__hip_bfloat16));
      bb.take(op.Weff_bf16_lo, (size_t)nwb * sizeof(__hip_bfloat16));
      pairs_split_rows(ctx, Weff, o, v, op.Weff_bf16.p, op.Weff_bf16_lo.p);
      // bf16 three-body operands in the pair GEMM's layout: Vp^T [v][(ij)a] and -t2
      // [(ij)a][d]
      {
        const size_t nvt = (size_t)(pairs_pad_rows(V) * pairs_pad_k(PV));
        bb.take(op.VpT_bf16, nvt * sizeof(__hip_bfloat16));
        bb.take(op.VpT_bf16_lo, nvt * sizeof(__hip_bfloat16));
        pairs_split_general(ctx, Vp, 1, V, V, PV, op.VpT_bf16.p, op.VpT_bf16_lo.p);
      }
      WorkBuf bt(bb);
      double* t2p = BW(bt, PV * V);
      // -t2 packed rows = columns o.. of W4c
      {
        int64_t d4[4] = {1, 1, PV, V};
        int64_t s4[4] = {0, 0, O + V, 1};
        permute4(ctx, W4c + o, d4, s4, t2p, 1.0, 0.0);
      }
      {
        const size_t nt2 = (size_t)(pairs_pad_rows(PV) * pairs_pad_k(V));
        bb.take(op.T2p_bf16, nt2 * sizeof(__hip_bfloat16));
        bb.take(op.T2p_bf16_lo, nt2 * sizeof(__hip_bfloat16));
        pairs_split_general(ctx, t2p, V, 1, PV, V, op.T2p_bf16.p, op.T2p_bf16_lo.p);
      }
      // FP32 W4 = first o columns of W4c (the three-body columns go through bf16)
      {
        WorkBuf bw(bb);
        double* w4 = BW(bw, PV * O);
        int64_t d4[4] = {1, 1, PV, O};
        int64_t s4[4] = {0, 0, O + V, 1};
        permute4(ctx, W4c, d4, s4, w4, 1.0, 0.0);
        cast_f64_f32(ctx, w4, F(g.W4, PV * O), PV * O);
      }
    }
  }
  GFCC_HIP(hipStreamSynchronize(st));
  op.built = true;
  // captured solver steps survive a rebuild only where every operator piece kept its address
  // (and its shape: the step shapes carry o and v through D)
  std::vector<const void*> addr = operator_addresses(op);
  if (addr != ctx->op_addresses) {
    drop_step_graphs(ctx);
    ctx->op_addresses = std::move(addr);
  }
  size_t pooled = 0;
  for (const DevBuf& b : ctx->build_pool) pooled += b.bytes;
  if (pooled > BUILD_POOL_MAX) ctx->build_pool.clear();
}

}  // namespace gfcc
