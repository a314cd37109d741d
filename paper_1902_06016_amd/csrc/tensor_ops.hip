// Memory-bound helpers: strided permutation, fills, casts, transposes, finiteness check.
#include "common.h"

#include <algorithm>

namespace gfcc {
namespace {

__global__ void permute4_kernel(const double* __restrict__ src, int64_t d1, int64_t d2,
                                int64_t d3, int64_t s0, int64_t s1, int64_t s2, int64_t s3,
                                int64_t n, double* __restrict__ dst, double alpha, double beta) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = idx;
    int64_t i3 = t % d3; t /= d3;
    int64_t i2 = t % d2; t /= d2;
    int64_t i1 = t % d1; t /= d1;
    int64_t i0 = t;
    double val = alpha * src[i0 * s0 + i1 * s1 + i2 * s2 + i3 * s3];
    if (beta != 0.0) val += beta * dst[idx];
    dst[idx] = val;
  }
}

template <typename T>
__global__ void fill_kernel(T* p, int64_t n, T val) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = val;
}

__global__ void cast_f32_kernel(const double* __restrict__ s, float* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (float)s[i];
}

__global__ void cast_bf16_kernel(const double* __restrict__ s, __hip_bfloat16* __restrict__ d,
                                 int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = __float2bfloat16((float)s[i]);
}

__global__ void cast_f32_f64_kernel(const float* __restrict__ s, double* __restrict__ d,
                                    int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = (double)s[i];
}

__global__ void transpose_kernel(const double* __restrict__ src, int64_t rows, int64_t cols,
                                 double* __restrict__ dst) {
  __shared__ double tile[32][33];
  int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
  int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows per pass
  for (int k = ty; k < 32; k += 8) {
    int64_t r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) tile[k][tx] = src[r * cols + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    int64_t c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) dst[c * rows + r] = tile[tx][k];
  }
}

// Non-finite entries of up to NF_MAX arrays in two launches: blockIdx.y picks the array, whose
// blocks count grid-stride into partial[y][blockIdx.x]; then one block per array adds its
// partials in a fixed order.
constexpr int NF_MAX = 16;
struct NonfiniteArgs {
  const double* p[NF_MAX];
  int64_t n[NF_MAX];
};

__global__ void nonfinite_kernel(NonfiniteArgs a, unsigned long long* __restrict__ partial) {
  __shared__ unsigned long long red[256];
  const double* p = a.p[blockIdx.y];
  const int64_t n = a.n[blockIdx.y];
  unsigned long long local = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    local += isfinite(p[i]) ? 0ull : 1ull;
  red[threadIdx.x] = local;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

__global__ void sum_u64_kernel(const unsigned long long* __restrict__ partial, int n,
                               unsigned long long* __restrict__ out) {
  __shared__ unsigned long long red[256];
  const unsigned long long* pp = partial + (int64_t)blockIdx.x * n;
  unsigned long long local = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) local += pp[i];
  red[threadIdx.x] = local;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 65536) b = 65536;
  return (unsigned)(b < 1 ? 1 : b);
}

}  // namespace

void permute4(gfcc_ctx* ctx, const double* src, const int64_t d[4], const int64_t s[4],
              double* dst, double alpha, double beta) {
  int64_t n = d[0] * d[1] * d[2] * d[3];
  if (n == 0) return;
  hipLaunchKernelGGL(permute4_kernel, dim3(grid_for(n)), dim3(256), 0, ctx->stream, src, d[1],
                     d[2], d[3], s[0], s[1], s[2], s[3], n, dst, alpha, beta);
  GFCC_LAUNCH_CHECK();
}

void fill(gfcc_ctx* ctx, double* p, int64_t n, double val) {
  if (n == 0) return;
  hipLaunchKernelGGL(fill_kernel<double>, dim3(grid_for(n)), dim3(256), 0, ctx->stream, p, n, val);
  GFCC_LAUNCH_CHECK();
}

void fill_f(gfcc_ctx* ctx, float* p, int64_t n, float val) {
  if (n == 0) return;
  hipLaunchKernelGGL(fill_kernel<float>, dim3(grid_for(n)), dim3(256), 0, ctx->stream, p, n, val);
  GFCC_LAUNCH_CHECK();
}

const void* zero_row(gfcc_ctx* ctx, size_t bytes) {
  bytes = (std::max<size_t>(bytes, 256) + 7) / 8 * 8;
  if (ctx->zrow.bytes < bytes) {
    ws_ensure(ctx, ctx->zrow, bytes);
    fill(ctx, ctx->zrow.as<double>(), (int64_t)(ctx->zrow.bytes / sizeof(double)), 0.0);
  }
  return ctx->zrow.p;
}

void cast_f64_f32(gfcc_ctx* ctx, const double* s, float* d, int64_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(cast_f32_kernel, dim3(grid_for(n)), dim3(256), 0, ctx->stream, s, d, n);
  GFCC_LAUNCH_CHECK();
}

void cast_f32_f64(gfcc_ctx* ctx, const float* s, double* d, int64_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(cast_f32_f64_kernel, dim3(grid_for(n)), dim3(256), 0, ctx->stream, s, d, n);
  GFCC_LAUNCH_CHECK();
}

void transpose2d(gfcc_ctx* ctx, const double* src, int64_t rows, int64_t cols, double* dst) {
  if (rows == 0 || cols == 0) return;
  dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
  GFCC_REQUIRE(grid.y < 65536, GFCC_EINVAL, "transpose2d: too many rows");
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, ctx->stream, src, rows, cols, dst);
  GFCC_LAUNCH_CHECK();
}

std::vector<int64_t> count_nonfinite(gfcc_ctx* ctx,
                                     const std::vector<std::pair<const double*, int64_t>>& arrs) {
  const size_t na = arrs.size();
  std::vector<int64_t> out(na, 0);
  if (na == 0) return out;
  std::vector<unsigned long long> h(na);
  for (size_t k0 = 0; k0 < na; k0 += NF_MAX) {
    const int cnt = (int)std::min<size_t>(NF_MAX, na - k0);
    NonfiniteArgs a{};
    int64_t nmax = 0;
    for (int k = 0; k < cnt; ++k) {
      a.p[k] = arrs[k0 + k].first;
      a.n[k] = arrs[k0 + k].second;
      nmax = std::max(nmax, a.n[k]);
    }
    // blocks per array: enough for the largest, at most 1024; one copy and one wait for all
    const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (nmax + 255) / 256));
    ws_ensure(ctx, ctx->ws_e, sizeof(unsigned long long) * (size_t)(nb + 1) * cnt);
    auto* part = ctx->ws_e.as<unsigned long long>();
    auto* tot = part + (size_t)nb * cnt;
    hipLaunchKernelGGL(nonfinite_kernel, dim3(nb, cnt), dim3(256), 0, ctx->stream, a, part);
    GFCC_LAUNCH_CHECK();
    hipLaunchKernelGGL(sum_u64_kernel, dim3(cnt), dim3(256), 0, ctx->stream, part, nb, tot);
    GFCC_LAUNCH_CHECK();
    GFCC_HIP(hipMemcpyAsync(h.data() + k0, tot, sizeof(unsigned long long) * cnt,
                            hipMemcpyDeviceToHost, ctx->stream));
    GFCC_HIP(hipStreamSynchronize(ctx->stream));
  }
  for (size_t k = 0; k < na; ++k) out[k] = (int64_t)h[k];
  return out;
}

}  // namespace gfcc
