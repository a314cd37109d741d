// bf16 x bf16 -> fp32 products on CDNA4 matrix cores (v_mfma_f32_16x16x32_bf16).
// Used for the three-body term of the mixed-precision sigma product, whose operands (<kl||cd>
// and t2) are streamed from HBM in bf16 while accumulation stays in FP32.
//
// Tile 128 x 128 x 32 per workgroup of 4 wavefronts (2 x 2, 64 x 64 each). Operands are staged
// k-contiguous in LDS so each lane's 8 consecutive k values are one 16-byte read.
#include "common.h"

namespace gfcc {
namespace {

constexpr int BM = 128, BN = 128, BK = 32, NT = 256, KP = BK + 8;
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

struct P16 {
  int M, N, K;
  const __hip_bfloat16* A; int64_t lda;
  const __hip_bfloat16* B; int64_t ldb;
  float* C; int64_t ldc, sC;
  float alpha, beta;
  int kchunk, mtiles, ntiles;
};

template <bool TA, bool SPLIT>
__global__ __launch_bounds__(NT) void gemm_bf16_kernel(P16 p) {
  __shared__ __attribute__((aligned(16))) __hip_bfloat16 As[BM][KP];
  __shared__ __attribute__((aligned(16))) __hip_bfloat16 Bs[BN][KP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int mt = blockIdx.x % p.mtiles, nt = blockIdx.x / p.mtiles;
  const int m0 = mt * BM, n0 = nt * BN;
  int kbeg = 0, kend = p.K;
  if (SPLIT) { kbeg = blockIdx.z * p.kchunk; kend = min(p.K, kbeg + p.kchunk); }
  const __hip_bfloat16 zero = __float2bfloat16(0.0f);

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0, 0, 0, 0};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // A tile -> As[m][k]
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      int m, k;
      if (TA) { m = tid % BM; k = tid / BM + 2 * r; }
      else    { k = tid % BK; m = tid / BK + 8 * r; }
      int gm = m0 + m, gk = k0 + k;
      __hip_bfloat16 val = zero;
      if (gm < p.M && gk < kend) val = TA ? p.A[(int64_t)gk * p.lda + gm] : p.A[(int64_t)gm * p.lda + gk];
      As[m][k] = val;
    }
    // B tile ([K][N] row-major) -> Bs[n][k]
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      int n = tid % BN, k = tid / BN + 2 * r;
      int gn = n0 + n, gk = k0 + k;
      __hip_bfloat16 val = zero;
      if (gn < p.N && gk < kend) val = p.B[(int64_t)gk * p.ldb + gn];
      Bs[n][k] = val;
    }
    __syncthreads();
    const int rl = lane & 15, kq = (lane >> 4) * 8;
    bf8 af[4], bfr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      af[i] = *reinterpret_cast<const bf8*>(&As[wm * 64 + i * 16 + rl][kq]);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      bfr[j] = *reinterpret_cast<const bf8*>(&Bs[wn * 64 + j * 16 + rl][kq]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }

  float* C = p.C;
  if (SPLIT) C += (int64_t)blockIdx.z * p.sC;
  const int col_l = lane & 15, rq = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + wn * 64 + j * 16 + col_l;
      if (n >= p.N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wm * 64 + i * 16 + rq + q;
        if (m >= p.M) continue;
        float* dst = C + (int64_t)m * p.ldc + n;
        if (SPLIT) {
          *dst = acc[i][j][q];
        } else {
          float val = p.alpha * acc[i][j][q];
          if (p.beta != 0.0f) val += p.beta * *dst;
          *dst = val;
        }
      }
    }
}

__global__ void reduce_f32(const float* __restrict__ part, int splits, int M, int N,
                           int64_t pstride, float* __restrict__ C, int64_t ldc, float alpha,
                           float beta) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)M * N) return;
  int m = (int)(idx / N), n = (int)(idx % N);
  float s = 0.0f;
  for (int z = 0; z < splits; ++z) s += part[z * pstride + idx];
  float* dst = C + (int64_t)m * ldc + n;
  float val = alpha * s;
  if (beta != 0.0f) val += beta * *dst;
  *dst = val;
}

}  // namespace

void gemm_bf16(gfcc_ctx* ctx, bool transA, int M, int N, int K, float alpha,
               const __hip_bfloat16* A, int64_t lda, const __hip_bfloat16* B, int64_t ldb,
               float beta, float* C, int64_t ldc) {
  if (M <= 0 || N <= 0) return;
  P16 p{};
  p.M = M; p.N = N; p.K = K < 0 ? 0 : K;
  p.A = A; p.lda = lda; p.B = B; p.ldb = ldb;
  p.alpha = alpha; p.beta = beta;
  p.mtiles = (M + BM - 1) / BM;
  p.ntiles = (N + BN - 1) / BN;
  const int64_t tiles = (int64_t)p.mtiles * p.ntiles;
  int splits = 1;
  if (tiles < 512 && p.K >= BK * 16) {
    splits = (int)std::min<int64_t>((1024 + tiles - 1) / tiles, p.K / (BK * 8));
    if (splits < 1) splits = 1;
  }
  int64_t chunk = ((int64_t)p.K + splits - 1) / splits;
  chunk = (chunk + BK - 1) / BK * BK;
  if (chunk == 0) chunk = BK;
  splits = (int)std::max<int64_t>(1, ((int64_t)p.K + chunk - 1) / chunk);
  p.kchunk = (int)chunk;
  if (splits == 1) {
    p.C = C; p.ldc = ldc; p.sC = 0;
    dim3 grid((unsigned)tiles, 1, 1);
    if (transA) hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(NT), 0, ctx->stream, p);
    else hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(NT), 0, ctx->stream, p);
    GFCC_LAUNCH_CHECK();
    return;
  }
  const int64_t slab = (int64_t)M * N;
  ws_ensure(ctx, ctx->ws_gemm, sizeof(float) * (size_t)slab * splits);
  float* part = ctx->ws_gemm.as<float>();
  p.C = part; p.ldc = N; p.sC = slab;
  dim3 grid((unsigned)tiles, 1, (unsigned)splits);
  if (transA) hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(NT), 0, ctx->stream, p);
  else hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(NT), 0, ctx->stream, p);
  GFCC_LAUNCH_CHECK();
  hipLaunchKernelGGL(reduce_f32, dim3(blocks_for(slab, 256)), dim3(256), 0, ctx->stream, part,
                     splits, M, N, slab, C, ldc, alpha, beta);
  GFCC_LAUNCH_CHECK();
}

}  // namespace gfcc
