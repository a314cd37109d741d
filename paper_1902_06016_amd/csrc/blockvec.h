// Complex arithmetic and the per-column partial-sum reductions shared by the block solvers
// (GMRES in solve.hip, DIIS in diis.hip). Vector blocks are D-major complex128 [D][nb]; the
// partial-sum kernels give every lane of a wavefront one right-hand side.
#pragma once

#include "common.h"

namespace gfcc {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  double s = fabs(b.x) + fabs(b.y);
  double ar = a.x / s, ai = a.y / s, br = b.x / s, bi = b.y / s;
  double d = br * br + bi * bi;
  return make_double2((ar * br + ai * bi) / d, (ai * br - ar * bi) / d);
}

constexpr int JG = 16;  // basis vectors per dot pass
constexpr int CW = 64;  // right-hand sides per reduction block: one wavefront, one per lane

// h[(j0+jj)][r] = sum_blk partial[blk][jj][r] (partial rows STRIDE apart per block). Grid
// (ceil(nb/64), nj), 256 threads: the lanes are 64 consecutive right-hand sides (coalesced
// reads), wave w sums the blocks w, w+4, ..., and the four wave sums are added in a fixed
// order.
template <int STRIDE>
__global__ __launch_bounds__(256) void dots_reduce_s(const double2* __restrict__ partial,
                                                     int nblk, int j0, int nj, int nb,
                                                     double2* __restrict__ h) {
  constexpr int JG = STRIDE;
  __shared__ double2 red[4][CW];
  const int lane = threadIdx.x % CW, w = threadIdx.x / CW;
  const int r = blockIdx.x * CW + lane, jj = blockIdx.y;
  double2 s0 = make_double2(0.0, 0.0), s1 = make_double2(0.0, 0.0);
  if (r < nb && jj < nj) {
    int b = w;
    for (; b + 4 < nblk; b += 8) {
      const double2 x = partial[((int64_t)b * JG + jj) * nb + r];
      const double2 y = partial[((int64_t)(b + 4) * JG + jj) * nb + r];
      s0.x += x.x; s0.y += x.y;
      s1.x += y.x; s1.y += y.y;
    }
    for (; b < nblk; b += 4) {
      const double2 x = partial[((int64_t)b * JG + jj) * nb + r];
      s0.x += x.x; s0.y += x.y;
    }
  }
  red[w][lane] = make_double2(s0.x + s1.x, s0.y + s1.y);
  __syncthreads();
  if (w == 0 && r < nb && jj < nj) {
    double2 t = red[0][lane];
    for (int q = 1; q < 4; ++q) {
      t.x += red[q][lane].x;
      t.y += red[q][lane].y;
    }
    h[(int64_t)(j0 + jj) * nb + r] = t;
  }
}

// out[r] = sqrt(sum_blk partial[blk][r]); same scheme as dots_reduce, grid ceil(nb/64)
__global__ __launch_bounds__(256) void norm_reduce(const double* __restrict__ partial, int nblk,
                                                   int nb, double* __restrict__ out) {
  __shared__ double red[4][CW];
  const int lane = threadIdx.x % CW, w = threadIdx.x / CW;
  const int r = blockIdx.x * CW + lane;
  double s0 = 0.0, s1 = 0.0;
  if (r < nb) {
    int b = w;
    for (; b + 4 < nblk; b += 8) {
      s0 += partial[(int64_t)b * nb + r];
      s1 += partial[(int64_t)(b + 4) * nb + r];
    }
    for (; b < nblk; b += 4) s0 += partial[(int64_t)b * nb + r];
  }
  red[w][lane] = s0 + s1;
  __syncthreads();
  if (w == 0 && r < nb) out[r] = sqrt(red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane]);
}

inline unsigned gridn(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 16384) b = 16384;
  return (unsigned)(b < 1 ? 1 : b);
}

template <typename T> T* carve(char*& cur, int64_t n) {
  T* p = reinterpret_cast<T*>(cur);
  cur += ((n * (int64_t)sizeof(T) + 255) / 256) * 256;
  return p;
}

}  // namespace
}  // namespace gfcc
