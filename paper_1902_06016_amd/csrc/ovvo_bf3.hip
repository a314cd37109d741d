// The ovvo contraction of the IP sigma product (Eq. xplin's T5, T6 and T8 terms through Weff)
// on bf16 matrix cores with two-term operands, for the reduced-precision sigma of the mixed
// solver:
//   Z[(i,a)][(j,c)] = sum_(m,e) W[(i,a)][(m,e)] r_mj^e[c],     r_mj^e = +-X2[pair(m,j)][e][c]
// W is held as bf16 pairs W = Wh + Wl; the FP32 packed block X2 is expanded (sign, zero
// segment m = j) and split into hi + lo (round to nearest even on the packed converter) while
// the B tile is staged in LDS. Every 16 x 16 block takes hi.hi + hi.lo + lo.hi on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation: about 16 significant bits per operand
// (|lo| <= 2^-8 |x| after round-to-nearest, so the dropped lo.lo term is at most about 2^-16
// of the product), at three bf16
// products per FP32 one.
//
// Tile 128 x 128 x 64, 256 threads as 2 x 2 wavefronts of 64 x 64 (4 x 4 blocks of 16 x 16),
// two workgroups per CU (74 KB of LDS each). The next slab's global loads are issued before
// the current slab's MFMAs and stored to LDS after them. Only the column-block shape is
// handled (nc a multiple of 128, so a tile's columns share one j and every row's liveness,
// sign and X2 address are wavefront-uniform), with v >= 32; slabs that lie wholly inside the
// tile's zero segment m = j are skipped.
#include "common.h"

namespace gfcc {
namespace {

constexpr int BN = 128;
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef __bf16 b2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef const float __attribute__((address_space(1)))* gptr;   // global loads, not flat

struct Bf3Args {
  const unsigned short* Wh;   // [M][ldw] high parts, rows zero-padded to ldw, then >= BK zeros
  const unsigned short* Wl;   // remainders, same layout
  int64_t ldw;
  const float* X2;            // packed 2h1p block [(pair, e)][ldx]
  const float* zrow;          // >= nc zeros
  float* Z;                   // [M][N]
  int64_t ldx;
  int o, v, nc, M, N, K, mtiles, ntiles;
};

// WM x 2 wavefronts of 64 x 64: tile (64 WM) x 128
template <int BK, int WM, int OCC>
__global__ __launch_bounds__(128 * WM, OCC) void ovvo_bf3_kernel(Bf3Args p) {
  constexpr int BM = 64 * WM, NT = 128 * WM;
  constexpr int LDK = BK + 8;               // LDS row pitch (16 bytes of padding)
  constexpr int CPR = BK / 8;               // 16-byte A chunks per tile row and slab
  constexpr int ACH = BM * CPR / NT;        // A chunks per thread, slab and half
  constexpr int RB = BK * BN / NT;          // B rows per thread and slab
  __shared__ __attribute__((aligned(16))) unsigned short Ah[BM][LDK];
  __shared__ __attribute__((aligned(16))) unsigned short Al[BM][LDK];
  __shared__ __attribute__((aligned(16))) unsigned short Bh[BN][LDK];
  __shared__ __attribute__((aligned(16))) unsigned short Bl[BN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // tile order: workgroups are dealt to the 8 XCDs round robin; XCD x takes the range
  // [x T8, (x+1) T8) of an order that walks 8 M-tiles down before the next N-tile
  constexpr int GM = 8;
  const int ntot = p.mtiles * p.ntiles;
  const int T8 = (ntot + 7) / 8;
  const int L = (int)(blockIdx.x & 7) * T8 + (int)(blockIdx.x >> 3);
  if (L >= ntot) return;
  const int grp = L / (GM * p.ntiles);
  const int rows = min(GM, p.mtiles - grp * GM);
  const int idx = L - grp * GM * p.ntiles;
  const int mt = grp * GM + idx % rows, nt = idx / rows;
  const int m0 = mt * BM, n0 = nt * BN;
  const int o = p.o, v = p.v, M = p.M, nslabs = (p.K + BK - 1) / BK;

  // B ownership: column bn of the tile, rows kh * RB .. kh * RB + RB - 1 of every slab
  const int j = n0 / p.nc;
  const int bn = tid & (BN - 1);
  const int kh = __builtin_amdgcn_readfirstlane(tid / BN);
  const int c = n0 + bn - j * p.nc;
  // slabs [zlo, zhi) lie wholly inside the zero segment m = j
  const int zlo = (j * v + BK - 1) / BK, zhi = ((j + 1) * v) / BK;
  auto skip = [&](int s) { return (s >= zlo && s < zhi) ? zhi : s; };

  // A ownership: chunk r is row (tid + NT r) / CPR, k offset 8 ((tid + NT r) % CPR) of the slab
  int64_t aoff[ACH];
#pragma unroll
  for (int r = 0; r < ACH; ++r) {
    const int f = tid + NT * r;
    aoff[r] = (int64_t)min(m0 + f / CPR, M - 1) * p.ldw + (f % CPR) * 8;
  }

  // scalar base address and row stride of X2 row (pair(mm, j), ee), or of the zero row
  auto seg = [&](int mm, int ee, uint64_t& ptr, uint64_t& stride) {
    const int lo = min(mm, j), hi = max(mm, j);
    const int64_t pr = (int64_t)lo * o - ((lo * (lo + 1)) >> 1) + hi - lo - 1;
    const uint64_t live = 0ull - (uint64_t)((mm < o) & (mm != j));
    const uint64_t a = reinterpret_cast<uint64_t>(p.X2) +
                       (uint64_t)((pr * v + ee) * p.ldx) * sizeof(float);
    ptr = (a & live) | (reinterpret_cast<uint64_t>(p.zrow) & ~live);
    stride = ((uint64_t)p.ldx * sizeof(float)) & live;
  };

  us8 rah[ACH], ral[ACH];
  float rb[RB];
  unsigned rneg = 0;
  // (m, e) of the first B row this thread loads in slab s: k = s BK + kh RB = m v + e
  auto load = [&](int s, int m, int e) {
    const int k0 = s * BK;
#pragma unroll
    for (int r = 0; r < ACH; ++r) {
      rah[r] = *reinterpret_cast<const us8*>(p.Wh + aoff[r] + k0);
      ral[r] = *reinterpret_cast<const us8*>(p.Wl + aoff[r] + k0);
    }
    // rows k = (m, e): the RB rows start at (m, e) and cross at most into segment m + 1
    // (v >= RB); rows r < rc lie in segment m. Rows with m >= o (past K) or m = j read the
    // zero row with stride 0. All of it is wavefront-uniform scalar code without branches.
    const int rc = v - e;
    uint64_t q0, d0, q1, d1;
    seg(m, e, q0, d0);
    seg(m + 1, 0, q1, d1);
    // row r of segment m + 1 sits at q1 + (r - rc) d1: both bases advance by one row stride
    // per row (wrapping arithmetic), so each row costs two 64-bit adds and one select
    uint64_t a0 = q0, a1 = q1 - (uint64_t)rc * d1;
#pragma unroll
    for (int r = 0; r < RB; ++r) {
      rb[r] = reinterpret_cast<gptr>(r < rc ? a0 : a1)[c];
      a0 += d0;
      a1 += d1;
    }
    const unsigned hi = rc >= RB ? 0u : ~0u << rc;   // rows in segment m + 1
    rneg = (m > j ? ~hi : 0u) | (m + 1 > j ? hi : 0u);
  };
  auto store = [&]() {
#pragma unroll
    for (int r = 0; r < ACH; ++r) {
      const int f = tid + NT * r;
      *reinterpret_cast<us8*>(&Ah[f / CPR][(f % CPR) * 8]) = rah[r];
      *reinterpret_cast<us8*>(&Al[f / CPR][(f % CPR) * 8]) = ral[r];
    }
#pragma unroll
    for (int g = 0; g < RB / 8; ++g) {
      u4 hh, ll;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int r = g * 8 + 2 * u;
        const f2 x = {((rneg >> r) & 1u) ? -rb[r] : rb[r],
                      ((rneg >> (r + 1)) & 1u) ? -rb[r + 1] : rb[r + 1]};
        // round to nearest even on the packed converter; bf16 -> f32 is exact
        const b2 h = __builtin_convertvector(x, b2);
        const f2 hf = __builtin_convertvector(h, f2);
        const f2 rem = {x[0] - hf[0], x[1] - hf[1]};
        hh[u] = __builtin_bit_cast(unsigned, h);
        ll[u] = __builtin_bit_cast(unsigned, __builtin_convertvector(rem, b2));
      }
      *reinterpret_cast<u4*>(&Bh[bn][kh * RB + g * 8]) = hh;
      *reinterpret_cast<u4*>(&Bl[bn][kh * RB + g * 8]) = ll;
    }
  };

  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[i][q] = f4{0, 0, 0, 0};

  const int rl = lane & 15, kq = (lane >> 4) * 8;
  auto compute = [&]() {
#pragma unroll
    for (int ks = 0; ks < BK / 32; ++ks) {
      bf8 ah[4], al[4], bh[4], bl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ah[i] = *reinterpret_cast<const bf8*>(&Ah[wm * 64 + i * 16 + rl][ks * 32 + kq]);
        al[i] = *reinterpret_cast<const bf8*>(&Al[wm * 64 + i * 16 + rl][ks * 32 + kq]);
        bh[i] = *reinterpret_cast<const bf8*>(&Bh[wn * 64 + i * 16 + rl][ks * 32 + kq]);
        bl[i] = *reinterpret_cast<const bf8*>(&Bl[wn * 64 + i * 16 + rl][ks * 32 + kq]);
      }
      // lo.hi, hi.lo, then hi.hi, in separate passes over the 16 blocks, so that no MFMA
      // waits on the previous one's accumulator
#pragma unroll
      for (int t = 0; t < 3; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            acc[i][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                t == 0 ? al[i] : ah[i], t == 1 ? bl[q] : bh[q], acc[i][q], 0, 0, 0);
    }
  };

  // at least one slab lies outside the zero segment (o >= 2)
  int s = skip(0);
  int lm = (s * BK + kh * RB) / v, le = s * BK + kh * RB - lm * v;
  load(s, lm, le);
  while (true) {
    store();
    __syncthreads();
    const int sn = skip(s + 1);
    if (sn < nslabs) {
      // advance (m, e) by the slabs moved over (at most v + 2 BK rows after a skip)
      le += (sn - s) * BK;
      while (le >= v) {
        le -= v;
        ++lm;
      }
      load(sn, lm, le);
    }
    compute();
    __syncthreads();
    if (sn >= nslabs) break;
    s = sn;
  }

  const int col = n0 + wn * 64 + rl, rq = (lane >> 4) * 4;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int mrow = m0 + wm * 64 + i * 16 + rq + e;
        if (mrow < M) p.Z[(int64_t)mrow * p.N + col + q * 16] = acc[i][q][e];
      }
}

}  // namespace

bool ovvo_bf3(gfcc_ctx* ctx, int o, int v, int nc, const void* Wh, const void* Wl, int64_t ldw,
              const float* X2, int64_t ldx, float* Z) {
  if (o < 2 || v < 32 || nc < BN || nc % BN != 0 || ldx < nc) return false;
  const int64_t OV = (int64_t)o * v;
  if (!Wh || !Wl || ldw < OV || ldw % 8 != 0 || reinterpret_cast<uintptr_t>(Wh) % 16 != 0 ||
      reinterpret_cast<uintptr_t>(Wl) % 16 != 0)
    return false;
  if (OV >= (1LL << 30) || (int64_t)o * nc >= (1LL << 31)) return false;
  Bf3Args p{};
  p.Wh = static_cast<const unsigned short*>(Wh);
  p.Wl = static_cast<const unsigned short*>(Wl);
  p.ldw = ldw;
  p.X2 = X2;
  p.ldx = ldx;
  p.Z = Z;
  p.o = o; p.v = v; p.nc = nc;
  p.M = (int)OV; p.K = (int)OV; p.N = o * nc;
  constexpr int WM = 2, BM = 64 * WM;
  p.mtiles = (p.M + BM - 1) / BM;
  p.ntiles = p.N / BN;
  const int64_t tiles = (int64_t)p.mtiles * p.ntiles;
  if (tiles >= (1LL << 31) - 8) return false;
  p.zrow = static_cast<const float*>(zero_row(ctx, (size_t)nc * sizeof(float)));
  const dim3 grid((unsigned)((tiles + 7) / 8 * 8));
  // Measured alternatives at o=70, v=260, 512 right-hand sides, all within 3% of this one
  // (about 250 TF/s useful): 32-deep slabs at three workgroups per CU, 256 x 128 tiles of 8
  // wavefronts, and XOR-swizzled LDS rows (half the bank conflicts)
  hipLaunchKernelGGL((ovvo_bf3_kernel<64, WM, 2>), grid, dim3(128 * WM), 0, ctx->stream, p);
  GFCC_LAUNCH_CHECK();
  return true;
}

}  // namespace gfcc
