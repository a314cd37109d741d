/*
 * Seeded synthetic inputs for the IP-GFCC problem: orbital energies, T1 amplitudes and
 * blocks of the antisymmetrised two-electron integral tensor <pq||rs>.
 *
 * This file holds no part of the Green's-function method. It only draws random numbers.
 *
 * Every value is a pure function of (seed, stream, key), so any block of the integral
 * tensor can be produced on its own and agrees with every other block on shared elements.
 *
 * Generator: SplitMix64 (G. Steele, D. Lea, C. Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) used as a counter-based hash; normals by the Box-Muller transform.
 *
 * Integral model: chemists'-notation values (pr|qs) = g are iid N(0,1), one per class of the
 * 8-fold real-orbital symmetry {(pr|qs) = (rp|qs) = (pr|sq) = (qs|pr) ...}. Then
 *   <pq|rs>  = (pr|qs)
 *   <pq||rs> = scale/sqrt(2) * ( <pq|rs> - <pq|sr> )
 * which is exactly antisymmetric in each index pair, Hermitian (<pq||rs> = <rs||pq>) and has
 * standard deviation `scale` off the symmetry-degenerate index sets.
 */
#include <math.h>
#include <stdint.h>

static inline uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t hash3(uint64_t seed, uint64_t stream, uint64_t key) {
  return splitmix64(splitmix64(splitmix64(seed) ^ (stream * 0xD1B54A32D192ED03ULL)) ^ key);
}

/* uniform in the open interval (0, 1) */
static inline double u01(uint64_t h) { return ((double)(h >> 11) + 0.5) * 0x1.0p-53; }

static inline double normal_of(uint64_t seed, uint64_t stream, uint64_t key) {
  const double two_pi = 6.283185307179586476925286766559;
  double u1 = u01(hash3(seed, stream, 2 * key));
  double u2 = u01(hash3(seed, stream, 2 * key + 1));
  return sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
}

static inline uint64_t tri(uint64_t a, uint64_t b) { /* a >= b */
  return a * (a + 1) / 2 + b;
}

/* canonical key of the 8-fold symmetry class of (pr|qs) */
static inline uint64_t eri_key(uint64_t p, uint64_t q, uint64_t r, uint64_t s) {
  uint64_t x = p > r ? tri(p, r) : tri(r, p);
  uint64_t y = q > s ? tri(q, s) : tri(s, q);
  return x > y ? tri(x, y) : tri(y, x);
}

void synth_uniform(uint64_t seed, uint64_t stream, int64_t n, double lo, double hi,
                   double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = lo + (hi - lo) * u01(hash3(seed, stream, (uint64_t)i));
}

void synth_normal(uint64_t seed, uint64_t stream, int64_t n, double sigma, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = sigma * normal_of(seed, stream, (uint64_t)i);
}

/*
 * out[ip][iq][ir][is] = <p q || r s> with p = p0 + ip, q = q0 + iq, r = r0 + ir, s = s0 + is
 * (global spin-orbital indices; row-major, `is` fastest).
 */
void synth_eri_block(uint64_t seed, uint64_t stream, double scale, int64_t p0, int64_t np,
                     int64_t q0, int64_t nq, int64_t r0, int64_t nr, int64_t s0, int64_t ns,
                     double* out) {
  const double f = scale * 0.70710678118654752440084436210485;
#pragma omp parallel for collapse(2) schedule(static)
  for (int64_t ip = 0; ip < np; ++ip)
    for (int64_t iq = 0; iq < nq; ++iq) {
      uint64_t p = (uint64_t)(p0 + ip), q = (uint64_t)(q0 + iq);
      double* row = out + ((ip * nq + iq) * nr) * ns;
      for (int64_t ir = 0; ir < nr; ++ir) {
        uint64_t r = (uint64_t)(r0 + ir);
        for (int64_t is = 0; is < ns; ++is) {
          uint64_t s = (uint64_t)(s0 + is);
          double g1 = normal_of(seed, stream, eri_key(p, q, r, s)); /* <pq|rs> = (pr|qs) */
          double g2 = normal_of(seed, stream, eri_key(p, q, s, r)); /* <pq|sr> = (ps|qr) */
          row[ir * ns + is] = f * (g1 - g2);
        }
      }
    }
}
