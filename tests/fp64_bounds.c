/* CPU check of the FP64 modular arithmetic of the NTT kernels (paper_2403_14111_amd/csrc/ntt.hip: fmul, fred),
 * against exact 128-bit integer arithmetic, for moduli q < 2^50:
 *   fmul(a, w): |a| <= 2^51, 0 <= w < q  ->  a w - f q exactly, in (-0.75 q, 1.75 q)
 *   fred(v):    integer |v| < 2^52       ->  v - f q exactly, in [0, q]
 * The lazy forward butterflies of moduli below 2^42 rely on fmul of |a| <= 2^47 landing in (-0.05 q, 1.05 q);
 * that is checked too.  Usage: fp64_bounds ITERATIONS; prints the number of failures, exit status 1 on any. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

static uint64_t s = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void) {
  s ^= s << 13;
  s ^= s >> 7;
  s ^= s << 17;
  return s;
}

static double fmul(double a, double w, double q, double qinv, double* f) {
  const double p = a * w;
  const double e = fma(a, w, -p);
  *f = floor(p * qinv);
  return fma(-*f, q, p) + e;
}

static double fred(double v, double q, double qinv, double* f) {
  *f = floor(v * qinv);
  return fma(-*f, q, v);
}

int main(int argc, char** argv) {
  const long iters = argc > 1 ? atol(argv[1]) : 1000000;
  const uint64_t qs[] = {(1ull << 50) - 27, (1ull << 50) - 1, 1125899906842597ull, (1ull << 49) + 1,
                         4398046511093ull /* below 2^42 */, (1ull << 40) - 87, 1099511627689ull, 65537, 12289};
  long bad = 0;
  for (size_t qi = 0; qi < sizeof(qs) / sizeof(qs[0]); ++qi) {
    const uint64_t Q = qs[qi];
    const double q = (double)Q, qinv = 1.0 / q;
    const int small = Q < (1ull << 42);
    for (long it = 0; it < iters; ++it) {
      double f;
      /* fmul over |a| <= 2^51 (2^47 for the lazy bound on small moduli) */
      const int lazy = small && (it & 1);
      const uint64_t span = lazy ? (1ull << 47) : (1ull << 51);
      int64_t a = (int64_t)(rnd() % (2 * span + 1)) - (int64_t)span;
      uint64_t w = rnd() % Q;
      if (it < 64) {
        a = (it & 2) ? (int64_t)span - (it >> 2) : -(int64_t)span + (it >> 2);
        w = Q - 1 - (uint64_t)(it >> 3) % Q;
      }
      const double r = fmul((double)a, (double)w, q, qinv, &f);
      const __int128 ex = (__int128)a * (__int128)w - (__int128)(int64_t)f * (__int128)Q;
      const double lo = lazy ? -0.05 * q : -0.75 * q, hi = lazy ? 1.05 * q : 1.75 * q;
      if ((__int128)r != ex || !(r > lo && r < hi)) ++bad;
      /* fred over |v| < 2^52, with near-multiples of q */
      int64_t v = (int64_t)(rnd() % ((1ull << 53) - 1)) - (int64_t)((1ull << 52) - 1);
      if (it < 4096) {
        const int64_t kmax = (int64_t)(((1ull << 52) - 3) / Q) - 1;
        const int64_t k = kmax > 0 ? (int64_t)(it % (2 * kmax + 1)) - kmax : 0;
        v = k * (int64_t)Q + (int64_t)(it % 5) - 2;
      }
      const double rr = fred((double)v, q, qinv, &f);
      const __int128 ex2 = (__int128)v - (__int128)(int64_t)f * (__int128)Q;
      if ((__int128)rr != ex2 || !(rr >= 0 && rr <= q)) ++bad;
    }
  }
  printf("%ld\n", bad);
  return bad != 0;
}
