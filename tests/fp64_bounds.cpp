// CPU check of the FP64 modular arithmetic the NTT passes and the fused key-switch kernels use: this program
// includes the kernels' own header (paper_2403_14111_amd/csrc/ntt_fp64.hpp) and checks, against exact 128-bit
// integer arithmetic, for moduli q < 2^50:
//   fmul(a, w): |a| <= 2^51, 0 <= w < q  ->  congruent to a w, an integer in (-0.75 q, 1.75 q)
//               (|a| <= 2^47: in (-0.05 q, 1.05 q), the bound the lazy forward butterflies use)
//   fred(v):    integer |v| < 2^52       ->  congruent to v, an integer in [0, q]
// and whole 8-stage passes of the butterflies as the kernels chain them, lazy forms included, at the largest
// moduli of each kind (below 2^42 for the lazy forms, below 2^50 for the reducing ones): a forward pass from
// worst-case fused-conversion sums (three terms, in (-2.25 q, 5.25 q)), an inverse pass with its halfway
// reduction and the final stage's scaling, and the key inner product's sums over up to 8 digits.  Every
// intermediate is checked against the precondition of the operation that consumes it.
// Usage: fp64_bounds ITERATIONS; prints the number of failures, exit status 1 on any.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <initializer_list>

#include "ntt_fp64.hpp"

using namespace hetal::fp64;
typedef __int128 i128;

static uint64_t s_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd() {
  s_state ^= s_state << 13;
  s_state ^= s_state >> 7;
  s_state ^= s_state << 17;
  return s_state;
}

static long bad = 0;
static void check(bool ok) { bad += ok ? 0 : 1; }
static i128 mod(i128 v, uint64_t q) {
  i128 r = v % (i128)q;
  return r < 0 ? r + q : r;
}
static bool is_int(double v) { return v == std::floor(v); }

// the operand checks of the helpers: fmul's |a| <= 2^51, fred's |v| < 2^52
static double c_fmul(double a, double w, double q, double qi) {
  check(std::fabs(a) <= 2251799813685248.0 && w >= 0 && w < q);
  return fmul(a, w, q, qi);
}
static double c_fred(double v, double q, double qi) {
  check(std::fabs(v) < 4503599627370496.0);
  return fred(v, q, qi);
}

static void single_ops(uint64_t Q, long iters) {
  const double q = (double)Q, qinv = 1.0 / q;
  const bool small = Q < (1ull << 42);
  for (long it = 0; it < iters; ++it) {
    const bool lazy = small && (it & 1);
    const uint64_t span = lazy ? (1ull << 47) : (1ull << 51);
    int64_t a = (int64_t)(rnd() % (2 * span + 1)) - (int64_t)span;
    uint64_t w = rnd() % Q;
    if (it < 64) {
      a = (it & 2) ? (int64_t)span - (it >> 2) : -(int64_t)span + (it >> 2);
      w = Q - 1 - (uint64_t)(it >> 3) % Q;
    }
    const double r = fmul((double)a, (double)w, q, qinv);
    const double lo = lazy ? -0.05 * q : -0.75 * q, hi = lazy ? 1.05 * q : 1.75 * q;
    check(is_int(r) && mod((i128)a * (i128)w - (i128)r, Q) == 0 && r > lo && r < hi);
    int64_t v = (int64_t)(rnd() % ((1ull << 53) - 1)) - (int64_t)((1ull << 52) - 1);
    if (it < 4096) {
      const int64_t kmax = (int64_t)(((1ull << 52) - 3) / Q) - 1;
      const int64_t k = kmax > 0 ? (int64_t)(it % (2 * kmax + 1)) - kmax : 0;
      v = k * (int64_t)Q + (int64_t)(it % 5) - 2;
    }
    const double rr = fred((double)v, q, qinv);
    check(is_int(rr) && mod((i128)v - (i128)rr, Q) == 0 && rr >= 0 && rr <= q);
  }
}

// One 256-point transform of the pass structure (stages over a 16 x 16 view: 4 stages on one index, 4 on the
// other), with arbitrary twiddles: the butterfly network's positions do not affect the bounds, so each stage
// pairs x[i] with x[i + half] over all 256 values, half = 128, 64, ... (forward) or 1, 2, ... (inverse).
template <bool LAZY>
static void forward_pass(uint64_t Q, int mode) {
  const double q = (double)Q, qi = 1.0 / q;
  double x[256];
  i128 ex[256];
  for (int i = 0; i < 256; ++i) {
    // fused-conversion sums: three products in (-0.75 q, 1.75 q) (reducing form: reduced to [0, q])
    double v;
    if (mode == 0) v = std::floor(5.25 * q) - 1 - (double)(rnd() % 16);
    else if (mode == 1) v = std::ceil(-2.25 * q) + 1 + (double)(rnd() % 16);
    else v = std::floor(((double)(rnd() >> 11) / 9007199254740992.0) * 7.5 * q - 2.25 * q);
    if (!LAZY) v = (double)(rnd() % (Q + 1));
    x[i] = v;
    ex[i] = (i128)v;
  }
  for (int half = 128; half >= 1; half >>= 1)
    for (int i = 0; i < 256; ++i) {
      if (i & half) continue;
      const uint64_t w = mode == 0 ? Q - 1 : rnd() % Q;
      const double xi = x[i], yi = x[i + half];
      check(std::fabs(yi) <= (LAZY ? 140737488355328.0 : q));  // |y| <= 2^47 lazily, [0, q] reduced
      (void)c_fmul(yi, (double)w, q, qi);
      fwd_bfly<LAZY>(x[i], x[i + half], (double)w, q, qi);
      const i128 t = (i128)yi * w;
      ex[i + half] = (i128)xi - t;
      ex[i] = (i128)xi + t;
      for (int k : {i, i + half}) {
        check(is_int(x[k]) && mod(ex[k] - (i128)x[k], Q) == 0);
        if (!LAZY) check(x[k] >= 0 && x[k] <= q);
        ex[k] = (i128)x[k];
      }
    }
  // the pass's final reduction and the store's [0, q) mapping
  for (int i = 0; i < 256; ++i) {
    const double r = ffix(c_fred(x[i], q, qi), q);
    check(r >= 0 && r < q && mod(ex[i] - (i128)r, Q) == 0);
  }
}

// reduce_after: the lazy stages before the one reduction (4 in the passes of 16 elements per thread; 5 covers
// any split of 8 stages into register phases of 2, 3 and 3)
template <bool LAZY>
static void inverse_pass(uint64_t Q, int mode, int reduce_after) {
  const double q = (double)Q, qi = 1.0 / q;
  double x[256];
  i128 ex[256];
  for (int i = 0; i < 256; ++i) {
    x[i] = mode == 0 ? q : (double)(rnd() % (Q + 1));  // inputs in [0, q]
    ex[i] = (i128)x[i];
  }
  int stage = 0;
  for (int half = 1; half <= 128; half <<= 1, ++stage) {
    if (LAZY && stage == reduce_after)
      for (int i = 0; i < 256; ++i) x[i] = c_fred(x[i], q, qi);  // halfway reduction
    const bool last = half == 128;
    for (int i = 0; i < 256; ++i) {
      if (i & half) continue;
      const uint64_t w = mode == 0 ? Q - 1 : rnd() % Q;
      const double xi = x[i], yi = x[i + half];
      if (last) {
        // the transform's last stage with the final scaling merged into both outputs
        const uint64_t k0 = rnd() % Q, k1 = rnd() % Q;
        const double s = xi + yi, d = xi - yi;
        x[i] = ffix(c_fred(c_fmul(s, (double)k0, q, qi), q, qi), q);
        x[i + half] = ffix(c_fred(c_fmul(d, (double)k1, q, qi), q, qi), q);
        check(x[i] >= 0 && x[i] < q && x[i + half] >= 0 && x[i + half] < q);
        check(mod(((i128)xi + (i128)yi) * k0 - (i128)x[i], Q) == 0);
        check(mod(((i128)xi - (i128)yi) * k1 - (i128)x[i + half], Q) == 0);
        continue;
      }
      (void)c_fmul(xi - yi, (double)w, q, qi);
      inv_bfly<LAZY>(x[i], x[i + half], (double)w, q, qi);
      check(is_int(x[i]) && is_int(x[i + half]));
      check(mod((i128)xi + (i128)yi - (i128)x[i], Q) == 0);
      check(mod(((i128)xi - (i128)yi) * w - (i128)x[i + half], Q) == 0);
      if (!LAZY) check(x[i] >= 0 && x[i] <= q && x[i + half] >= 0 && x[i + half] <= q);
      // the lazy sums grow by doubling: at most 2^k q after k stages since the last reduction
      if (LAZY) check(std::fabs(x[i]) <= 32 * q && std::fabs(x[i + half]) <= 32 * q);
    }
  }
  (void)ex;
}

// The key inner product: sum over beta digits of x_j k_j, x_j and k_j in [0, q]; the reducing form folds
// every term in with fred, the lazy one (q < 2^42) sums all beta products and reduces once.
template <bool LAZY>
static void inner_sum(uint64_t Q, int beta, int mode) {
  const double q = (double)Q, qi = 1.0 / q;
  double acc = 0;
  i128 ex = 0;
  for (int j = 0; j < beta; ++j) {
    const uint64_t xv = mode == 0 ? Q : rnd() % (Q + 1), kv = mode == 0 ? Q - 1 : rnd() % Q;
    const double t = c_fmul((double)xv, (double)kv, q, qi);
    acc = LAZY ? acc + t : c_fred(acc + t, q, qi);
    ex += (i128)xv * kv;
  }
  const double r = ffix(c_fred(acc, q, qi), q);
  check(r >= 0 && r < q && mod(ex - (i128)r, Q) == 0);
}

int main(int argc, char** argv) {
  const long iters = argc > 1 ? atol(argv[1]) : 1000000;
  const uint64_t qs[] = {(1ull << 50) - 27, (1ull << 50) - 1, 1125899906842597ull, (1ull << 49) + 1,
                         4398046511093ull /* below 2^42 */, (1ull << 40) - 87, 1099511627689ull, 65537, 12289};
  for (uint64_t Q : qs) single_ops(Q, iters);
  // whole passes at the largest moduli of each form: below 2^42 (lazy) and below 2^50 (reducing)
  const uint64_t lazy_q[] = {4398046511093ull, (1ull << 42) - 11, 1099511627689ull};
  const uint64_t red_q[] = {(1ull << 50) - 27, 1125899906842597ull, (1ull << 49) + 1};
  const long passes = iters / 2000 + 8;
  for (long it = 0; it < passes; ++it) {
    const int mode = it < 6 ? (int)(it % 3) : 2;
    for (uint64_t Q : lazy_q) {
      forward_pass<true>(Q, mode);
      inverse_pass<true>(Q, mode % 2, 4);
      inverse_pass<true>(Q, mode % 2, 5);
      for (int beta = 1; beta <= 8; ++beta) inner_sum<true>(Q, beta, mode % 2);
    }
    for (uint64_t Q : red_q) {
      forward_pass<false>(Q, mode);
      inverse_pass<false>(Q, mode % 2, 4);
      for (int beta = 1; beta <= 8; ++beta) inner_sum<false>(Q, beta, mode % 2);
    }
  }
  printf("%ld\n", bad);
  return bad != 0;
}
