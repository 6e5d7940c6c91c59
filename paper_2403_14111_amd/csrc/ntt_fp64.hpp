// Exact modular arithmetic on residues held in FP64, as the NTT passes and the fused key-switch kernels use it.
//
// Every modulus is a prime q < 2^50; residues are integers held exactly in doubles (below 2^53).  The
// method is Dekker's exact product (the error of a rounded product recovered by one fused multiply-add,
// "TwoProduct" with an FMA) followed by a floor-quotient reduction:
//   * fmul: for integers |a| <= 2^51 and 0 <= w < q, p = fl(a w) and e = fma(a, w, -p) give a w = p + e
//     exactly; f = floor(fl(p fl(1/q))) is within one of floor(a w / q) (the relative error of the
//     quotient estimate is below 3 * 2^-53 and a w / q < 2^52), so fma(-f, q, p) + e = a w - f q is exact
//     and lies in (-0.75 q, 1.75 q);
//   * fred: for an integer |v| < 2^52, fma(-floor(fl(v fl(1/q))), q, v) is exact and lies in [0, q].
// The butterflies built on them either reduce both outputs back to [0, q] (any q < 2^50) or, for q below
// LAZY_MODULUS = 2^42, leave them unreduced within a pass (bounds at fwd_bfly / inv_bfly).
//
// The arithmetic helpers are host and device functions: a CPU test compiles this header with a host
// compiler and checks them against exact integer arithmetic.  Contraction is off throughout: every
// product, sum and FMA above is the operation written.
#pragma once

#if defined(__HIPCC__)
#define HETAL_HD __host__ __device__ __forceinline__
#else
#define HETAL_HD inline
#endif

namespace hetal {
namespace fp64 {

// Moduli below this take the lazy butterflies.
constexpr double LAZY_MODULUS = 4398046511104.0;  // 2^42

// a w mod q, exact, in (-0.75q, 1.75q), for integers |a| <= 2^51 and 0 <= w < q < 2^50.
HETAL_HD double fmul(double a, double w, double q, double qinv) {
#pragma clang fp contract(off)
  const double p = a * w;
  const double e = __builtin_fma(a, w, -p);
  const double f = __builtin_floor(p * qinv);
  return __builtin_fma(-f, q, p) + e;
}

// v mod q, exact, in [0, q], for integers |v| < 2^52.
HETAL_HD double fred(double v, double q, double qinv) {
#pragma clang fp contract(off)
  return __builtin_fma(-__builtin_floor(v * qinv), q, v);
}

// [0, q] -> [0, q)
HETAL_HD double ffix(double v, double q) { return v >= q ? v - q : v; }

// Cooley-Tukey butterfly: T = y w, then x + T and x - T.  Reduced (LAZY false): inputs and outputs in
// [0, q].  LAZY (moduli below 2^42 only): nothing is reduced; with |y| <= 2^47 the product T lies in
// (-0.05q, 1.05q), so each stage widens the bound by 1.05q: 8 stages from inputs below 5.5q stay below
// 5.5q + 8 * 1.05q = 13.9q < 2^46.
template <bool LAZY>
HETAL_HD void fwd_bfly(double& x, double& y, double w, double q, double qinv) {
#pragma clang fp contract(off)
  const double t = fmul(y, w, q, qinv);
  if (LAZY) {
    y = x - t;
    x = x + t;
  } else {
    y = fred(x - t, q, qinv);
    x = fred(x + t, q, qinv);
  }
}

// Gentleman-Sande butterfly: x + y, and (x - y) w.  Reduced: [0, q] in and out.  LAZY (moduli below
// 2^42): nothing is reduced; the sum doubles the bound per stage (the difference's product stays in
// (-0.75q, 1.75q)), so from [0, q] four stages stay below 16q and a pass of eight reduces once halfway.
template <bool LAZY>
HETAL_HD void inv_bfly(double& x, double& y, double w, double q, double qinv) {
#pragma clang fp contract(off)
  const double s = x + y;
  const double d = x - y;
  if (LAZY) {
    y = fmul(d, w, q, qinv);
    x = s;
  } else {
    y = fred(fmul(d, w, q, qinv), q, qinv);
    x = fred(s, q, qinv);
  }
}

}  // namespace fp64
}  // namespace hetal

#undef HETAL_HD
