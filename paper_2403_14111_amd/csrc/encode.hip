// CKKS encoding and decoding on the GPU, and the block layout of matrices.
//
// Encoding computes m_j = (1/N) sum_{e odd} Z[e] w^(-e j), w = exp(2 pi i / 2N),
// where Z[5^k mod 2N] = z_k and Z[-5^k mod 2N] = conj(z_k): the inverse
// canonical embedding with slot k at zeta^(5^k).  It is evaluated as a
// radix-2 DFT of size 2N in double-double arithmetic (error ~2^-100 relative),
// then scaled and rounded half to even with a 2^-24 tie window, so that the
// integer coefficients do not depend on the order of the floating-point work.
// Decoding evaluates the plaintext polynomial at the same points with the
// same DFT (sign +), from the centred CRT value of the first two limbs.
#include "hetal_internal.hpp"

#pragma clang fp contract(off)

namespace hetal {

namespace {

struct dd {
  double hi, lo;
};
struct cdd {
  dd re, im;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double v = s - a;
  return dd{s, (a - (s - v)) + (b - v)};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
  double s = a + b;
  return dd{s, b - (s - a)};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
  double p = a * b;
  return dd{p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return fast_two_sum(p.hi, p.lo);
}
__device__ __forceinline__ dd dd_div_d(dd a, double b) {
  double q1 = a.hi / b;
  dd r = dd_sub(a, two_prod(q1, b));
  return fast_two_sum(q1, (r.hi + r.lo) / b);
}
__device__ __forceinline__ cdd cdd_mul(cdd a, cdd b) {
  return cdd{dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
}

__device__ __forceinline__ cdd load_cdd(const double* p) { return cdd{dd{p[0], p[1]}, dd{p[2], p[3]}}; }
__device__ __forceinline__ void store_cdd(double* p, cdd v) {
  p[0] = v.re.hi;
  p[1] = v.re.lo;
  p[2] = v.im.hi;
  p[3] = v.im.lo;
}

// exp(2 pi i j / m): the angle is folded into [0, pi/4] (quadrant rotation by
// i^q and the complement pi/2 - x are exact) and the series of cos and sin
// are summed in double-double.
__global__ void roots_kernel(double* __restrict__ roots, int log_m) {
  const long m = 1l << log_m;
  const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const long quarter = m >> 2, eighth = m >> 3;
  const long quad = j / quarter;
  long r = j % quarter;
  bool complement = r > eighth;
  if (complement) r = quarter - r;
  const dd pi = dd{3.141592653589793116e+00, 1.224646799147353207e-16};
  const dd x = dd_mul_d(pi, 2.0 * (double)r / (double)m);
  const dd x2 = dd_mul(x, x);
  dd term = x, s = x;
  for (int k = 1; k < 40 && fabs(term.hi) > 1e-40; ++k) {
    term = dd_neg(dd_div_d(dd_mul(term, x2), (double)(2 * k) * (double)(2 * k + 1)));
    s = dd_add(s, term);
  }
  dd c = dd{1.0, 0.0};
  term = c;
  for (int k = 1; k < 40 && fabs(term.hi) > 1e-40; ++k) {
    term = dd_neg(dd_div_d(dd_mul(term, x2), (double)(2 * k - 1) * (double)(2 * k)));
    c = dd_add(c, term);
  }
  cdd w = complement ? cdd{s, c} : cdd{c, s};
  for (long t = 0; t < quad; ++t) w = cdd{dd_neg(w.im), w.re};
  store_cdd(roots + 4 * j, w);
}

__device__ __forceinline__ u32 brev_bits(u32 x, int bits) { return __builtin_bitreverse32(x) >> (32 - bits); }

// Z (bit-reversed positions of a size-2N array) from the slots of `count` messages.
__global__ void encode_scatter_kernel(const double* __restrict__ re, const double* __restrict__ im, size_t slot_stride,
                                      const u32* __restrict__ pow5, double* __restrict__ z, int log_n) {
  const int n = 1 << log_n;
  const int log_m = log_n + 1;
  const int m = 2 * n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n / 2) return;
  const size_t b = blockIdx.y;
  const double vr = re[b * slot_stride + k];
  const double vi = im ? im[b * slot_stride + k] : 0.0;
  const u32 e = pow5[k];
  double* zb = z + b * (size_t)m * 4;
  store_cdd(zb + 4 * (size_t)brev_bits(e, log_m), cdd{dd{vr, 0.0}, dd{vi, 0.0}});
  store_cdd(zb + 4 * (size_t)brev_bits((u32)(m - e), log_m), cdd{dd{vr, 0.0}, dd{-vi, 0.0}});
}

// Scatter of integer coefficients (decode): position brev(j) <- m_j, j < N (the rest stays 0).
__global__ void decode_scatter_kernel(const u64* __restrict__ m, int limbs, const ModInfo* __restrict__ mods,
                                      const PrimeConsts* __restrict__ pc, double* __restrict__ z, int log_n,
                                      u64 q0_inv_mod_q1) {
  const int n = 1 << log_n;
  const int log_m = log_n + 1;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const u64 q0 = mods[0].q;
  u64 mag_hi = 0, mag_lo;
  bool negative;
  if (limbs == 1) {
    const u64 x = m[j];
    negative = x > (q0 >> 1);
    mag_lo = negative ? q0 - x : x;
  } else {
    const ModInfo m1 = mods[1];
    const u64 x0 = m[j], x1 = m[(size_t)n + j];
    const u64 t = mul_mod(sub_mod(x1, reduce64(x0, m1), m1.q), q0_inv_mod_q1, m1);
    U128 x = mul_wide(q0, t);
    acc_wide(x, U128{x0, 0});
    const U128 big = mul_wide(q0, m1.q);
    const U128 half = U128{(big.lo >> 1) | (big.hi << 63), big.hi >> 1};
    negative = x.hi > half.hi || (x.hi == half.hi && x.lo > half.lo);
    if (negative) {  // big - x
      mag_lo = big.lo - x.lo;
      mag_hi = big.hi - x.hi - (big.lo < x.lo ? 1 : 0);
    } else {
      mag_lo = x.lo;
      mag_hi = x.hi;
    }
  }
  // exact double-double value of the magnitude from three exactly representable pieces
  dd v = dd_add(dd_add(dd{(double)mag_hi * 18446744073709551616.0, 0.0}, dd{(double)(mag_lo >> 32) * 4294967296.0, 0.0}),
                dd{(double)(mag_lo & 0xffffffffull), 0.0});
  if (negative) v = dd_neg(v);
  store_cdd(z + 4 * (size_t)brev_bits((u32)j, log_m), cdd{v, dd{0.0, 0.0}});
}

// One radix-2 stage (butterfly span `half`) of the DFT X[k] = sum_j x[j] w^(sign j k).
__global__ void dft_stage_kernel(double* __restrict__ z, const double* __restrict__ roots, int log_m, int log_half,
                                 int sign) {
  const int m = 1 << log_m;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m / 2) return;
  const int half = 1 << log_half;
  const int jj = t & (half - 1);
  const int base = ((t >> log_half) << (log_half + 1)) + jj;
  double* zb = z + (size_t)blockIdx.y * m * 4;
  const int e = (jj << (log_m - log_half - 1)) & (m - 1);
  cdd w = load_cdd(roots + 4 * (size_t)(sign > 0 ? e : ((m - e) & (m - 1))));
  cdd u = load_cdd(zb + 4 * (size_t)base);
  cdd v = cdd_mul(load_cdd(zb + 4 * (size_t)(base + half)), w);
  store_cdd(zb + 4 * (size_t)base, cdd{dd_add(u.re, v.re), dd_add(u.im, v.im)});
  store_cdd(zb + 4 * (size_t)(base + half), cdd{dd_sub(u.re, v.re), dd_sub(u.im, v.im)});
}

// Round half to even; within 2^-24 of a half-integer counts as a half.
__device__ __forceinline__ bool round_dd(dd v, i64* out) {
  if (!(fabs(v.hi) < 4611686018427387904.0)) return false;
  const double fh = floor(v.hi);
  i64 f;
  double frac;
  if (fh == v.hi) {
    const double fl = floor(v.lo);
    f = (i64)v.hi + (i64)fl;
    frac = v.lo - fl;
  } else {
    f = (i64)fh;
    frac = (v.hi - fh) + v.lo;
  }
  const double d = frac - 0.5;
  if (fabs(d) <= 5.9604644775390625e-08) *out = f + (f & 1);
  else *out = f + (d > 0.0 ? 1 : 0);
  return true;
}

// Coefficients m_j = round(scale * Re(X[j]) / N), reduced into each limb (coefficient form).
__global__ void encode_round_kernel(const double* __restrict__ z, u64* __restrict__ out, size_t out_stride,
                                    const ModInfo* __restrict__ mods, int log_n, int level, double scale,
                                    int* __restrict__ status) {
  const int n = 1 << log_n;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const size_t b = blockIdx.y;
  const double* zb = z + b * (size_t)(2 * n) * 4;
  dd v = dd{zb[4 * (size_t)j], zb[4 * (size_t)j + 1]};
  v = dd_mul_d(dd_div_d(v, (double)n), scale);
  i64 c = 0;
  if (!round_dd(v, &c)) {
    status[0] = 1;
    c = 0;
  }
  const u64 mag = c < 0 ? (u64)(-c) : (u64)c;
  u64* o = out + b * out_stride;
  for (int i = 0; i <= level; ++i) {
    const ModInfo md = mods[i];
    const u64 r = reduce64(mag, md);
    o[(size_t)i * n + j] = c < 0 ? neg_mod(r, md.q) : r;
  }
}

// Slots z_k = X[5^k] / scale.
__global__ void decode_gather_kernel(const double* __restrict__ z, const u32* __restrict__ pow5, double scale,
                                     double* __restrict__ re, double* __restrict__ im, int log_n) {
  const int n = 1 << log_n;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n / 2) return;
  const cdd v = load_cdd(z + 4 * (size_t)pow5[k]);
  const dd r = dd_div_d(v.re, scale), i = dd_div_d(v.im, scale);
  re[k] = r.hi + r.lo;
  if (im) im[k] = i.hi + i.lo;
}

// Slot vectors of the blocks of a (tiled, zero padded) matrix, block (bi, bj) at bi * n_cb + bj.
__global__ void block_layout_kernel(const double* __restrict__ mat, int rows, int cols, int tiling, int c, int s0,
                                    int s1, int n_cb, double* __restrict__ slots) {
  const int s = s0 * s1;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= s) return;
  const int blk = blockIdx.y;
  const int bi = blk / n_cb, bj = blk % n_cb;
  const int r = t / s1, col = t % s1;
  long R = (long)bi * s0 + r, C = (long)bj * s1 + col;
  if (tiling == 1) R %= c;
  if (tiling == 2) C %= c;
  slots[(size_t)blk * s + t] = (R < rows && C < cols) ? mat[R * cols + C] : 0.0;
}

constexpr int EB = 256;

void run_dft(Context& c, double* z, int batch, int sign) {
  const int log_m = c.log_n + 1;
  const int m = 1 << log_m;
  for (int lh = 0; lh < log_m; ++lh) {
    c.begin_launch();
  hipLaunchKernelGGL(dft_stage_kernel, dim3((m / 2 + EB - 1) / EB, batch), dim3(EB), 0, c.stream, z, c.d_roots,
                       log_m, lh, sign);
    c.end_launch(KC_ENCODE, 0.0);
  }
}

}  // namespace

void make_roots(Context& c) {
  const int log_m = c.log_n + 1;
  const int m = 1 << log_m;
  c.begin_launch();
  hipLaunchKernelGGL(roots_kernel, dim3((m + EB - 1) / EB), dim3(EB), 0, c.stream, c.d_roots, log_m);
  c.end_launch(KC_ENCODE, 0.0);
}

void k_encode(Context& c, const double* d_re, const double* d_im, int count, size_t slot_stride, int level,
              double scale, u64* out, size_t out_stride, int* d_status) {
  const size_t m = 2 * (size_t)c.n;
  Tmp zbuf(c.pool, (size_t)count * m * 4);
  double* z = reinterpret_cast<double*>(zbuf.p);
  HCHECK(hipMemsetAsync(z, 0, (size_t)count * m * 4 * sizeof(double), c.stream));
  c.begin_launch();
  hipLaunchKernelGGL(encode_scatter_kernel, dim3((c.slots + EB - 1) / EB, count), dim3(EB), 0, c.stream, d_re, d_im,
                     slot_stride, c.d_pow5, z, c.log_n);
  c.end_launch(KC_ENCODE, 0.0);
  run_dft(c, z, count, -1);
  c.begin_launch();
  hipLaunchKernelGGL(encode_round_kernel, dim3((c.n + EB - 1) / EB, count), dim3(EB), 0, c.stream, z, out, out_stride,
                     c.d_mod, c.log_n, level, scale, d_status);
  c.end_launch(KC_ENCODE, 0.0);
  RowsRef rows = c.rows(ROWS_CT, level);
  ntt_forward(c, out, out_stride, count, RowsRef{rows.d, level + 1});
}

void k_decode(Context& c, const u64* m_coeff, int level, double scale, double* d_re, double* d_im) {
  const size_t m = 2 * (size_t)c.n;
  Tmp zbuf(c.pool, m * 4);
  double* z = reinterpret_cast<double*>(zbuf.p);
  HCHECK(hipMemsetAsync(z, 0, m * 4 * sizeof(double), c.stream));
  const int limbs = level >= 1 ? 2 : 1;
  u64 q0_inv = 0;
  if (limbs == 2) {
    // q_0^-1 mod q_1 by Fermat
    const u64 q1 = c.primes[1];
    unsigned __int128 r = 1, b = c.primes[0] % q1;
    u64 e = q1 - 2;
    while (e) {
      if (e & 1) r = r * b % q1;
      b = b * b % q1;
      e >>= 1;
    }
    q0_inv = (u64)r;
  }
  c.begin_launch();
  hipLaunchKernelGGL(decode_scatter_kernel, dim3((c.n + EB - 1) / EB), dim3(EB), 0, c.stream, m_coeff, limbs, c.d_mod,
                     c.d_pc, z, c.log_n, q0_inv);
  c.end_launch(KC_ENCODE, 0.0);
  run_dft(c, z, 1, +1);
  c.begin_launch();
  hipLaunchKernelGGL(decode_gather_kernel, dim3((c.slots + EB - 1) / EB), dim3(EB), 0, c.stream, z, c.d_pow5, scale,
                     d_re, d_im, c.log_n);
  c.end_launch(KC_ENCODE, 0.0);
}

void k_block_layout(Context& c, const double* d_mat, int rows, int cols, int tiling, int c_rep, int s0, int s1,
                    int n_rb, int n_cb, double* d_slots) {
  c.begin_launch();
  hipLaunchKernelGGL(block_layout_kernel, dim3((s0 * s1 + EB - 1) / EB, n_rb * n_cb), dim3(EB), 0, c.stream, d_mat,
                     rows, cols, tiling, c_rep, s0, s1, n_cb, d_slots);
  c.end_launch(KC_ENCODE, 0.0);
}

}  // namespace hetal
