// RNS kernels for gfx950 and the key-switch and rescale schedules built on them.
//
// A hybrid key switch (Sec. 2.2) runs as: the inverse NTT of the input's c1,
// its last stage also applying the ModUp conversion's first factor; the
// forward NTT of the ModUp rows, its first pass computing the conversion; the
// key inner product, with the Galois automorphism fused into its loads; the
// inverse NTT of the special rows, scaled for ModDown's conversion; and the
// forward NTT of the ModDown rows, with the conversion in its first pass and
// the combine (acc - conv) P^-1 + addends in its last (see ntt.hip).  The
// standalone ModUp / ModDown conversion kernels here serve parameter sets the
// fused passes do not cover (more than 4 terms, or other ring sizes).
//
// The kernels stream limbs through HBM once; each thread handles one
// coefficient index, so consecutive lanes touch consecutive words of a limb.
#include "hetal_internal.hpp"

namespace hetal {

namespace {

constexpr int TPB = 256;

inline dim3 grid_for(const Context& c, int y, int z) { return dim3((unsigned)(c.n / TPB), (unsigned)y, (unsigned)z); }

// Device address of a field of a device-resident table (address arithmetic only, nothing is read).
template <class T, class S>
const T* device_field(const S* table, size_t offset) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(table) + offset);
}

// ---------------------------------------------------------------- ModUp
// For digit j (blockIdx.y): every row of the extended basis outside the digit q_0..q_l, p_0..p_{K-1} receives the fast
// basis conversion of the digit's coefficient-form residues
//   sum_i [x_i (D/d_i)^-1]_{d_i} (D/d_i) mod t
// as a sum of lazy Shoup products by the constants (D/d_i) mod t (each below 4t, the sum below 4 ALPHA t < 2^55),
// reduced once.  ALPHA is the digit length; a shorter last digit takes zero terms.
template <int ALPHA>
__global__ void __launch_bounds__(TPB) modup_kernel(const u64* __restrict__ coef, size_t coef_stride,
                                                    u64* __restrict__ dt, size_t dt_stride,
                                                    const ModUpTab* __restrict__ tabs, const ModInfo* __restrict__ mods,
                                                    int log_n, int level, int num_q, int num_p) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int ext = l + num_p;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int jd = blockIdx.y;
  const ModUpTab& tb = tabs[jd];
  const u64* __restrict__ cf = coef + blockIdx.z * coef_stride;
  u64* __restrict__ out = dt + blockIdx.z * dt_stride + (size_t)jd * ext * n;
  u64 y[ALPHA];
#pragma unroll
  for (int i = 0; i < ALPHA; ++i) {
    const int s = tb.first + (i < tb.nsrc ? i : 0);
    const u64 v = mul_shoup(cf[(size_t)s * n + k], tb.dinv[i], tb.dinv_sh[i], mods[s].q);
    y[i] = i < tb.nsrc ? v : 0;
  }
  for (int r = 0; r < ext; ++r) {
    if (r >= tb.first && r < tb.first + tb.nsrc) continue;  // the digit's own rows are read from the input
    const int t = r < l ? r : num_q + (r - l);
    const u64 q = mods[t].q, nq = 0 - q;
    u64 s = mul_shoup_lazy4n(y[0], tb.dhat[0][t], tb.dhat_sh[0][t], nq);
#pragma unroll
    for (int i = 1; i < ALPHA; ++i) s += mul_shoup_lazy4n(y[i], tb.dhat[i][t], tb.dhat_sh[i][t], nq);
    out[(size_t)r * n + k] = csub(csub(reduce_lazy4(s, mods[t].one_sh, nq), 2 * q), q);
  }
}

// ---------------------------------------------------------------- key inner product
// acc_b[r][k] = sum_j dt_j[r][src(k)] * b_j[t][k], acc_a likewise, where src is
// the Galois gather of the automorphism (identity for g = 1) and t the global
// prime of extended row r.  BETA is the number of digits at the level.
struct IpArgs {
  const u64* key[MAX_BATCH];
  u32 g[MAX_BATCH];
};

template <int BETA>
__global__ void __launch_bounds__(TPB) inner_product_kernel(const u64* __restrict__ dt, size_t dt_stride,
                                                            const u64* __restrict__ in, size_t in_stride,
                                                            u64* __restrict__ acc, size_t acc_stride, IpArgs args,
                                                            const ModInfo* __restrict__ mods, int log_n, int level,
                                                            int num_q, int num_p, int nprimes, int alpha) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int ext = l + num_p;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int r = blockIdx.y;
  const int item = blockIdx.z;
  const int t = r < l ? r : num_q + (r - l);
  const u32 g = args.g[item];
  const u64* __restrict__ key = args.key[item];
  const u64* __restrict__ d = dt + item * dt_stride + (size_t)r * n;
  const u64* __restrict__ own = in + item * in_stride + (size_t)r * n;
  const int rd = r < l ? r / alpha : -1;  // the digit that row r belongs to
  const u32 src = g == 1 ? (u32)k : galois_source((u32)k, g, log_n);
  u64 x[BETA];
#pragma unroll
  for (int j = 0; j < BETA; ++j) x[j] = j == rd ? own[src] : d[(size_t)j * ext * n + src];
  U128 sb = {0, 0}, sa = {0, 0};
#pragma unroll
  for (int j = 0; j < BETA; ++j) {
    acc_wide(sb, mul_wide(x[j], key[((size_t)(2 * j) * nprimes + t) * n + k]));
    acc_wide(sa, mul_wide(x[j], key[((size_t)(2 * j + 1) * nprimes + t) * n + k]));
  }
  const ModInfo m = mods[t];
  u64* __restrict__ o = acc + item * acc_stride;
  o[(size_t)r * n + k] = reduce128(sb, m);
  o[(size_t)(ext + r) * n + k] = reduce128(sa, m);
}

// Same, for `count` items that share one key and Galois element: the key
// words are loaded once per coefficient and reused for every item; two items
// are in flight at a time.
template <int BETA>
__global__ void __launch_bounds__(TPB) inner_product_shared_kernel(const u64* __restrict__ dt, size_t dt_stride,
                                                                   const u64* __restrict__ in, size_t in_stride,
                                                                   u64* __restrict__ acc, size_t acc_stride,
                                                                   const u64* __restrict__ key, u32 g, int count,
                                                                   const ModInfo* __restrict__ mods, int log_n,
                                                                   int level, int num_q, int num_p, int nprimes,
                                                                   int alpha) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int ext = l + num_p;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int r = blockIdx.y;
  const int t = r < l ? r : num_q + (r - l);
  const u32 src = g == 1 ? (u32)k : galois_source((u32)k, g, log_n);
  u64 kb[BETA], ka[BETA];
#pragma unroll
  for (int j = 0; j < BETA; ++j) {
    kb[j] = key[((size_t)(2 * j) * nprimes + t) * n + k];
    ka[j] = key[((size_t)(2 * j + 1) * nprimes + t) * n + k];
  }
  const ModInfo m = mods[t];
  const int rd = r < l ? r / alpha : -1;  // the digit that row r belongs to
  auto load = [&](int item, u64 (&x)[BETA]) {
    const u64* __restrict__ d = dt + item * dt_stride + (size_t)r * n;
    const u64* __restrict__ own = in + item * in_stride + (size_t)r * n;
#pragma unroll
    for (int j = 0; j < BETA; ++j) x[j] = j == rd ? own[src] : d[(size_t)j * ext * n + src];
  };
  auto finish = [&](int item, const u64 (&x)[BETA]) {
    U128 sb = {0, 0}, sa = {0, 0};
#pragma unroll
    for (int j = 0; j < BETA; ++j) {
      acc_wide(sb, mul_wide(x[j], kb[j]));
      acc_wide(sa, mul_wide(x[j], ka[j]));
    }
    u64* __restrict__ o = acc + item * acc_stride;
    o[(size_t)r * n + k] = reduce128(sb, m);
    o[(size_t)(ext + r) * n + k] = reduce128(sa, m);
  };
  int item = 0;
  for (; item + 1 < count; item += 2) {
    u64 x0[BETA], x1[BETA];
    load(item, x0);
    load(item + 1, x1);
    finish(item, x0);
    finish(item + 1, x1);
  }
  if (item < count) {
    u64 x0[BETA];
    load(item, x0);
    finish(item, x0);
  }
}

// ---------------------------------------------------------------- ModDown
// Centred conversion of the special-prime part (coefficient form) to each q_i:
// y_k = [x_k (P/p_k)^-1]_{p_k} taken in (-p_k/2, p_k/2]; conv_i = sum_k y_k (P/p_k) mod q_i.  K special primes.
// Each term is a lazy Shoup product |y_k| (P/p_k) in [0, 4 q_i), negated as 4 q_i - it; one reduction ends the sum.
template <int K>
__global__ void __launch_bounds__(TPB) moddown_conv_kernel(const u64* __restrict__ acc, size_t acc_stride,
                                                           u64* __restrict__ conv, size_t conv_stride,
                                                           const ModDownTab* __restrict__ tab,
                                                           const ModInfo* __restrict__ mods, int log_n, int level,
                                                           int num_q) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int ext = l + K;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int poly = blockIdx.y;
  const u64* __restrict__ a = acc + blockIdx.z * acc_stride + (size_t)poly * ext * n;
  u64* __restrict__ o = conv + blockIdx.z * conv_stride + (size_t)poly * l * n;
  u64 y[K];
  bool neg[K];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    const u64 pk = mods[num_q + kk].q;
    const u64 v = mul_shoup(a[(size_t)(l + kk) * n + k], tab->pkinv[kk], tab->pkinv_sh[kk], pk);
    neg[kk] = v > (pk >> 1);
    y[kk] = neg[kk] ? pk - v : v;
  }
  for (int i = 0; i < l; ++i) {
    const u64 q = mods[i].q, nq = 0 - q, q4 = 4 * q;
    u64 s = 0;
#pragma unroll
    for (int kk = 0; kk < K; ++kk) {
      const u64 t = mul_shoup_lazy4n(y[kk], tab->phat[kk][i], tab->phat_sh[kk][i], nq);
      s += neg[kk] ? q4 - t : t;
    }
    o[(size_t)i * n + k] = csub(csub(reduce_lazy4(s, mods[i].one_sh, nq), 2 * q), q);
  }
}

// ---------------------------------------------------------------- rescale
// top[p][k] = coefficient-form limb `level` of poly p; spread[p][i][k] = [top]_centred mod q_i.
__global__ void __launch_bounds__(TPB) rescale_spread_kernel(const u64* __restrict__ top, size_t top_stride,
                                                             u64* __restrict__ spread, size_t spread_stride,
                                                             const ModInfo* __restrict__ mods, int log_n, int level) {
  const int n = 1 << log_n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int poly = blockIdx.y;
  const u64 qt = mods[level].q;
  const u64 x = top[blockIdx.z * top_stride + (size_t)poly * n + k];
  const bool negative = x > (qt >> 1);
  const u64 mag = negative ? qt - x : x;
  u64* __restrict__ o = spread + blockIdx.z * spread_stride + (size_t)poly * level * n;
  for (int i = 0; i < level; ++i) {
    const ModInfo m = mods[i];
    const u64 r = reduce64(mag, m);
    o[(size_t)i * n + k] = negative ? neg_mod(r, m.q) : r;
  }
}

// ---------------------------------------------------------------- elementwise
__global__ void __launch_bounds__(TPB) add_kernel(const u64* __restrict__ a, const u64* __restrict__ b,
                                                  u64* __restrict__ o, const ModInfo* __restrict__ mods, int log_n,
                                                  int period, int sub) {
  const int n = 1 << log_n;
  const size_t idx = (size_t)blockIdx.y * n + blockIdx.x * TPB + threadIdx.x;
  const u64 q = mods[blockIdx.y % period].q;
  o[idx] = sub ? sub_mod(a[idx], b[idx], q) : add_mod(a[idx], b[idx], q);
}

__global__ void __launch_bounds__(TPB) mul_rows_kernel(const u64* __restrict__ a, const u64* __restrict__ b,
                                                       u64* __restrict__ o, const ModInfo* __restrict__ mods,
                                                       int log_n, int period, int b_period) {
  const int n = 1 << log_n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int row = blockIdx.y;
  const ModInfo m = mods[row % period];
  o[(size_t)row * n + k] = mul_mod(a[(size_t)row * n + k], b[(size_t)(row % b_period) * n + k], m);
}

// Multiplication by X^(N/2): the value at exponent e = 2 brev(k) + 1 is
// multiplied by i_q^e = i_q (e = 1 mod 4, k < N/2) or -i_q (k >= N/2).
__global__ void __launch_bounds__(TPB) mul_i_kernel(const u64* __restrict__ a, u64* __restrict__ o,
                                                    const ModInfo* __restrict__ mods,
                                                    const PrimeConsts* __restrict__ pc, int log_n, int period) {
  const int n = 1 << log_n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int pr = blockIdx.y % period;
  const u64 q = mods[pr].q;
  const size_t idx = (size_t)blockIdx.y * n + k;
  u64 v = mul_shoup(a[idx], pc[pr].iq, pc[pr].iq_sh, q);
  o[idx] = k < (n >> 1) ? v : neg_mod(v, q);
}

__global__ void __launch_bounds__(TPB) galois_kernel(const u64* __restrict__ a, u64* __restrict__ o, int log_n,
                                                     u32 g) {
  const int n = 1 << log_n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const size_t row = (size_t)blockIdx.y * n;
  o[row + k] = a[row + galois_source((u32)k, g, log_n)];
}

// d0 = a0 b0, d1 = a0 b1 + a1 b0 (written to d01 = [2][l][N]), d2 = a1 b1.
__global__ void __launch_bounds__(TPB) tensor_kernel(const u64* __restrict__ a, const u64* __restrict__ b,
                                                     u64* __restrict__ d01, u64* __restrict__ d2,
                                                     const ModInfo* __restrict__ mods, int log_n, int level) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int i = blockIdx.y;
  const ModInfo m = mods[i];
  const size_t i0 = (size_t)i * n + k, i1 = (size_t)(l + i) * n + k;
  const u64 a0 = a[i0], a1 = a[i1], b0 = b[i0], b1 = b[i1];
  U128 cross = mul_wide(a0, b1);
  acc_wide(cross, mul_wide(a1, b0));
  d01[i0] = mul_mod(a0, b0, m);
  d01[i1] = reduce128(cross, m);
  d2[i0] = mul_mod(a1, b1, m);
}

// out[r][k] = coeffs[k] mod prime(r) for the rows of a row table.
__global__ void __launch_bounds__(TPB) reduce_signed_kernel(const i64* __restrict__ coeffs, size_t coeff_stride,
                                                            u64* __restrict__ out, size_t out_stride,
                                                            const int2* __restrict__ rows,
                                                            const ModInfo* __restrict__ mods, int log_n) {
  const int n = 1 << log_n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int2 rj = rows[blockIdx.y];
  const ModInfo m = mods[rj.y];
  const i64 v = coeffs[blockIdx.z * coeff_stride + k];
  const u64 mag = v < 0 ? (u64)(-v) : (u64)v;
  const u64 r = reduce64(mag, m);
  out[blockIdx.z * out_stride + (size_t)rj.x * n + k] = v < 0 ? neg_mod(r, m.q) : r;
}

// ct = (-a s + m + e, a), all in NTT form.
__global__ void __launch_bounds__(TPB) encrypt_kernel(const u64* __restrict__ a, const u64* __restrict__ e,
                                                      const u64* __restrict__ m, const u64* __restrict__ s,
                                                      u64* __restrict__ ct, const ModInfo* __restrict__ mods,
                                                      int log_n, int level) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int i = blockIdx.y;
  const ModInfo md = mods[i];
  const size_t idx = (size_t)i * n + k;
  const u64 av = a[idx];
  u64 v = neg_mod(mul_mod(av, s[idx], md), md.q);
  v = add_mod(v, m[idx], md.q);
  v = add_mod(v, e[idx], md.q);
  ct[idx] = v;
  ct[(size_t)(l + i) * n + k] = av;
}

__global__ void __launch_bounds__(TPB) decrypt_kernel(const u64* __restrict__ ct, const u64* __restrict__ s,
                                                      u64* __restrict__ m, const ModInfo* __restrict__ mods,
                                                      int log_n, int level) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int i = blockIdx.y;
  const ModInfo md = mods[i];
  const size_t idx = (size_t)i * n + k;
  m[idx] = add_mod(ct[idx], mul_mod(ct[(size_t)(l + i) * n + k], s[idx], md), md.q);
}

// key[j][0][t] = -a_j s + e_j + (t in digit j ? (P mod q_t) s' : 0); key[j][1][t] = a_j (NTT form).
__global__ void __launch_bounds__(TPB) keygen_kernel(const u64* __restrict__ a, const u64* __restrict__ e,
                                                     const u64* __restrict__ s, const u64* __restrict__ sp,
                                                     u64* __restrict__ key, const ModInfo* __restrict__ mods,
                                                     const PrimeConsts* __restrict__ pc, int log_n, int nprimes,
                                                     int num_q, int alpha) {
  const int n = 1 << log_n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int t = blockIdx.y;
  const int j = blockIdx.z;
  const ModInfo md = mods[t];
  const size_t in_idx = ((size_t)j * nprimes + t) * n + k;
  const size_t sk_idx = (size_t)t * n + k;
  const u64 av = a[in_idx];
  u64 v = neg_mod(mul_mod(av, s[sk_idx], md), md.q);
  v = add_mod(v, e[in_idx], md.q);
  if (t < num_q && t / alpha == j) v = add_mod(v, mul_shoup(sp[sk_idx], pc[t].pmod, pc[t].pmod_sh, md.q), md.q);
  key[((size_t)(2 * j) * nprimes + t) * n + k] = v;
  key[((size_t)(2 * j + 1) * nprimes + t) * n + k] = av;
}

}  // namespace

// ---------------------------------------------------------------- launchers

size_t key_switch_scratch_words(const Context& c, int level, int count) {
  const size_t n = c.n;
  const size_t l = level + 1, ext = l + c.num_p, beta = c.beta(level);
  // coefficient form of the inputs, extended digits, accumulators, ModDown conversion rows (as key_switch)
  return Pool::arena_round(count * l * n) + Pool::arena_round(count * beta * ext * n) +
         Pool::arena_round(count * 2 * ext * n) + Pool::arena_round(count * 2 * l * n);
}

void key_switch(Context& c, const KsJob& job) {
  const int level = job.level;
  const int l = level + 1;
  const int ext = l + c.num_p;
  const int beta = c.beta(level);
  const int m = job.count;
  if (m < 1 || m > MAX_BATCH) fail(HETAL_E_INVALID_ARG, "key switch batch size");
  const bool hoisted = job.in_stride == 0;
  const int m_in = hoisted ? 1 : m;
  const size_t n = c.n;
  const size_t poly = (size_t)l * n;
  const size_t dt_words = (size_t)beta * ext * n;
  const size_t acc_words = 2 * (size_t)ext * n;
  const size_t conv_words = 2 * poly;

  // The basis conversions run fused into the first pass of the NTT that follows them when the pass shape and
  // term count allow (the inverse NTT before each then applies the conversion's first factor).
  const bool fuse_up = c.alpha <= MAX_FUSED_CONV && (c.log_n == 12 || c.log_n == 16);
  const bool fuse_down = c.num_p <= MAX_FUSED_CONV && (c.log_n == 12 || c.log_n == 16);

  // 1. coefficient form of the input(s): the inverse NTT reads the input in place of a copy
  Tmp coef(c.pool, m_in * poly);
  RowsRef ct_rows = c.rows(ROWS_CT, level);
  NttSrc src;
  src.p = job.in;
  src.batch_stride = hoisted ? 0 : job.in_stride;
  ntt_inverse(c, coef, poly, m_in, RowsRef{ct_rows.d, l}, src,
              fuse_up ? c.d_modup_scale + (size_t)level * MAX_PRIMES : nullptr, fuse_up);

  // 2. ModUp of every digit, then the NTT of the converted rows
  Tmp dt(c.pool, m_in * dt_words);
  if (fuse_up) {
    NttConv cv;
    cv.kind = CONV_MODUP;
    cv.count = c.alpha;
    cv.y = coef.p;
    cv.y_stride = poly;
    cv.ext = ext;
    cv.num_q = c.num_q;
    cv.modup = c.d_modup + (size_t)level * c.dnum;
    ntt_forward(c, dt, dt_words, m_in, c.rows(ROWS_MODUP, level), NttSrc{}, nullptr, &cv);
  } else {
    c.begin_launch();
    switch (c.alpha) {
#define HETAL_MODUP(A)                                                                                          \
  case A:                                                                                                     \
    hipLaunchKernelGGL(modup_kernel<A>, grid_for(c, beta, m_in), dim3(TPB), 0, c.stream, coef.p, poly, dt.p, dt_words, \
                       c.d_modup + (size_t)level * c.dnum, c.d_mod, c.log_n, level, c.num_q, c.num_p);        \
    break;
      HETAL_MODUP(1) HETAL_MODUP(2) HETAL_MODUP(3) HETAL_MODUP(4) HETAL_MODUP(5) HETAL_MODUP(6) HETAL_MODUP(7)
      HETAL_MODUP(8)
#undef HETAL_MODUP
      default:
        fail(HETAL_E_PARAMS, "digit length above 8");
    }
    // reads: each digit's coefficient-form limbs (l rows in all); writes the beta * ext - l rows outside the digits
    c.end_launch(KC_MODUP, 8.0 * n * m_in * ((double)beta * ext));
    ntt_forward(c, dt, dt_words, m_in, c.rows(ROWS_MODUP, level));
  }

  // 3. inner product with the keys, automorphism applied on the loads
  Tmp acc(c.pool, m * acc_words);
  bool shared = !hoisted;
  for (int i = 1; i < m && shared; ++i) shared = job.item[i].key == job.item[0].key && job.item[i].g == job.item[0].g;
  if (beta < 1 || beta > 8) fail(HETAL_E_PARAMS, "more than 8 digits");
  if (shared) {
    c.begin_launch();
    switch (beta) {
#define HETAL_IPS(B)                                                                                              \
  case B:                                                                                                       \
    hipLaunchKernelGGL(inner_product_shared_kernel<B>, grid_for(c, ext, 1), dim3(TPB), 0, c.stream, dt.p, dt_words, \
                       job.in, job.in_stride, acc.p, acc_words, job.item[0].key, job.item[0].g, m, c.d_mod,     \
                       c.log_n, level, c.num_q, c.num_p, c.nprimes, c.alpha);                                   \
    break;
      HETAL_IPS(1) HETAL_IPS(2) HETAL_IPS(3) HETAL_IPS(4) HETAL_IPS(5) HETAL_IPS(6) HETAL_IPS(7) HETAL_IPS(8)
#undef HETAL_IPS
    }
    // reads: the extended digits of every item and 2 beta ext key rows once; writes 2 ext rows per item
    c.end_launch(KC_INNER, 8.0 * n * ((double)m * beta * ext + 2.0 * beta * ext + (double)m * 2.0 * ext));
  } else {
    IpArgs ip;
    for (int i = 0; i < MAX_BATCH; ++i) {
      ip.key[i] = i < m ? job.item[i].key : nullptr;
      ip.g[i] = i < m ? job.item[i].g : 1;
    }
    const size_t dts = hoisted ? (size_t)0 : dt_words, ins = hoisted ? (size_t)0 : job.in_stride;
    c.begin_launch();
    switch (beta) {
#define HETAL_IP(B)                                                                                             \
  case B:                                                                                                     \
    hipLaunchKernelGGL(inner_product_kernel<B>, grid_for(c, ext, m), dim3(TPB), 0, c.stream, dt.p, dts, job.in, ins, \
                       acc.p, acc_words, ip, c.d_mod, c.log_n, level, c.num_q, c.num_p, c.nprimes, c.alpha);   \
    break;
      HETAL_IP(1) HETAL_IP(2) HETAL_IP(3) HETAL_IP(4) HETAL_IP(5) HETAL_IP(6) HETAL_IP(7) HETAL_IP(8)
#undef HETAL_IP
    }
    // reads: the extended digits (once per input) and 2 beta ext key rows per item; writes 2 ext rows per item
    c.end_launch(KC_INNER, 8.0 * n * ((double)m_in * beta * ext + (double)m * (2.0 * beta * ext + 2.0 * ext)));
  }

  // 4. ModDown: special rows to coefficient form, centred conversion, NTT, combine
  ntt_inverse(c, acc, acc_words, m, c.rows(ROWS_SPECIAL, level), NttSrc{}, fuse_down ? c.d_moddown_scale : nullptr,
              fuse_down);
  Tmp conv(c.pool, m * conv_words);
  NttConv cv;
  if (fuse_down) {
    cv.kind = CONV_MODDOWN;
    cv.count = c.num_p;
    cv.y = acc.p;
    cv.y_stride = acc_words;
    cv.ext = ext;
    cv.l = l;
    cv.num_q = c.num_q;
    cv.moddown = c.d_moddown;
  } else {
    c.begin_launch();
    switch (c.num_p) {
#define HETAL_CONV(K)                                                                                          \
  case K:                                                                                                    \
    hipLaunchKernelGGL(moddown_conv_kernel<K>, grid_for(c, 2, m), dim3(TPB), 0, c.stream, acc.p, acc_words, conv.p, \
                       conv_words, c.d_moddown, c.d_mod, c.log_n, level, c.num_q);                           \
    break;
      HETAL_CONV(1) HETAL_CONV(2) HETAL_CONV(3) HETAL_CONV(4) HETAL_CONV(5) HETAL_CONV(6) HETAL_CONV(7) HETAL_CONV(8)
#undef HETAL_CONV
      default:
        fail(HETAL_E_PARAMS, "more than 8 special primes");
    }
    c.end_launch(KC_MODDOWN, 8.0 * n * m * (2.0 * c.num_p + 2.0 * l));
  }
  // ... and the combine (acc_Q - conv) P^-1 + addends as the epilogue of the NTT's last pass
  NttEpilogue epi;
  epi.a = acc.p;
  epi.a_stride = acc_words;
  epi.a_poly_rows = ext;
  epi.l = l;
  epi.cst = device_field<u64>(c.d_moddown, offsetof(ModDownTab, pinv));
  epi.cst_sh = device_field<u64>(c.d_moddown, offsetof(ModDownTab, pinv_sh));
  epi.out = job.out;
  epi.out_stride = job.out_stride;
  epi.add0 = job.add0;
  epi.add0_stride = job.add0_stride;
  epi.gather = job.add0_galois ? 1 : 0;
  epi.add1 = job.add1;
  epi.add1_stride = job.add1_stride;
  epi.addx = job.addx;
  epi.addx_stride = job.addx_stride;
  for (int i = 0; i < MAX_BATCH; ++i) epi.g[i] = i < m ? job.item[i].g : 1;
  ntt_forward(c, conv, conv_words, m, ct_rows, NttSrc{}, &epi, fuse_down ? &cv : nullptr);
  c.counters[5] += m;
  c.ks_items[level] += m;
  c.ks_key_reads[level] += shared ? 1 : m;
}

void k_add(Context& c, const u64* a, const u64* b, u64* out, int rows, int period) {
  c.begin_launch();
  hipLaunchKernelGGL(add_kernel, grid_for(c, rows, 1), dim3(TPB), 0, c.stream, a, b, out, c.d_mod, c.log_n, period, 0);
  c.end_launch(KC_ELEMWISE, 24.0 * c.n * rows);
}

void k_sub(Context& c, const u64* a, const u64* b, u64* out, int rows, int period) {
  c.begin_launch();
  hipLaunchKernelGGL(add_kernel, grid_for(c, rows, 1), dim3(TPB), 0, c.stream, a, b, out, c.d_mod, c.log_n, period, 1);
  c.end_launch(KC_ELEMWISE, 24.0 * c.n * rows);
}

void k_mul_rows(Context& c, const u64* a, const u64* b, u64* out, int rows, int period, int b_period) {
  c.begin_launch();
  hipLaunchKernelGGL(mul_rows_kernel, grid_for(c, rows, 1), dim3(TPB), 0, c.stream, a, b, out, c.d_mod, c.log_n,
                     period, b_period);
  c.end_launch(KC_ELEMWISE, 24.0 * c.n * rows);
}

void k_mul_i(Context& c, const u64* a, u64* out, int rows, int period) {
  c.begin_launch();
  hipLaunchKernelGGL(mul_i_kernel, grid_for(c, rows, 1), dim3(TPB), 0, c.stream, a, out, c.d_mod, c.d_pc, c.log_n,
                     period);
  c.end_launch(KC_ELEMWISE, 16.0 * c.n * rows);
}

void k_galois(Context& c, const u64* a, u64* out, int rows, int period, u32 g) {
  (void)period;
  c.begin_launch();
  hipLaunchKernelGGL(galois_kernel, grid_for(c, rows, 1), dim3(TPB), 0, c.stream, a, out, c.log_n, g);
  c.end_launch(KC_ELEMWISE, 16.0 * c.n * rows);
}

void k_tensor(Context& c, const u64* a, const u64* b, u64* d01, u64* d2, int level) {
  c.begin_launch();
  hipLaunchKernelGGL(tensor_kernel, grid_for(c, level + 1, 1), dim3(TPB), 0, c.stream, a, b, d01, d2, c.d_mod, c.log_n,
                     level);
  c.end_launch(KC_ELEMWISE, 8.0 * c.n * (level + 1) * 7);
}

void k_rescale(Context& c, const u64* in, u64* out, int level, int batch, size_t in_stride, size_t out_stride) {
  const size_t n = c.n;
  // groups of at most MAX_BATCH items (the NTT epilogue's per-launch limit)
  for (int first = 0; first < batch; first += MAX_BATCH) {
    const int m = std::min(MAX_BATCH, batch - first);
    const u64* in_m = in + (size_t)first * in_stride;
    u64* out_m = out + (size_t)first * out_stride;
    Tmp top(c.pool, (size_t)m * 2 * n);
    NttSrc src;
    src.p = in_m;
    src.batch_stride = in_stride;
    src.row_mul = level + 1;  // top row of poly p: p (level + 1) + level
    src.row_add = level;
    ntt_inverse(c, top, 2 * n, m, c.rows(ROWS_TOP, level), src);
    Tmp spread(c.pool, (size_t)m * 2 * level * n);
    c.begin_launch();
    hipLaunchKernelGGL(rescale_spread_kernel, grid_for(c, 2, m), dim3(TPB), 0, c.stream, top.p, 2 * n, spread.p,
                       2 * (size_t)level * n, c.d_mod, c.log_n, level);
    c.end_launch(KC_RESCALE, 8.0 * n * m * (2.0 + 2.0 * level));
    // out = (in - spread) q_level^-1, as the epilogue of the spread rows' NTT
    NttEpilogue epi;
    epi.a = in_m;
    epi.a_stride = in_stride;
    epi.a_poly_rows = level + 1;
    epi.l = level;
    epi.cst = device_field<u64>(c.d_rescale + level, offsetof(RescaleTab, inv));
    epi.cst_sh = device_field<u64>(c.d_rescale + level, offsetof(RescaleTab, inv_sh));
    epi.out = out_m;
    epi.out_stride = out_stride;
    for (int i = 0; i < MAX_BATCH; ++i) epi.g[i] = 1;
    ntt_forward(c, spread, 2 * (size_t)level * n, m, c.rows(ROWS_CT, level - 1), NttSrc{}, &epi);
  }
  c.counters[4] += batch;
}

void k_reduce_signed(Context& c, const i64* coeffs, u64* out, RowsRef rows, int batch, size_t coeff_stride,
                     size_t out_stride) {
  c.begin_launch();
  hipLaunchKernelGGL(reduce_signed_kernel, grid_for(c, rows.count, batch), dim3(TPB), 0, c.stream, coeffs,
                     coeff_stride, out, out_stride, rows.d, c.d_mod, c.log_n);
  c.end_launch(KC_ELEMWISE, 8.0 * c.n * (double)rows.count * batch);
}

void k_encrypt(Context& c, const u64* a_ntt, const u64* e_ntt, const u64* m, const u64* s, u64* ct, int level) {
  c.begin_launch();
  hipLaunchKernelGGL(encrypt_kernel, grid_for(c, level + 1, 1), dim3(TPB), 0, c.stream, a_ntt, e_ntt, m, s, ct, c.d_mod,
                     c.log_n, level);
  c.end_launch(KC_ELEMWISE, 40.0 * c.n * (level + 1));
}

void k_decrypt(Context& c, const u64* ct, const u64* s, u64* m, int level) {
  c.begin_launch();
  hipLaunchKernelGGL(decrypt_kernel, grid_for(c, level + 1, 1), dim3(TPB), 0, c.stream, ct, s, m, c.d_mod, c.log_n,
                     level);
  c.end_launch(KC_ELEMWISE, 32.0 * c.n * (level + 1));
}

void k_keygen(Context& c, const u64* a_ntt, const u64* e_ntt, const u64* s, const u64* sp, u64* key) {
  c.begin_launch();
  hipLaunchKernelGGL(keygen_kernel, grid_for(c, c.nprimes, c.dnum), dim3(TPB), 0, c.stream, a_ntt, e_ntt, s, sp, key,
                     c.d_mod, c.d_pc, c.log_n, c.nprimes, c.num_q, c.alpha);
  c.end_launch(KC_ELEMWISE, 48.0 * c.n * c.nprimes * c.dnum);
}

}  // namespace hetal
