// RNS kernels for gfx950: elementwise operations, encryption and key generation.
// (The key switch lives in keyswitch.hip.)
//
// The kernels stream limbs through HBM once; each thread handles one
// coefficient index, so consecutive lanes touch consecutive words of a limb.
#include "hetal_internal.hpp"

namespace hetal {

namespace {

constexpr int TPB = 256;

inline dim3 grid_for(const Context& c, int y, int z) { return dim3((unsigned)(c.n / TPB), (unsigned)y, (unsigned)z); }

// ---------------------------------------------------------------- elementwise
__global__ void __launch_bounds__(TPB) add_kernel(const u64* __restrict__ a, const u64* __restrict__ b,
                                                  u64* __restrict__ o, const ModInfo* __restrict__ mods, int log_n,
                                                  int period, int sub) {
  const int n = 1 << log_n;
  const size_t idx = (size_t)blockIdx.y * n + blockIdx.x * TPB + threadIdx.x;
  const u64 q = mods[blockIdx.y % period].q;
  o[idx] = sub ? sub_mod(a[idx], b[idx], q) : add_mod(a[idx], b[idx], q);
}

// Row r of item z of the output (polynomial r / l, limb r % l) from the operands' rows of the same polynomial and
// limb, each operand with its own rows per polynomial and item stride.
__global__ void __launch_bounds__(TPB) addsub_rows_kernel(const u64* __restrict__ a, size_t a_stride, int a_rows,
                                                          const u64* __restrict__ b, size_t b_stride, int b_rows,
                                                          u64* __restrict__ o, const ModInfo* __restrict__ mods,
                                                          int log_n, int l, int sub) {
  const int n = 1 << log_n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int r = blockIdx.y, z = blockIdx.z;
  const int p = r / l, i = r - p * l;
  const u64 q = mods[i].q;
  const u64 x = a[(size_t)z * a_stride + (size_t)(p * a_rows + i) * n + k];
  const u64 y = b[(size_t)z * b_stride + (size_t)(p * b_rows + i) * n + k];
  o[((size_t)z * 2 * l + r) * n + k] = sub ? sub_mod(x, y, q) : add_mod(x, y, q);
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

// key[j][0][t] = -a_j s + e_j + (t in digit j ? (P mod q_t) s' : 0); key[j][1][t] = a_j (NTT form), stored for the
// key switch (keyswitch.hip): permuted by tau_g^-1 (the word of position k goes to position galois_source(k, g)),
// in key_slot order within each chunk, as the bit patterns of the (exact) doubles.
__global__ void __launch_bounds__(TPB) keygen_kernel(const u64* __restrict__ a, const u64* __restrict__ e,
                                                     const u64* __restrict__ s, const u64* __restrict__ sp,
                                                     u64* __restrict__ key, const ModInfo* __restrict__ mods,
                                                     const PrimeConsts* __restrict__ pc, int log_n, int nprimes,
                                                     int num_q, int alpha, u32 g) {
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
  const u32 slot = key_slot(g == 1 ? (u32)k : galois_source((u32)k, g, log_n));
  key[((size_t)(2 * j) * nprimes + t) * n + slot] = (u64)__double_as_longlong((double)v);
  key[((size_t)(2 * j + 1) * nprimes + t) * n + slot] = (u64)__double_as_longlong((double)av);
}

}  // namespace

// ---------------------------------------------------------------- launchers

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

void k_addsub_rows(Context& c, const u64* a, size_t a_stride, int a_rows, const u64* b, size_t b_stride, int b_rows,
                   u64* out, int level, int count, bool subtract) {
  const int l = level + 1;
  if (a_rows < l || b_rows < l || count < 1) fail(HETAL_E_INVALID_ARG, "addsub operand shape");
  c.begin_launch();
  hipLaunchKernelGGL(addsub_rows_kernel, grid_for(c, 2 * l, count), dim3(TPB), 0, c.stream, a, a_stride, a_rows, b,
                     b_stride, b_rows, out, c.d_mod, c.log_n, l, subtract ? 1 : 0);
  c.end_launch(KC_ELEMWISE, 24.0 * c.n * 2 * l * count);
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

void k_keygen(Context& c, const u64* a_ntt, const u64* e_ntt, const u64* s, const u64* sp, u64* key, u32 g) {
  c.begin_launch();
  hipLaunchKernelGGL(keygen_kernel, grid_for(c, c.nprimes, c.dnum), dim3(TPB), 0, c.stream, a_ntt, e_ntt, s, sp, key,
                     c.d_mod, c.d_pc, c.log_n, c.nprimes, c.num_q, c.alpha, g);
  c.end_launch(KC_ELEMWISE, 48.0 * c.n * c.nprimes * c.dnum);
}

}  // namespace hetal
