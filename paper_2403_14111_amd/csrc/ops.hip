// CKKS operations (Sec. 2.2 of the paper) as compositions of the RNS kernels.
#include <cstring>

#include "ops.hpp"

namespace hetal {

namespace {

void check_pair(CtView a, CtView b) {
  if (a.level != b.level) fail(HETAL_E_LEVEL, "operands at different levels");
  if (std::abs(a.scale - b.scale) > 1e-9 * std::max(std::abs(a.scale), std::abs(b.scale)))
    fail(HETAL_E_SCALE, "operands with different scales");
}

// Slot values of a mask block: re/im [s0 * s1] (row-major).
__global__ void mask_kernel(double* __restrict__ re, double* __restrict__ im, int kind, int k, int cc, int s0, int s1,
                            double t) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= s0 * s1) return;
  const int i = idx / s1, j = idx % s1;
  double vr = 0.0, vi = 0.0;
  if (kind == MASK_OFFDIAG_CPLX) {
    // t/2 M^(k, c) - i t/2 M^(k + c/2, c), M^(k, c)_{ij} = [j = i + k (mod c)]
    const int d = ((j - i - k) % cc + cc) % cc;
    if (d == 0) vr = 0.5 * t;
    if (d == cc / 2) vi = -0.5 * t;
  } else if (kind == MASK_FIRST_COL) {
    vr = j == 0 ? 1.0 : 0.0;
  } else if (kind == MASK_LEFT_COLS) {
    vr = j < s1 - k ? 1.0 : 0.0;
  } else if (kind == MASK_PAD_COLS) {
    vr = j % cc >= k ? t : 0.0;
  } else {
    vr = j >= k ? t : 0.0;
  }
  re[idx] = vr;
  im[idx] = vi;
}

}  // namespace

u32 galois_rot(const Context& c, int r) {
  const long half = c.slots;
  long e = ((long)r % half + half) % half;
  const u64 m = 2ull * c.n;
  u64 g = 1, b = 5;
  for (; e; e >>= 1) {
    if (e & 1) g = g * b % m;
    b = b * b % m;
  }
  return (u32)g;
}

u32 galois_conj(const Context& c) { return (u32)(2 * c.n - 1); }

void encode_slots(Context& c, const double* d_re, const double* d_im, int count, size_t slot_stride, int level,
                  double scale, u64* out, size_t out_stride) {
  Tmp status(c.pool, 1);
  HCHECK(hipMemsetAsync(status.p, 0, sizeof(u64), c.stream));
  k_encode(c, d_re, d_im, count, slot_stride, level, scale, out, out_stride, reinterpret_cast<int*>(status.p));
  u64 h = 0;
  HCHECK(hipMemcpyAsync(&h, status.p, sizeof(u64), hipMemcpyDeviceToHost, c.stream));
  HCHECK(hipStreamSynchronize(c.stream));
  if (h) fail(HETAL_E_OVERFLOW, "an encoded coefficient does not fit in 62 bits");
}

void op_add(Context& c, CtView a, CtView b, u64* out, double* scale_out, bool subtract) {
  check_pair(a, b);
  const int l = a.level + 1;
  if (subtract) k_sub(c, a.d, b.d, out, 2 * l, l);
  else k_add(c, a.d, b.d, out, 2 * l, l);
  *scale_out = a.scale;
}

void op_mul_i(Context& c, CtView a, u64* out) { k_mul_i(c, a.d, out, 2 * (a.level + 1), a.level + 1); }

void op_mod_drop(Context& c, CtView a, int level, u64* out) {
  if (level > a.level || level < 0) fail(HETAL_E_LEVEL, "mod_drop target level out of range");
  const size_t rows = (size_t)(level + 1) * c.n;
  if (out == a.d && level == a.level) return;
  if (out == a.d) {
    // c0 stays in place; c1 moves down through a temporary (the two ranges can overlap)
    Tmp t(c.pool, rows);
    HCHECK(hipMemcpyAsync(t.p, a.d + c.poly_words(a.level), rows * 8, hipMemcpyDeviceToDevice, c.stream));
    HCHECK(hipMemcpyAsync(out + rows, t.p, rows * 8, hipMemcpyDeviceToDevice, c.stream));
    return;
  }
  HCHECK(hipMemcpyAsync(out, a.d, rows * 8, hipMemcpyDeviceToDevice, c.stream));
  HCHECK(hipMemcpyAsync(out + rows, a.d + c.poly_words(a.level), rows * 8, hipMemcpyDeviceToDevice, c.stream));
}

void op_rescale(Context& c, CtView a, u64* out) {
  if (a.level < 1) fail(HETAL_E_LEVEL, "no level left to rescale");
  if (out == a.d) {
    Tmp t(c.pool, c.ct_words(a.level - 1));
    k_rescale(c, a.d, t.p, a.level, 1, 0, 0);
    HCHECK(hipMemcpyAsync(out, t.p, c.ct_words(a.level - 1) * 8, hipMemcpyDeviceToDevice, c.stream));
    return;
  }
  k_rescale(c, a.d, out, a.level, 1, 0, 0);
}

void op_cmult(Context& c, CtView a, const u64* pt, u64* out) {
  const int l = a.level + 1;
  k_mul_rows(c, a.d, pt, out, 2 * l, l, l);
  c.counters[3] += 1;
}

void op_hmult(Context& c, const KeySet& k, CtView a, CtView b, u64* out) {
  if (a.level != b.level) fail(HETAL_E_LEVEL, "operands at different levels");
  if (!k.relin) fail(HETAL_E_NO_KEY, "relinearisation key missing");
  const int l = a.level + 1;
  Tmp d01(c.pool, c.ct_words(a.level));
  Tmp d2(c.pool, c.poly_words(a.level));
  k_tensor(c, a.d, b.d, d01, d2, a.level);
  KsJob job;
  job.level = a.level;
  job.count = 1;
  job.in = d2;
  job.in_stride = c.poly_words(a.level);
  job.item[0] = KsItem{k.relin, 1};
  job.out = out;
  job.out_stride = c.ct_words(a.level);
  job.add0 = d01;
  job.add1 = d01.p + (size_t)l * c.n;
  key_switch(c, job);
  c.counters[2] += 1;
}

void op_galois(Context& c, const KeySet& k, CtView a, u32 g, u64* out) {
  if (g == 1) {  // rotation by a multiple of N/2 slots: the identity
    if (out != a.d)
      HCHECK(hipMemcpyAsync(out, a.d, c.ct_words(a.level) * 8, hipMemcpyDeviceToDevice, c.stream));
    return;
  }
  const u64* key = k.get(g);
  if (!key) fail(HETAL_E_NO_KEY, "no key for Galois element " + std::to_string(g));
  if (out == a.d) {
    Tmp t(c.pool, c.ct_words(a.level));
    op_galois(c, k, a, g, t.p);
    HCHECK(hipMemcpyAsync(out, t.p, c.ct_words(a.level) * 8, hipMemcpyDeviceToDevice, c.stream));
    return;
  }
  KsJob job;
  job.level = a.level;
  job.count = 1;
  job.in = a.d + c.poly_words(a.level);
  job.in_stride = c.poly_words(a.level);
  job.item[0] = KsItem{key, g};
  job.out = out;
  job.out_stride = c.ct_words(a.level);
  job.add0 = a.d;
  job.add0_galois = true;
  key_switch(c, job);
}

Cipher add(Context& c, CtView a, CtView b) {
  Cipher o(c, a.level);
  op_add(c, a, b, o.d, &o.scale, false);
  return o;
}

Cipher sub(Context& c, CtView a, CtView b) {
  Cipher o(c, a.level);
  op_add(c, a, b, o.d, &o.scale, true);
  return o;
}

Cipher mul_i(Context& c, CtView a) {
  Cipher o(c, a.level);
  op_mul_i(c, a, o.d);
  o.scale = a.scale;
  return o;
}

Cipher mod_drop(Context& c, CtView a, int level) {
  Cipher o(c, level);
  op_mod_drop(c, a, level, o.d);
  o.scale = a.scale;
  return o;
}

Cipher rescale(Context& c, CtView a) {
  if (a.level < 1) fail(HETAL_E_LEVEL, "no level left to rescale");
  Cipher o(c, a.level - 1);
  op_rescale(c, a, o.d);
  o.scale = a.scale / (double)c.primes[a.level];
  return o;
}

Cipher hmult(Context& c, const KeySet& k, CtView a, CtView b) {
  Cipher o(c, a.level);
  op_hmult(c, k, a, b, o.d);
  o.scale = a.scale * b.scale;
  return o;
}

Cipher rotate(Context& c, const KeySet& k, CtView a, int r) {
  Cipher o(c, a.level);
  op_galois(c, k, a, galois_rot(c, r), o.d);
  o.scale = a.scale;
  c.counters[0] += 1;
  return o;
}

Cipher conjugate(Context& c, const KeySet& k, CtView a) {
  Cipher o(c, a.level);
  op_galois(c, k, a, galois_conj(c), o.d);
  o.scale = a.scale;
  c.counters[1] += 1;
  return o;
}

MaskCache::~MaskCache() {
  if (!c) return;
  for (auto& kv : pts) c->pool.put(kv.second);
}

const u64* mask_pt(Context& c, MaskCache& cache, MaskKind kind, int k, int cc, int s0, int s1, double t, int level) {
  auto key = std::make_tuple((int)kind, k, cc, s0, s1, t, level);
  auto it = cache.pts.find(key);
  if (it != cache.pts.end()) return it->second;
  cache.c = &c;
  const int s = s0 * s1;
  Tmp vals(c.pool, 2 * (size_t)s);
  double* re = reinterpret_cast<double*>(vals.p);
  double* im = re + s;
  c.begin_launch();
  hipLaunchKernelGGL(mask_kernel, dim3((s + 255) / 256), dim3(256), 0, c.stream, re, im, (int)kind, k, cc, s0, s1, t);
  c.end_launch(KC_ENCODE, 0.0);
  u64* pt = c.pool.get(c.poly_words(level));
  encode_slots(c, re, im, 1, 0, level, (double)c.primes[level], pt, 0);
  cache.pts[key] = pt;
  return pt;
}

void mask_slots(Context& c, MaskKind kind, int k, int cc, int s0, int s1, double t, double* d_re, double* d_im) {
  const int s = s0 * s1;
  c.begin_launch();
  hipLaunchKernelGGL(mask_kernel, dim3((s + 255) / 256), dim3(256), 0, c.stream, d_re, d_im, (int)kind, k, cc, s0, s1, t);
  c.end_launch(KC_ENCODE, 0.0);
}

Cipher cmult_mask(Context& c, MaskCache& cache, CtView a, MaskKind kind, int k, int cc, int s0, int s1, double t) {
  const u64* pt = mask_pt(c, cache, kind, k, cc, s0, s1, t, a.level);
  Cipher o(c, a.level);
  op_cmult(c, a, pt, o.d);
  o.scale = a.scale * (double)c.primes[a.level];
  return o;
}

}  // namespace hetal
