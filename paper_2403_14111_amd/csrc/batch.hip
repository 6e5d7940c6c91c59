// Batched CKKS operations: many ciphertexts at one level per launch, so that
// every launch spans enough limbs to fill the 256 CUs, and ciphertexts that
// share a key share its HBM reads.  Each item goes through exactly the same
// key switches and rescales as it would alone, so results are bit-identical
// to the one-at-a-time operations.
#include <algorithm>

#include "ops.hpp"

namespace hetal {

namespace {

constexpr int TPB = 256;

struct PtrArgs {
  const u64* a[MAX_BATCH];
  const u64* b[MAX_BATCH];
  int ra[MAX_BATCH];  // rows per polynomial of each operand (its level + 1); an operand above the product's level
  int rb[MAX_BATCH];  // is read as its mod-drop would be: the first level + 1 rows of each polynomial
};

// d01[item] = (a0 b0, a0 b1 + a1 b0), d2[item] = a1 b1.
__global__ void __launch_bounds__(TPB) tensor_batch_kernel(PtrArgs p, u64* __restrict__ d01, u64* __restrict__ d2,
                                                           const ModInfo* __restrict__ mods, int log_n, int level) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int i = blockIdx.y;
  const int item = blockIdx.z;
  const ModInfo m = mods[i];
  const u64* __restrict__ a = p.a[item];
  const u64* __restrict__ b = p.b[item];
  const size_t i0 = (size_t)i * n + k, i1 = (size_t)(l + i) * n + k;
  const u64 a0 = a[i0], a1 = a[(size_t)(p.ra[item] + i) * n + k], b0 = b[i0], b1 = b[(size_t)(p.rb[item] + i) * n + k];
  U128 cross = mul_wide(a0, b1);
  acc_wide(cross, mul_wide(a1, b0));
  u64* __restrict__ o = d01 + (size_t)item * 2 * l * n;
  o[i0] = mul_mod(a0, b0, m);
  o[i1] = reduce128(cross, m);
  d2[(size_t)item * l * n + i0] = mul_mod(a1, b1, m);
}

// Segment g of a launch is items [start[g], start[g+1]) of the input (start[0] = 0 relative to the launch's
// first item); its sum goes to item dst[g] of the output.
constexpr int MAX_SEGMENTS = 64;
struct SegArgs {
  int start[MAX_SEGMENTS + 1];
  int dst[MAX_SEGMENTS];
};

// out[dst[g]][row] = sum over the items t of segment g of a[t][row].
__global__ void __launch_bounds__(TPB) sum_segments_kernel(const u64* __restrict__ a, size_t a_stride, SegArgs sg,
                                                           u64* __restrict__ out, const ModInfo* __restrict__ mods,
                                                           int log_n, int level) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int row = blockIdx.y;
  const int g = blockIdx.z;
  const u64 q = mods[row % l].q;
  const int t0 = sg.start[g], t1 = sg.start[g + 1];
  const u64* __restrict__ src = a + (size_t)t0 * a_stride + (size_t)row * n + k;
  u64 s = 0;
  for (int t = 0; t < t1 - t0; ++t) s = add_mod(s, src[(size_t)t * a_stride], q);
  out[(size_t)sg.dst[g] * 2 * l * n + (size_t)row * n + k] = s;
}

dim3 grid3(const Context& c, int y, int z) { return dim3((unsigned)(c.n / TPB), (unsigned)y, (unsigned)z); }

void check_same(BView a, BView b) {
  if (a.level != b.level || a.count != b.count) fail(HETAL_E_LEVEL, "batch operands differ in level or count");
  if (std::abs(a.scale - b.scale) > 1e-9 * std::max(std::abs(a.scale), std::abs(b.scale)))
    fail(HETAL_E_SCALE, "batch operands with different scales");
}

bool packed(const Context& c, BView a) { return a.stride == c.ct_words(a.level); }

Batch to_packed(Context& c, BView a) {
  Batch o(c, a.level, a.count);
  const size_t w = c.ct_words(a.level);
  if (a.stride >= w) {
    HCHECK(hipMemcpy2DAsync(o.d, w * 8, a.d, a.stride * 8, w * 8, a.count, hipMemcpyDeviceToDevice, c.stream));
  } else {  // broadcast (stride 0): one ciphertext repeated
    for (int i = 0; i < a.count; ++i)
      HCHECK(hipMemcpyAsync(o.d + (size_t)i * w, a.d + (size_t)i * a.stride, w * 8, hipMemcpyDeviceToDevice,
                            c.stream));
  }
  o.scale = a.scale;
  return o;
}

}  // namespace

Batch b_pack(Context& c, const std::vector<CtView>& items) {
  if (items.empty()) fail(HETAL_E_INVALID_ARG, "empty batch");
  Batch o(c, items[0].level, (int)items.size());
  const size_t w = c.ct_words(o.level);
  for (size_t i = 0; i < items.size(); ++i) {
    if (items[i].level != o.level) fail(HETAL_E_LEVEL, "batch items at different levels");
    HCHECK(hipMemcpyAsync(o.d + i * w, items[i].d, w * 8, hipMemcpyDeviceToDevice, c.stream));
  }
  o.scale = items[0].scale;
  return o;
}

static Batch b_addsub(Context& c, BView a, BView b, bool subtract) {
  check_same(a, b);
  Batch pa, pb;
  if (!packed(c, a)) {
    pa = to_packed(c, a);
    a = pa.v();
  }
  if (!packed(c, b)) {
    pb = to_packed(c, b);
    b = pb.v();
  }
  Batch o(c, a.level, a.count);
  const int l = a.level + 1;
  if (subtract) k_sub(c, a.d, b.d, o.d, 2 * l * a.count, l);
  else k_add(c, a.d, b.d, o.d, 2 * l * a.count, l);
  o.scale = a.scale;
  return o;
}

Batch b_add(Context& c, BView a, BView b) { return b_addsub(c, a, b, false); }
Batch b_sub(Context& c, BView a, BView b) { return b_addsub(c, a, b, true); }

Batch b_addsub_at(Context& c, BView a, BView b, int level, bool subtract) {
  if (a.count != b.count) fail(HETAL_E_LEVEL, "batch operands differ in count");
  if (a.level < level || b.level < level || level < 0) fail(HETAL_E_LEVEL, "operand below the sum's level");
  if (std::abs(a.scale - b.scale) > 1e-9 * std::max(std::abs(a.scale), std::abs(b.scale)))
    fail(HETAL_E_SCALE, "batch operands with different scales");
  Batch o(c, level, a.count);
  k_addsub_rows(c, a.d, a.stride, a.level + 1, b.d, b.stride, b.level + 1, o.d, level, a.count, subtract);
  o.scale = a.scale;
  return o;
}

Batch b_mul_i(Context& c, BView a) {
  Batch pa;
  if (!packed(c, a)) {
    pa = to_packed(c, a);
    a = pa.v();
  }
  Batch o(c, a.level, a.count);
  const int l = a.level + 1;
  k_mul_i(c, a.d, o.d, 2 * l * a.count, l);
  o.scale = a.scale;
  return o;
}

Batch b_mod_drop(Context& c, BView a, int level) {
  if (level > a.level || level < 0) fail(HETAL_E_LEVEL, "mod_drop target level out of range");
  Batch o(c, level, a.count);
  const size_t rows = c.poly_words(level), src_poly = c.poly_words(a.level);
  // 2 count blocks of `rows` words: block (i, p) starts at i * stride + p * src_poly
  if (a.stride == 2 * src_poly) {
    HCHECK(hipMemcpy2DAsync(o.d, rows * 8, a.d, src_poly * 8, rows * 8, 2 * (size_t)a.count, hipMemcpyDeviceToDevice,
                            c.stream));
  } else if (a.stride < 2 * src_poly) {  // broadcast view
    for (int i = 0; i < a.count; ++i)
      for (int p = 0; p < 2; ++p)
        HCHECK(hipMemcpyAsync(o.d + ((size_t)i * 2 + p) * rows, a.d + (size_t)i * a.stride + p * src_poly, rows * 8,
                              hipMemcpyDeviceToDevice, c.stream));
  } else {
    for (int p = 0; p < 2; ++p)
      HCHECK(hipMemcpy2DAsync(o.d + p * rows, 2 * rows * 8, a.d + p * src_poly, a.stride * 8, rows * 8, a.count,
                              hipMemcpyDeviceToDevice, c.stream));
  }
  o.scale = a.scale;
  return o;
}

Batch b_rescale(Context& c, BView a) {
  if (a.level < 1) fail(HETAL_E_LEVEL, "no level left to rescale");
  Batch o(c, a.level - 1, a.count);
  k_rescale(c, a.d, o.d, a.level, a.count, a.stride, c.ct_words(a.level - 1));
  o.scale = a.scale / (double)c.primes[a.level];
  return o;
}

static void run_rotations(Context& c, const KeySet& k, const u64* in0, size_t in_stride, int count, bool hoisted,
                          const std::vector<u32>& gal, int level, u64* out, const u64* addx = nullptr,
                          size_t addx_stride = 0, size_t out_stride = 0) {
  const size_t poly = c.poly_words(level);
  const size_t w = out_stride ? out_stride : c.ct_words(level);
  const int group = std::max(1, std::min(MAX_BATCH, c.tune.ks_group));
  for (int first = 0; first < count; first += group) {
    const int m = std::min(group, count - first);
    KsJob job;
    job.level = level;
    job.count = m;
    job.in = (hoisted ? in0 : in0 + (size_t)first * in_stride) + poly;
    job.in_stride = hoisted ? 0 : in_stride;
    for (int i = 0; i < m; ++i) {
      const u32 g = gal[first + i];
      const u64* key = k.get(g);
      if (!key) fail(HETAL_E_NO_KEY, "no key for Galois element " + std::to_string(g));
      job.item[i] = KsItem{key, g};
    }
    job.out = out + (size_t)first * w;
    job.out_stride = w;
    job.add0 = hoisted ? in0 : in0 + (size_t)first * in_stride;
    job.add0_stride = hoisted ? 0 : in_stride;
    job.add0_galois = true;
    if (addx) {
      job.addx = addx + (size_t)first * addx_stride;
      job.addx_stride = addx_stride;
    }
    key_switch(c, job);
  }
}

Batch b_rotate(Context& c, const KeySet& k, BView a, const std::vector<int>& steps) {
  if (steps.size() != 1 && (int)steps.size() != a.count) fail(HETAL_E_INVALID_ARG, "one step or one per item");
  std::vector<u32> gal(a.count);
  for (int i = 0; i < a.count; ++i) gal[i] = galois_rot(c, steps.size() == 1 ? steps[0] : steps[i]);
  for (u32 g : gal)
    if (g == 1) fail(HETAL_E_INVALID_ARG, "identity rotation inside a batch");
  Batch o(c, a.level, a.count);
  run_rotations(c, k, a.d, a.stride, a.count, false, gal, a.level, o.d);
  o.scale = a.scale;
  c.counters[0] += a.count;
  return o;
}

void b_rotate_into(Context& c, const KeySet& k, BView a, const std::vector<u32>& gal, u64* out, size_t out_stride) {
  if ((int)gal.size() != a.count) fail(HETAL_E_INVALID_ARG, "one Galois element per item");
  for (u32 g : gal)
    if (g == 1) fail(HETAL_E_INVALID_ARG, "identity rotation inside a batch");
  if (out_stride < c.ct_words(a.level)) fail(HETAL_E_INVALID_ARG, "output stride below one ciphertext");
  run_rotations(c, k, a.d, a.stride, a.count, false, gal, a.level, out, nullptr, 0, out_stride);
  c.counters[0] += a.count;
}

Batch b_rotate_add(Context& c, const KeySet& k, BView a, int step, const BView* addend) {
  const u32 g = galois_rot(c, step);
  if (g == 1) fail(HETAL_E_INVALID_ARG, "identity rotation inside a batch");
  BView x = addend ? *addend : a;
  if (x.level != a.level || x.count != a.count) fail(HETAL_E_LEVEL, "addend batch differs in level or count");
  if (std::abs(x.scale - a.scale) > 1e-9 * std::abs(a.scale)) fail(HETAL_E_SCALE, "addend with a different scale");
  Batch o(c, a.level, a.count);
  run_rotations(c, k, a.d, a.stride, a.count, false, std::vector<u32>(a.count, g), a.level, o.d, x.d, x.stride);
  o.scale = a.scale;
  c.counters[0] += a.count;
  return o;
}

Batch b_conj_add(Context& c, const KeySet& k, BView a) {
  Batch o(c, a.level, a.count);
  run_rotations(c, k, a.d, a.stride, a.count, false, std::vector<u32>(a.count, galois_conj(c)), a.level, o.d, a.d,
                a.stride);
  o.scale = a.scale;
  c.counters[1] += a.count;
  return o;
}

Batch b_rotate_hoisted(Context& c, const KeySet& k, CtView a, const std::vector<int>& steps) {
  const int count = (int)steps.size();
  std::vector<u32> gal(count);
  for (int i = 0; i < count; ++i) {
    gal[i] = galois_rot(c, steps[i]);
    if (gal[i] == 1) fail(HETAL_E_INVALID_ARG, "identity rotation inside a batch");
  }
  Batch o(c, a.level, count);
  run_rotations(c, k, a.d, 0, count, true, gal, a.level, o.d);
  o.scale = a.scale;
  c.counters[0] += count;
  return o;
}

Batch b_conj(Context& c, const KeySet& k, BView a) {
  std::vector<u32> gal(a.count, galois_conj(c));
  Batch o(c, a.level, a.count);
  run_rotations(c, k, a.d, a.stride, a.count, false, gal, a.level, o.d);
  o.scale = a.scale;
  c.counters[1] += a.count;
  return o;
}

// The key switch of one launch group of Mults (items first .. first + m - 1) into out.  Groups of at least
// FUSED_TENSOR_ITEMS compute the tensor product where the key switch reads it (one launch and three limb rows per
// item fewer); smaller ones, whose launches are latency-bound, store it first with its own kernel, which is faster
// there.  The words are the same either way.
constexpr int FUSED_TENSOR_ITEMS = 8;

static void hmult_group(Context& c, const KeySet& k, const std::vector<CtView>& a, const std::vector<CtView>& b,
                        int first, int m, int level, u64* out, size_t out_stride, u64* top_out) {
  const int l = level + 1;
  const size_t poly = c.poly_words(level), w = c.ct_words(level);
  KsJob job;
  job.level = level;
  job.count = m;
  for (int i = 0; i < m; ++i) job.item[i] = KsItem{k.relin, 1};
  job.out = out;
  job.out_stride = out_stride;
  job.top_out = top_out;
  bool at_level = true;  // the fused form reads its operands at the product's level only
  for (int i = first; i < first + m; ++i) at_level = at_level && a[i].level == level && b[i].level == level;
  if (m >= FUSED_TENSOR_ITEMS && at_level) {
    job.tensor = true;
    for (int i = 0; i < m; ++i) {
      job.ta[i] = a[first + i].d;
      job.tb[i] = b[first + i].d;
    }
    key_switch(c, job);
    return;
  }
  Tmp d01(c.pool, (size_t)m * w), d2(c.pool, (size_t)m * poly);
  PtrArgs p;
  for (int i = 0; i < MAX_BATCH; ++i) {
    p.a[i] = i < m ? a[first + i].d : nullptr;
    p.b[i] = i < m ? b[first + i].d : nullptr;
    p.ra[i] = i < m ? a[first + i].level + 1 : 0;
    p.rb[i] = i < m ? b[first + i].level + 1 : 0;
  }
  c.begin_launch();
  hipLaunchKernelGGL(tensor_batch_kernel, grid3(c, l, m), dim3(TPB), 0, c.stream, p, d01.p, d2.p, c.d_mod, c.log_n,
                     level);
  c.end_launch(KC_ELEMWISE, 8.0 * c.n * l * 7.0 * m);
  job.in = d2;
  job.in_stride = poly;
  job.add0 = d01;
  job.add0_stride = w;
  job.add1 = d01.p + poly;
  job.add1_stride = w;
  key_switch(c, job);
}

// The product's level: `level`, with every operand at or above it (read as if mod-dropped), or with level < 0 the
// common level of all operands.
static int product_level(const std::vector<CtView>& a, const std::vector<CtView>& b, int level) {
  if (a.size() != b.size() || a.empty()) fail(HETAL_E_INVALID_ARG, "hmult batch operand counts differ");
  const int lv = level < 0 ? a[0].level : level;
  for (size_t i = 0; i < a.size(); ++i) {
    if (level < 0 && (a[i].level != lv || b[i].level != lv)) fail(HETAL_E_LEVEL, "hmult operands at different levels");
    if (a[i].level < lv || b[i].level < lv) fail(HETAL_E_LEVEL, "hmult operand below the product's level");
  }
  return lv;
}

Batch b_hmult(Context& c, const KeySet& k, const std::vector<CtView>& a, const std::vector<CtView>& b, int at) {
  const int level = product_level(a, b, at), count = (int)a.size();
  if (!k.relin) fail(HETAL_E_NO_KEY, "relinearisation key missing");
  Batch o(c, level, count);
  const size_t w = c.ct_words(level);
  const int group = std::max(1, std::min(MAX_BATCH, c.tune.ks_group));
  for (int first = 0; first < count; first += group) {
    const int m = std::min(group, count - first);
    hmult_group(c, k, a, b, first, m, level, o.d + (size_t)first * w, w, nullptr);
  }
  o.scale = a[0].scale * b[0].scale;
  c.counters[2] += count;
  return o;
}

Batch b_hmult_rescale(Context& c, const KeySet& k, const std::vector<CtView>& a, const std::vector<CtView>& b,
                      int at) {
  const int level = product_level(a, b, at), count = (int)a.size();
  if (!k.relin) fail(HETAL_E_NO_KEY, "relinearisation key missing");
  if (level < 1) fail(HETAL_E_LEVEL, "no level left to rescale");
  Batch o(c, level - 1, count);
  const size_t w = c.ct_words(level), wo = c.ct_words(level - 1);
  const int group = std::max(1, std::min(MAX_BATCH, c.tune.ks_group));
  for (int first = 0; first < count; first += group) {
    const int m = std::min(group, count - first);
    Tmp prod(c.pool, (size_t)m * w), top(c.pool, (size_t)m * 2 * c.n);
    hmult_group(c, k, a, b, first, m, level, prod, w, top);
    k_rescale(c, prod, o.d + (size_t)first * wo, level, m, w, wo, nullptr, 0, nullptr, 0, top);
  }
  o.scale = (a[0].scale * b[0].scale) / (double)c.primes[level];
  c.counters[2] += count;
  return o;
}

Batch b_cmult_masks_rescale(Context& c, MaskCache& mc, BView a, const std::vector<MaskSpec>& masks) {
  if (masks.size() != 1 && (int)masks.size() != a.count) fail(HETAL_E_INVALID_ARG, "one mask or one per item");
  if (a.level < 1) fail(HETAL_E_LEVEL, "no level left to rescale");
  std::vector<const u64*> pts(a.count);
  for (int i = 0; i < a.count; ++i) {
    const MaskSpec& s = masks.size() == 1 ? masks[0] : masks[i];
    pts[i] = mask_pt(c, mc, s.kind, s.k, s.cc, s.s0, s.s1, s.t, a.level);
  }
  Batch o(c, a.level - 1, a.count);
  k_rescale(c, a.d, o.d, a.level, a.count, a.stride, c.ct_words(a.level - 1), nullptr, 0, nullptr, 0, nullptr,
            pts.data());
  const double masked = a.scale * (double)c.primes[a.level];  // the CMult's scale, then the rescale's
  o.scale = masked / (double)c.primes[a.level];
  c.counters[3] += a.count;
  return o;
}

void b_sum_segments_into(Context& c, BView a, const std::vector<int>& sizes, const std::vector<int>& dst, Batch& out) {
  int total = 0;
  for (int z : sizes) {
    if (z < 1) fail(HETAL_E_INVALID_ARG, "empty segment");
    total += z;
  }
  if (sizes.empty() || total != a.count) fail(HETAL_E_INVALID_ARG, "segments must cover the batch");
  if (dst.size() != sizes.size() || out.level != a.level) fail(HETAL_E_INVALID_ARG, "segment destinations");
  for (int d : dst)
    if (d < 0 || d >= out.count) fail(HETAL_E_INVALID_ARG, "segment destination outside the output");
  const int l = a.level + 1;
  const int groups = (int)sizes.size();
  int item = 0;
  for (int first = 0; first < groups; first += MAX_SEGMENTS) {
    const int m = std::min(MAX_SEGMENTS, groups - first);
    SegArgs sg;
    sg.start[0] = 0;
    for (int g = 0; g < m; ++g) {
      sg.start[g + 1] = sg.start[g] + sizes[first + g];
      sg.dst[g] = dst[first + g];
    }
    c.begin_launch();
    hipLaunchKernelGGL(sum_segments_kernel, grid3(c, 2 * l, m), dim3(TPB), 0, c.stream, a.d + (size_t)item * a.stride,
                       a.stride, sg, out.d, c.d_mod, c.log_n, a.level);
    c.end_launch(KC_ELEMWISE, 8.0 * c.n * 2.0 * l * (sg.start[m] + m));
    item += sg.start[m];
  }
  out.scale = a.scale;
}

Batch b_sum_segments(Context& c, BView a, const std::vector<int>& sizes) {
  Batch o(c, a.level, std::max(1, (int)sizes.size()));
  std::vector<int> dst(sizes.size());
  for (size_t g = 0; g < dst.size(); ++g) dst[g] = (int)g;
  b_sum_segments_into(c, a, sizes, dst, o);
  return o;
}

Batch b_sum_groups(Context& c, BView a, int groups) {
  if (groups < 1 || a.count % groups) fail(HETAL_E_INVALID_ARG, "group count must divide the batch");
  return b_sum_segments(c, a, std::vector<int>(groups, a.count / groups));
}

}  // namespace hetal
