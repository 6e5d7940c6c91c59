// The paper's row-wise softmax approximation (App. softmax, Alg. "Row-wise softmax approximation"):
// ASoftmax = p o D_n o Norm on horizontally tiled block matrices, with the constant operations that
// evaluating real polynomials on ciphertexts needs.
//
// Readings where the paper is silent or garbled (the same as the oracle's):
//  * R = 8, L = 2, n = 5 by default; R_max = ceil(R L^n); M_max starts as M'; log2 c' max rounds.
//  * Acomp(a, b) = (f(g(g(g(a - b)))) + 1) / 2 (comp_g = 3 compositions of g): with two, the maximum
//    of 10 classes can stay ~6 below the true one and AInv leaves its range, against the error table.
//  * B_inv(x) = x + k (x^3 / R^2 - x^5 / R^4), the approximate inverse of D_n.
//  * The max is broadcast by Rrot(x, 2^j), j < log2 s1; "x 2 R_max" is an integer multiplication.
//  * D_c covers the first c columns of each row; the row sum runs over the first period CS-style;
//    slots outside the first period get 1 before AInv; M_sm = M_exp (x) M_Z; the output is
//    replicated by Rrot(x, 2^j c').
//  * AExp(x) = p(x / B)^B (B = 8, p of degree 12); AInv is Goldschmidt's iteration on x / R_inv.
//  * Real constants are encoded at scale q_level and rescaled; sums of operands with different
//    scales bring the second to the first's scale with a constant 1 (one level); an operand below
//    the depth of its next step is refreshed through the caller's callback (the paper bootstraps).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <set>

#include "matrix.hpp"
#include "softmax.hpp"

namespace hetal {

namespace {

constexpr int TPB = 256;

struct LimbConsts {
  u64 k[MAX_PRIMES];
  u64 ksh[MAX_PRIMES];
};

dim3 grid3(const Context& c, int y, int z) { return dim3((unsigned)(c.n / TPB), (unsigned)y, (unsigned)z); }

// out[item][row] = a[item][row] * K_i mod q_i (rows 0..2l-1, i = row mod l).
__global__ void __launch_bounds__(TPB) mul_const_kernel(const u64* __restrict__ a, size_t a_stride,
                                                        u64* __restrict__ out, size_t out_stride, LimbConsts kc,
                                                        const ModInfo* __restrict__ mods, int log_n, int level) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int row = blockIdx.y;
  const int i = row % l;
  const size_t item = blockIdx.z;
  out[item * out_stride + (size_t)row * n + k] =
      mul_shoup(a[item * a_stride + (size_t)row * n + k], kc.k[i], kc.ksh[i], mods[i].q);
}

// c0 rows get + K_i (a constant polynomial is K in every NTT-domain word); c1 rows are copied.
__global__ void __launch_bounds__(TPB) add_const_kernel(const u64* __restrict__ a, size_t a_stride,
                                                        u64* __restrict__ out, size_t out_stride, LimbConsts kc,
                                                        const ModInfo* __restrict__ mods, int log_n, int level) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int row = blockIdx.y;
  const size_t item = blockIdx.z;
  u64 v = a[item * a_stride + (size_t)row * n + k];
  if (row < l) v = add_mod(v, kc.k[row], mods[row].q);
  out[item * out_stride + (size_t)row * n + k] = v;
}

// c0 rows get + pt; c1 rows are copied.
__global__ void __launch_bounds__(TPB) add_plain_kernel(const u64* __restrict__ a, size_t a_stride,
                                                        const u64* __restrict__ pt, u64* __restrict__ out,
                                                        size_t out_stride, const ModInfo* __restrict__ mods, int log_n,
                                                        int level) {
  const int n = 1 << log_n;
  const int l = level + 1;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const int row = blockIdx.y;
  const size_t item = blockIdx.z;
  u64 v = a[item * a_stride + (size_t)row * n + k];
  if (row < l) v = add_mod(v, pt[(size_t)row * n + k], mods[row].q);
  out[item * out_stride + (size_t)row * n + k] = v;
}

// Coefficient-form plaintext m (rows 0..level) lifted from q_0: y = [m_0]_centred (*bad is set when a row
// i <= level disagrees with y mod q_i), re-encoded as rint(y * ratio) when `rescale` (ties to even), and written
// modulo each of the out_rows primes.
__global__ void __launch_bounds__(TPB) lift_q0_kernel(const u64* __restrict__ m, int level, u64* __restrict__ out,
                                                      int out_rows, const ModInfo* __restrict__ mods, int log_n,
                                                      double ratio, int rescale, int* __restrict__ bad) {
  const int n = 1 << log_n;
  const int k = blockIdx.x * TPB + threadIdx.x;
  const u64 q0 = mods[0].q;
  const u64 v = m[k];
  const bool neg = v > q0 / 2;
  u64 mag = neg ? q0 - v : v;  // |y|
  for (int i = 1; i <= level; ++i) {
    const u64 q = mods[i].q;
    const u64 r = mag % q;
    if ((neg ? (r ? q - r : 0) : r) != m[(size_t)i * n + k]) *bad = 1;
  }
  bool sneg = neg;
  if (rescale) {
    const double z = rint((double)(neg ? -(i64)mag : (i64)mag) * ratio);
    sneg = z < 0.0;
    mag = (u64)(sneg ? -z : z);
  }
  for (int i = 0; i < out_rows; ++i) {
    const u64 q = mods[i].q;
    const u64 r = mag % q;
    out[(size_t)i * n + k] = sneg ? (r ? q - r : 0) : r;
  }
}

LimbConsts limb_consts(const Context& c, i64 K, int level) {
  LimbConsts kc;
  std::memset(&kc, 0, sizeof(kc));
  for (int i = 0; i <= level; ++i) {
    const u64 q = c.primes[i];
    const u64 mag = (u64)(K < 0 ? -K : K) % q;
    const u64 r = K < 0 ? (mag ? q - mag : 0) : mag;
    kc.k[i] = r;
    kc.ksh[i] = (u64)(((unsigned __int128)r << 64) / q);
  }
  return kc;
}

}  // namespace

i64 round_const(double v) {
  const double r = std::nearbyint(v);
  if (!(std::fabs(r) < 4611686018427387904.0)) fail(HETAL_E_OVERFLOW, "constant does not fit in 62 bits");
  return (i64)r;
}

Batch b_mul_const(Context& c, BView a, double value, double sigma) {
  const i64 K = round_const(value * sigma);
  Batch o(c, a.level, a.count);
  const LimbConsts kc = limb_consts(c, K, a.level);
  c.begin_launch();
  hipLaunchKernelGGL(mul_const_kernel, grid3(c, 2 * (a.level + 1), a.count), dim3(TPB), 0, c.stream, a.d, a.stride,
                     o.d, c.ct_words(a.level), kc, c.d_mod, c.log_n, a.level);
  c.end_launch(KC_ELEMWISE, 16.0 * a.count * c.ct_words(a.level));
  o.scale = a.scale * sigma;
  return o;
}

Batch b_mul_const_rescale(Context& c, BView a, int level, double value, double sigma, const BView* addend) {
  if (level < 1 || level > a.level) fail(HETAL_E_LEVEL, "constant product and rescale: level out of range");
  const i64 K = round_const(value * sigma);
  const LimbConsts kc = limb_consts(c, K, level);
  double scale = a.scale * sigma / (double)c.primes[level];
  if (addend) {  // the checks of b_add(addend, result), whose scale is the addend's
    if (addend->level != level - 1 || addend->count != a.count)
      fail(HETAL_E_LEVEL, "batch operands differ in level or count");
    if (std::abs(addend->scale - scale) > 1e-9 * std::max(std::abs(addend->scale), std::abs(scale)))
      fail(HETAL_E_SCALE, "batch operands with different scales");
    scale = addend->scale;
  }
  Batch o(c, level - 1, a.count);
  k_rescale(c, a.d, o.d, level, a.count, a.stride, c.ct_words(level - 1), kc.k, a.level + 1,
            addend ? addend->d : nullptr, addend ? addend->stride : 0);
  o.scale = scale;
  return o;
}

Batch b_add_const(Context& c, BView a, double value) {
  const i64 K = round_const(value * a.scale);
  Batch o(c, a.level, a.count);
  const LimbConsts kc = limb_consts(c, K, a.level);
  c.begin_launch();
  hipLaunchKernelGGL(add_const_kernel, grid3(c, 2 * (a.level + 1), a.count), dim3(TPB), 0, c.stream, a.d, a.stride,
                     o.d, c.ct_words(a.level), kc, c.d_mod, c.log_n, a.level);
  c.end_launch(KC_ELEMWISE, 16.0 * a.count * c.ct_words(a.level));
  o.scale = a.scale;
  return o;
}

Batch b_add_plain(Context& c, BView a, const u64* pt) {
  Batch o(c, a.level, a.count);
  c.begin_launch();
  hipLaunchKernelGGL(add_plain_kernel, grid3(c, 2 * (a.level + 1), a.count), dim3(TPB), 0, c.stream, a.d, a.stride,
                     pt, o.d, c.ct_words(a.level), c.d_mod, c.log_n, a.level);
  c.end_launch(KC_ELEMWISE, 8.0 * a.count * c.ct_words(a.level) * 2.0 + 8.0 * c.poly_words(a.level));
  o.scale = a.scale;
  return o;
}

void refresh_encrypt(Context& c, const u64* s, CtView ct, double scale, const u64* a_ntt, const u64* e_ntt,
                     u64* out) {
  const int top = c.num_q - 1;
  const size_t poly = c.poly_words(ct.level);
  Tmp m(c.pool, poly);
  k_decrypt(c, ct.d, s, m, ct.level);
  RowsRef rows = c.rows(ROWS_CT, ct.level);
  ntt_inverse(c, m, 0, 1, RowsRef{rows.d, ct.level + 1});
  const int rescale = scale > 0.0 ? 1 : 0;
  const double ratio = rescale ? scale / ct.scale : 1.0;
  if (rescale && !(std::fabs(ratio) < 1e12)) fail(HETAL_E_SCALE, "refresh scale ratio out of range");
  Tmp lifted(c.pool, c.poly_words(top));
  Tmp flag(c.pool, 1);
  HCHECK(hipMemsetAsync(flag.p, 0, 8, c.stream));
  c.begin_launch();
  hipLaunchKernelGGL(lift_q0_kernel, dim3((unsigned)(c.n / TPB)), dim3(TPB), 0, c.stream, m.p, ct.level, lifted.p,
                     top + 1, c.d_mod, c.log_n, ratio, rescale, reinterpret_cast<int*>(flag.p));
  c.end_launch(KC_ELEMWISE, 8.0 * c.n * (ct.level + 1 + top + 1));
  int bad = 0;
  HCHECK(hipMemcpyAsync(&bad, flag.p, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  HCHECK(hipStreamSynchronize(c.stream));
  if (bad) fail(HETAL_E_OVERFLOW, "message too large to lift from q_0 (|m| >= q_0 / 2)");
  RowsRef top_rows = c.rows(ROWS_CT, top);
  ntt_forward(c, lifted, 0, 1, RowsRef{top_rows.d, top + 1});
  k_encrypt(c, a_ntt, e_ntt, lifted, s, out, top);
}

// ---------------------------------------------------------------- the level rule and the building blocks

namespace {

// Ciphertexts of one step: either the caller's (a view) or owned here.
struct Val {
  Batch own;
  std::shared_ptr<Batch> shared;  // a part of a batch several values were computed in
  BView v;
  Val() : v{nullptr, -1, 0, 0.0, 0} {}
  explicit Val(BView x) : v(x) {}
  explicit Val(Batch&& b) : own(std::move(b)) { v = own.v(); }
  Val(Val&& o) noexcept : own(std::move(o.own)), shared(std::move(o.shared)), v(o.v) {
    if (own.d) v = own.v();
  }
  Val& operator=(Val&& o) noexcept {
    own = std::move(o.own);
    shared = std::move(o.shared);
    v = o.v;
    if (own.d) v = own.v();
    return *this;
  }
  int level() const { return v.level; }
  double scale() const { return v.scale; }
};

int split_hi(int k) {
  int a = 1;
  while (a * 2 <= k) a *= 2;
  return a == k ? k / 2 : a;
}

int power_depth(int k) {
  if (k <= 1) return 0;
  const int a = split_hi(k), b = k - a;
  return std::max(power_depth(a), power_depth(b)) + 1;
}

struct Steps {
  Context& c;
  const KeySet& k;
  MaskCache* mc;
  Refresher& rf;
  int s0 = 0, s1 = 0;

  Val need(Val x, int d) {
    if (x.level() >= d) return x;
    const int top = c.num_q - 1;
    if (!rf.fn || d > top) fail(HETAL_E_LEVEL, "depth budget exhausted (no refresh, and the library does not bootstrap)");
    Batch out(c, top, x.v.count);
    const size_t wtop = c.ct_words(top), w = c.ct_words(x.level());
    for (int i = 0; i < x.v.count; ++i) {
      // the item goes into its slot of the output, where the key holder re-encrypts it in place
      u64* slot = out.d + (size_t)i * wtop;
      HCHECK(hipMemcpyAsync(slot, x.v.item(i).d, w * 8, hipMemcpyDeviceToDevice, c.stream));
      HCHECK(hipStreamSynchronize(c.stream));
      hetal_ct h;
      h.data = slot;
      h.capacity = wtop;
      h.level = x.level();
      h.scale = x.scale();
      const int rc = rf.fn(rf.user, &h);
      if (rc != HETAL_OK) fail(rc, "refresh callback failed");
      if (h.data != slot || h.level != top || !(h.scale > 0.0) || !std::isfinite(h.scale))
        fail(HETAL_E_INVALID_ARG, "refresh must re-encrypt in place at the top level with a positive scale");
      if (i > 0 && h.scale != out.scale) fail(HETAL_E_SCALE, "refresh gave the items of one batch different scales");
      out.scale = h.scale;
      rf.count += 1;
    }
    return Val(std::move(out));
  }

  Val rescale(const Val& x) { return Val(b_rescale(c, x.v)); }

  // x * v with v at scale q_level, rescaled (the scale is kept; one level).
  Val cconst(Val x, double v) {
    x = need(std::move(x), 1);
    const double q = (double)c.primes[x.level()];
    return Val(b_mul_const_rescale(c, x.v, x.level(), v, q));
  }

  Val mulint(const Val& x, i64 kk) { return Val(b_mul_const(c, x.v, (double)kk, 1.0)); }

  Val add_const(const Val& x, double v) { return Val(b_add_const(c, x.v, v)); }

  Val add_plain(const Val& x, MaskKind kind, int kk, int cc, double t) {
    Tmp slots(c.pool, 2 * (size_t)c.slots);
    double* re = reinterpret_cast<double*>(slots.p);
    mask_slots(c, kind, kk, cc, s0, s1, t, re, re + c.slots);
    Tmp pt(c.pool, c.poly_words(x.level()));
    encode_slots(c, re, re + c.slots, 1, 0, x.level(), x.scale(), pt, 0);
    return Val(b_add_plain(c, x.v, pt));
  }

  Val mask(Val x, MaskKind kind, int kk) {
    x = need(std::move(x), 1);
    return Val(b_cmult_masks_rescale(c, *mc, x.v, {MaskSpec{kind, kk, 0, s0, s1, 1.0}}));
  }

  Val rot(const Val& x, int r) { return Val(b_rotate(c, k, x.v, {r})); }

  Val mult(Val a, Val b, bool same) {
    a = need(std::move(a), 1);
    if (!same) b = need(std::move(b), 1);
    const BView av = a.v, bv = same ? a.v : b.v;
    const int lv = std::min(av.level, bv.level);  // an operand above it is read as its mod-drop (no copy)
    std::vector<CtView> va, vb;
    for (int i = 0; i < av.count; ++i) {
      va.push_back(av.item(i));
      vb.push_back(bv.item(i));
    }
    return Val(b_hmult_rescale(c, k, va, vb, lv));
  }

  // Independent products as one lockstep Mult + rescale: every item goes through the operations it would get
  // alone, and each result gets the scale a single product would ((s_a s_b) / q).  Only when no operand needs a
  // refresh and all pairs land on one level (else false, nothing done), so the refresh order is unchanged.
  bool mult_group(const std::vector<std::pair<BView, BView>>& ops, std::vector<Val>& out) {
    int lv = -1;
    for (const auto& op : ops) {
      if (op.first.level < 1 || op.second.level < 1) return false;
      const int l = std::min(op.first.level, op.second.level);
      if (lv >= 0 && l != lv) return false;
      lv = l;
    }
    std::vector<CtView> va, vb;
    for (const auto& op : ops) {
      for (int i = 0; i < op.first.count; ++i) {
        va.push_back(op.first.item(i));
        vb.push_back(op.second.item(i));
      }
    }
    auto r = std::make_shared<Batch>(b_hmult_rescale(c, k, va, vb, lv));
    const size_t w = c.ct_words(lv - 1);
    size_t off = 0;
    out.clear();
    for (const auto& op : ops) {
      Val x;
      x.shared = r;
      x.v = BView{r->d + off * w, lv - 1, op.first.count, op.first.scale * op.second.scale / (double)c.primes[lv], w};
      off += op.first.count;
      out.push_back(std::move(x));
    }
    return true;
  }

  Val combine(Val a, Val b, bool subtract) {
    const double sa = a.scale(), sb = b.scale();
    if (std::abs(sa - sb) > 1e-9 * std::max(std::abs(sa), std::abs(sb))) {
      b = need(std::move(b), 1);
      const double q = (double)c.primes[b.level()];
      const double sigma = sa * q / sb;
      b = Val(b_mul_const_rescale(c, b.v, b.level(), 1.0, sigma));
    }
    return Val(b_addsub_at(c, a.v, b.v, std::min(a.level(), b.level()), subtract));
  }

  Val poly(Val x, const std::vector<double>& coeffs) {
    std::vector<int> ks;
    for (int kk = 1; kk < (int)coeffs.size(); ++kk)
      if (coeffs[kk] != 0.0) ks.push_back(kk);
    if (ks.empty()) fail(HETAL_E_INVALID_ARG, "constant polynomial");
    int depth = 0;
    for (int kk : ks) depth = std::max(depth, power_depth(kk) + 1);
    x = need(std::move(x), depth);
    const double target = x.scale();
    std::set<int> needed;
    std::vector<int> stack(ks.begin(), ks.end());
    while (!stack.empty()) {
      const int kk = stack.back();
      stack.pop_back();
      if (!needed.insert(kk).second) continue;
      if (kk > 1) {
        stack.push_back(split_hi(kk));
        stack.push_back(kk - split_hi(kk));
      }
    }
    std::map<int, Val> pw;
    pw[1] = std::move(x);
    // the powers of one depth are independent: one batched product per depth (the factors stay in the table)
    int maxd = 0;
    for (int kk : needed) maxd = std::max(maxd, power_depth(kk));
    for (int d = 1; d <= maxd; ++d) {
      std::vector<int> kd;
      std::vector<std::pair<BView, BView>> ops;
      for (int kk : needed)
        if (kk > 1 && power_depth(kk) == d) {
          kd.push_back(kk);
          ops.push_back({pw[split_hi(kk)].v, pw[kk - split_hi(kk)].v});
        }
      std::vector<Val> res;
      if (mult_group(ops, res)) {
        for (size_t i = 0; i < kd.size(); ++i) pw[kd[i]] = std::move(res[i]);
      } else {
        for (int kk : kd) {
          const int a = split_hi(kk), b = kk - a;
          pw[kk] = mult(Val(pw[a].v), Val(pw[b].v), a == b);
        }
      }
    }
    int lt = 1 << 30;
    for (int kk : ks) lt = std::min(lt, pw[kk].level() - 1);
    const double q = (double)c.primes[lt + 1];
    Val acc;
    bool first = true;
    for (int kk : ks) {
      const double sigma = target * q / pw[kk].scale();
      if (first) {
        acc = Val(b_mul_const_rescale(c, pw[kk].v, lt + 1, coeffs[kk], sigma));
        first = false;
      } else {  // the running sum is the rescale's addend
        acc = Val(b_mul_const_rescale(c, pw[kk].v, lt + 1, coeffs[kk], sigma, &acc.v));
      }
    }
    if (coeffs[0] != 0.0) acc = add_const(acc, coeffs[0]);
    return acc;
  }
};

// The result as a batch of its own (a packed copy when it is still a view of the caller's input).
Batch owned(Context& c, Val&& x) {
  if (x.own.d) return std::move(x.own);
  std::vector<CtView> items;
  for (int i = 0; i < x.v.count; ++i) items.push_back(x.v.item(i));
  return b_pack(c, items);
}

// f and g of the comparison (App. softmax), integer numerators over power-of-two denominators.
constexpr int F_NUM[8] = {0, 35, 0, -35, 0, 21, 0, -5};
constexpr int G_NUM[8] = {0, 4589, 0, -16577, 0, 25614, 0, -12860};
constexpr double F_DEN = 16.0, G_DEN = 1024.0;

std::vector<double> g_coeffs() {
  std::vector<double> v(8);
  for (int i = 0; i < 8; ++i) v[i] = (double)G_NUM[i] / G_DEN;
  return v;
}

std::vector<double> comp_out_coeffs() {  // (f + 1) / 2
  std::vector<double> v(8);
  for (int i = 0; i < 8; ++i) v[i] = (double)F_NUM[i] / (2.0 * F_DEN);
  v[0] = 0.5;
  return v;
}

std::vector<double> dep_coeffs(const SoftmaxArgs& a, int i) {  // x - 4 x^3 / (27 R^2 L^(2i))
  return {0.0, 1.0, 0.0, -4.0 / (27.0 * a.R * a.R * std::pow(a.L, 2 * i))};
}

std::vector<double> dep_inv_coeffs(const SoftmaxArgs& a) {  // x + k (x^3 / R^2 - x^5 / R^4)
  const double l2 = std::pow(a.L, 2), l2n = std::pow(a.L, 2 * a.n);
  const double kk = 4.0 * l2 * (l2n - 1.0) / (27.0 * l2n * (l2 - 1.0));
  return {0.0, 1.0, 0.0, kk / std::pow(a.R, 2), 0.0, -kk / std::pow(a.R, 4)};
}

}  // namespace

Batch poly_eval(Context& c, const KeySet& k, BView x, const std::vector<double>& coeffs, Refresher& rf) {
  Steps S{c, k, nullptr, rf};
  Val r = S.poly(Val(x), coeffs);
  return owned(c, std::move(r));
}

std::vector<int> softmax_rot_steps(int cc, int s1) {
  int cp = 1;
  while (cp < cc) cp *= 2;
  std::set<int> st;
  for (int j = 1; j < cp; j *= 2) {
    st.insert(j);
    st.insert(-j);
  }
  for (int j = 1; j < s1; j *= 2) st.insert(-j);
  for (int j = cp; j < s1; j *= 2) st.insert(-j);
  return std::vector<int>(st.begin(), st.end());
}

Batch softmax_approx(Context& c, const KeySet& k, MaskCache& mc, BView m, int cc, int s0, int s1,
                     const SoftmaxArgs& a, Refresher& rf) {
  int cp = 1;
  while (cp < cc) cp *= 2;
  if (cc < 1 || cp > s1 || s1 % cp) fail(HETAL_E_SHAPE, "the padded class count c' must divide s1");
  if (a.exp_B < 1 || (a.exp_B & (a.exp_B - 1))) fail(HETAL_E_INVALID_ARG, "exp_B must be a power of two");
  Steps S{c, k, &mc, rf, s0, s1};
  const long rmax = (long)std::ceil(a.R * std::pow(a.L, a.extend ? a.n : 0));

  Val x0 = S.need(Val(m), 1);
  Val x = S.cconst(Val(x0.v), 1.0 / (2.0 * (double)rmax));
  if (cc != cp) x = S.add_plain(x, MASK_PAD_COLS, cc, cp, -0.5);
  // normalisation: approximate row maximum by pairwise comparisons, broadcast along the row
  Val mmax = std::move(x);
  for (int j = 1; j < cp; j *= 2) {
    Val mrot = S.rot(mmax, j);
    Val y = S.combine(Val(mmax.v), Val(mrot.v), true);
    for (int t = 0; t < a.comp_g; ++t) y = S.poly(std::move(y), g_coeffs());
    Val comp = S.poly(std::move(y), comp_out_coeffs());
    Val onem = S.add_const(S.mulint(comp, -1), 1.0);
    Val t1, t2;
    std::vector<Val> both;
    if (S.mult_group({{mmax.v, comp.v}, {mrot.v, onem.v}}, both)) {
      t1 = std::move(both[0]);
      t2 = std::move(both[1]);
    } else {
      t1 = S.mult(Val(mmax.v), Val(comp.v), false);
      t2 = S.mult(Val(mrot.v), Val(onem.v), false);
    }
    mmax = S.combine(std::move(t1), std::move(t2), false);
  }
  mmax = S.mask(std::move(mmax), MASK_FIRST_COL, 0);
  for (int j = 1; j < s1; j *= 2) mmax = S.combine(Val(mmax.v), S.rot(mmax, -j), false);
  mmax = S.mulint(mmax, 2 * rmax);
  Val xn = S.mask(S.combine(Val(x0.v), Val(mmax.v), true), MASK_LEFT_COLS, s1 - cc);
  // domain extension
  if (a.extend) {
    for (int i = a.n - 1; i >= 0; --i) xn = S.poly(std::move(xn), dep_coeffs(a, i));
    if (a.precise) xn = S.poly(std::move(xn), dep_inv_coeffs(a));
  }
  // exponential, row sum over the first period, reciprocal
  Val e = S.poly(std::move(xn), a.exp_coeffs);
  for (int b = a.exp_B; b > 1; b /= 2) e = S.mult(Val(e.v), Val(e.v), true);
  e = S.mask(std::move(e), MASK_LEFT_COLS, s1 - cc);
  Val s = Val(e.v);
  for (int j = 1; j < cp; j *= 2) s = S.combine(Val(s.v), S.rot(s, j), false);
  s = S.mask(std::move(s), MASK_FIRST_COL, 0);
  for (int j = 1; j < cp; j *= 2) s = S.combine(Val(s.v), S.rot(s, -j), false);
  s = S.add_plain(s, MASK_COLS_FROM, cp, 0, 1.0);
  Val y = S.cconst(std::move(s), 1.0 / a.inv_R);
  Val bq = S.add_const(S.mulint(y, -1), 1.0);
  Val av = S.add_const(bq, 1.0);
  // b <- b^2, a <- a (1 + b), pipelined: a's product of one step runs with the next step's square (both read the
  // same b) as one batch whenever neither needs a refresh; otherwise in the order written.
  if (a.inv_iters > 0) bq = S.mult(Val(bq.v), Val(bq.v), true);
  for (int t = 0; t < a.inv_iters; ++t) {
    Val onep = S.add_const(bq, 1.0);
    std::vector<Val> both;
    if (t + 1 < a.inv_iters && S.mult_group({{av.v, onep.v}, {bq.v, bq.v}}, both)) {
      av = std::move(both[0]);
      bq = std::move(both[1]);
    } else {
      av = S.mult(Val(av.v), std::move(onep), false);
      if (t + 1 < a.inv_iters) bq = S.mult(Val(bq.v), Val(bq.v), true);
    }
  }
  Val z = S.cconst(std::move(av), 1.0 / a.inv_R);
  Val sm = S.mult(Val(e.v), Val(z.v), false);
  for (int j = cp; j < s1; j *= 2) sm = S.combine(Val(sm.v), S.rot(sm, -j), false);
  return owned(c, std::move(sm));
}

NagResult nag_step(Context& c, const KeySet& k, MaskCache& mc, BView X, int n_rb, int n_cb, BView Y, BView W,
                   BView V, int cls, int s0, int s1, double lr, double gamma, const SoftmaxArgs& a, Refresher& rf) {
  int cp = 1;
  while (cp < cls) cp *= 2;
  Steps S{c, k, &mc, rf, s0, s1};
  Val Xv = S.need(Val(X), 3);
  Val Vv = S.need(Val(V), 3);
  std::vector<std::vector<CtView>> A(n_rb);
  for (int i = 0; i < n_rb; ++i)
    for (int j = 0; j < n_cb; ++j) A[i].push_back(Xv.v.item(i * n_cb + j));
  std::vector<CtView> Bbar;
  for (int j = 0; j < n_cb; ++j) Bbar.push_back(Vv.v.item(j));
  Batch L = diag_abt_batch(c, k, mc, A, Bbar, cp, s0, s1, 1.0);
  Batch P = softmax_approx(c, k, mc, L.v(), cls, s0, s1, a, rf);
  L = Batch();
  Val D = S.combine(Val(P.v()), Val(Y), true);
  D = S.need(std::move(D), 4);
  std::vector<CtView> Abar;
  for (int i = 0; i < n_rb; ++i) Abar.push_back(D.v.item(i));
  Batch G = diag_atb_batch(c, k, mc, Abar, A, cp, s0, s1, -lr);
  Val Wn = S.combine(Val(Vv.v), Val(G.v()), false);
  // the two scalings in this order (each may refresh its operand)
  Val t1 = S.cconst(Val(Wn.v), 1.0 - gamma);
  Val t2 = S.cconst(Val(W), gamma);
  Val Vn = S.combine(std::move(t1), std::move(t2), false);
  NagResult r;
  r.W = owned(c, std::move(Wn));
  r.V = owned(c, std::move(Vn));
  return r;
}

std::vector<double> default_exp_coeffs(int degree, int B) {
  // Gauss-Legendre nodes and weights (64 points) by Newton's iteration on P_64.
  const int np = 64;
  std::vector<double> xs(np), ws(np);
  for (int i = 0; i < np; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (np + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int kk = 2; kk <= np; ++kk) {
        const double p2 = ((2.0 * kk - 1.0) * x * p1 - (kk - 1.0) * p0) / kk;
        p0 = p1;
        p1 = p2;
      }
      const double dp = np * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::abs(dx) < 1e-17) break;
    }
    double p0 = 1.0, p1 = x;
    for (int kk = 2; kk <= np; ++kk) {
      const double p2 = ((2.0 * kk - 1.0) * x * p1 - (kk - 1.0) * p0) / kk;
      p0 = p1;
      p1 = p2;
    }
    const double dp = np * (x * p1 - p0) / (x * x - 1.0);
    xs[i] = x;
    ws[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  // Legendre coefficients of e^t, then the monomial coefficients of sum_k leg_k P_k.
  std::vector<std::vector<double>> P(degree + 1, std::vector<double>(degree + 1, 0.0));
  P[0][0] = 1.0;
  if (degree >= 1) P[1][1] = 1.0;
  for (int kk = 1; kk < degree; ++kk)
    for (int j = 0; j <= degree; ++j) {
      double v = -(double)kk * P[kk - 1][j];
      if (j > 0) v += (2.0 * kk + 1.0) * P[kk][j - 1];
      P[kk + 1][j] = v / (kk + 1.0);
    }
  std::vector<double> mono(degree + 1, 0.0);
  for (int kk = 0; kk <= degree; ++kk) {
    double acc = 0.0;
    for (int i = 0; i < np; ++i) {
      double p0 = 1.0, p1 = xs[i], pk = kk == 0 ? 1.0 : xs[i];
      for (int j = 2; j <= kk; ++j) {
        const double p2 = ((2.0 * j - 1.0) * xs[i] * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
        pk = p2;
      }
      acc += ws[i] * std::exp(xs[i]) * pk;
    }
    const double leg = (2.0 * kk + 1.0) / 2.0 * acc;
    for (int j = 0; j <= degree; ++j) mono[j] += leg * P[kk][j];
  }
  for (int j = 0; j <= degree; ++j) mono[j] /= std::pow((double)B, j);
  return mono;
}

}  // namespace hetal
