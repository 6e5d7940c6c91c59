// CKKS operations on device ciphertexts (host orchestration of the kernels).
#pragma once
#include <map>
#include <memory>
#include <tuple>
#include <utility>

#include "hetal_internal.hpp"

namespace hetal {

// A ciphertext in a pool buffer sized for its level (move-only).
struct Cipher {
  Context* c = nullptr;
  u64* d = nullptr;
  int level = -1;
  double scale = 0.0;

  Cipher() = default;
  Cipher(Context& ctx, int lv) : c(&ctx), d(ctx.pool.get(ctx.ct_words(lv))), level(lv) {}
  ~Cipher() {
    if (d) c->pool.put(d);
  }
  Cipher(Cipher&& o) noexcept : c(o.c), d(o.d), level(o.level), scale(o.scale) { o.d = nullptr; }
  Cipher& operator=(Cipher&& o) noexcept {
    if (this != &o) {
      if (d) c->pool.put(d);
      c = o.c;
      d = o.d;
      level = o.level;
      scale = o.scale;
      o.d = nullptr;
    }
    return *this;
  }
  Cipher(const Cipher&) = delete;
  Cipher& operator=(const Cipher&) = delete;
  u64* c0() const { return d; }
  u64* c1() const { return d + c->poly_words(level); }
};

// A read-only view of a ciphertext owned elsewhere (caller memory or a Cipher).
struct CtView {
  const u64* d;
  int level;
  double scale;
};

inline CtView view(const Cipher& x) { return CtView{x.d, x.level, x.scale}; }

struct SecretKeyDev {
  u64* s = nullptr;  // [nprimes][N], NTT form
};

struct KeySet {
  u64* relin = nullptr;
  std::map<u32, u64*> galois;
  const u64* get(u32 g) const {
    auto it = galois.find(g);
    return it == galois.end() ? nullptr : it->second;
  }
};

u32 galois_rot(const Context& c, int r);
u32 galois_conj(const Context& c);

// Elementary operations writing into `out` (a buffer with room for the result).
void op_add(Context& c, CtView a, CtView b, u64* out, double* scale_out, bool subtract);
void op_mul_i(Context& c, CtView a, u64* out);
void op_mod_drop(Context& c, CtView a, int level, u64* out);
void op_rescale(Context& c, CtView a, u64* out);
void op_cmult(Context& c, CtView a, const u64* pt, u64* out);
void op_hmult(Context& c, const KeySet& k, CtView a, CtView b, u64* out);
void op_galois(Context& c, const KeySet& k, CtView a, u32 g, u64* out);

// Same on pool ciphertexts.
Cipher add(Context& c, CtView a, CtView b);
Cipher sub(Context& c, CtView a, CtView b);
Cipher mul_i(Context& c, CtView a);
Cipher mod_drop(Context& c, CtView a, int level);
Cipher rescale(Context& c, CtView a);
Cipher hmult(Context& c, const KeySet& k, CtView a, CtView b);
Cipher rotate(Context& c, const KeySet& k, CtView a, int r);
Cipher conjugate(Context& c, const KeySet& k, CtView a);

// Masks: slot patterns of one s0 x s1 block, encoded at `level` with scale q_level.
// MASK_LEFT_COLS: 1 on the columns j < s1 - k.  MASK_PAD_COLS: t on the columns with j mod cc >= k.
// MASK_COLS_FROM: t on the columns j >= k.
enum MaskKind { MASK_OFFDIAG_CPLX = 0, MASK_FIRST_COL = 1, MASK_LEFT_COLS = 2, MASK_PAD_COLS = 3, MASK_COLS_FROM = 4 };
struct MaskCache {
  std::map<std::tuple<int, int, int, int, int, double, int>, u64*> pts;
  ~MaskCache();
  Context* c = nullptr;
};
const u64* mask_pt(Context& c, MaskCache& cache, MaskKind kind, int k, int cc, int s0, int s1, double t, int level);
Cipher cmult_mask(Context& c, MaskCache& cache, CtView a, MaskKind kind, int k, int cc, int s0, int s1, double t);
// Slot values (device, [s0 * s1] each) of a mask block.
void mask_slots(Context& c, MaskKind kind, int k, int cc, int s0, int s1, double t, double* d_re, double* d_im);

void encode_slots(Context& c, const double* d_re, const double* d_im, int count, size_t slot_stride, int level,
                  double scale, u64* out, size_t out_stride);

}  // namespace hetal

namespace hetal {

// `count` ciphertexts at one level and scale, item i at d + i * stride words.
struct BView {
  const u64* d;
  int level;
  int count;
  double scale;
  size_t stride;
  CtView item(int i) const { return CtView{d + (size_t)i * stride, level, scale}; }
  BView sub(int first, int n) const { return BView{d + (size_t)first * stride, level, n, scale, stride}; }
};

// A packed batch in one pool buffer (move-only).
struct Batch {
  Context* c = nullptr;
  u64* d = nullptr;
  int level = -1;
  int count = 0;
  double scale = 0.0;

  Batch() = default;
  Batch(Context& ctx, int lv, int n) : c(&ctx), d(ctx.pool.get(ctx.ct_words(lv) * (size_t)n)), level(lv), count(n) {}
  ~Batch() {
    if (d) c->pool.put(d);
  }
  Batch(Batch&& o) noexcept : c(o.c), d(o.d), level(o.level), count(o.count), scale(o.scale) { o.d = nullptr; }
  Batch& operator=(Batch&& o) noexcept {
    if (this != &o) {
      if (d) c->pool.put(d);
      c = o.c;
      d = o.d;
      level = o.level;
      count = o.count;
      scale = o.scale;
      o.d = nullptr;
    }
    return *this;
  }
  Batch(const Batch&) = delete;
  Batch& operator=(const Batch&) = delete;
  BView v() const { return BView{d, level, count, scale, c->ct_words(level)}; }
  CtView item(int i) const { return v().item(i); }
};

struct MaskSpec {
  MaskKind kind;
  int k, cc, s0, s1;
  double t;
};

Batch b_pack(Context& c, const std::vector<CtView>& items);
Batch b_add(Context& c, BView a, BView b);
Batch b_sub(Context& c, BView a, BView b);
// a ± b at `level`, the operands at or above it read as their mod-drops would be (no copy).
Batch b_addsub_at(Context& c, BView a, BView b, int level, bool subtract);
Batch b_mul_i(Context& c, BView a);
Batch b_mod_drop(Context& c, BView a, int level);
Batch b_rescale(Context& c, BView a);
// Item i rotated left by steps[i] (steps.size() == 1: the same step for all).
Batch b_rotate(Context& c, const KeySet& k, BView a, const std::vector<int>& steps);
// tau_{gal[i]}(a[i]) written to out + i out_stride (no identity elements; out must not overlap a).
void b_rotate_into(Context& c, const KeySet& k, BView a, const std::vector<u32>& gal, u64* out, size_t out_stride);
// addend[i] + Lrot(a[i], step) for every item (addend defaults to a itself),
// the addition fused into the key switch's last kernel.
Batch b_rotate_add(Context& c, const KeySet& k, BView a, int step, const BView* addend = nullptr);
// a[i] + conj(a[i]).
Batch b_conj_add(Context& c, const KeySet& k, BView a);
// One ciphertext rotated by each step, sharing one ModUp (hoisting).
Batch b_rotate_hoisted(Context& c, const KeySet& k, CtView a, const std::vector<int>& steps);
Batch b_conj(Context& c, const KeySet& k, BView a);
// Mult (tensor + relinearisation) of the pairs (a[i], b[i]), all at one level; or, with at >= 0, at level `at`
// from operands at or above it, read as their mod-drops would be (no copy).
Batch b_hmult(Context& c, const KeySet& k, const std::vector<CtView>& a, const std::vector<CtView>& b, int at = -1);
// b_hmult then b_rescale, with the rescale's first launch run by the key switch's epilogue: the same words.
Batch b_hmult_rescale(Context& c, const KeySet& k, const std::vector<CtView>& a, const std::vector<CtView>& b,
                      int at = -1);
// CMult of item i by mask masks[i] (or masks[0] for all), each encoded at the batch level with scale q_level,
// then the rescale: in the rescale's three launches, the products formed where the rows are read (the same words
// as a CMult kernel followed by b_rescale).
Batch b_cmult_masks_rescale(Context& c, MaskCache& mc, BView a, const std::vector<MaskSpec>& masks);
// out[g] = sum over t < per of a[g * per + t], per = a.count / groups.
Batch b_sum_groups(Context& c, BView a, int groups);
// out[g] = sum of the g-th run of sizes[g] consecutive items (the runs cover the batch in order).
Batch b_sum_segments(Context& c, BView a, const std::vector<int>& sizes);
// The same sums written to items dst[g] of `out` (allocated by the caller at a's level; other items untouched).
void b_sum_segments_into(Context& c, BView a, const std::vector<int>& sizes, const std::vector<int>& dst, Batch& out);

}  // namespace hetal
