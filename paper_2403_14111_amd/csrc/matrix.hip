// The paper's encrypted matrix products: DiagABT (Alg. 1, Prop. 1) and
// DiagATB (Alg. 4, Prop. 2) with RotLeft (Alg. 2), PRotUp (Alg. 3), and the
// block operations CS and RS (Sec. 4.2, App. B.3), over block-encoded
// matrices (App. B.1).
//
// Readings where the paper leaves the procedure open:
//  * RU(B, k) on a block is Lrot(B, k s1).
//  * CS: for m < log s1, x += Lrot(x, 2^m); x <- rescale(x * D_firstcol);
//    for m < log s1, x += Rrot(x, 2^m)   (2 log s1 rotations, one CMult).
//  * RS: for m < log s0, x += Lrot(x, 2^m s1).
//  * DiagATB uses the mask M^(-k, c) and sums over k < c/2.
//  * Every product of a loop is taken at one common level reached by
//    dropping moduli; masks are encoded with scale q_level, so CMult + rescale
//    keeps the scale; a block product sum is relinearised per product and
//    rescaled once.
//
// Schedule on the GPU: the c/2 iterations of the k-loop and all blocks run in
// lockstep as batches.  Same-key rotations (the CS / RS steps, the B_cplx
// rotation, the conjugations, every relinearisation) form one key-switch
// batch each, which reads the key once; the RU / RotLeft rotations of one
// ciphertext by k = 1 .. c/2-1 share one ModUp (hoisting).  Each ciphertext
// still goes through exactly the key switches and rescales the algorithm
// prescribes, so the result is bit-identical to the sequential schedule.
#include <algorithm>
#include <vector>

#include "matrix.hpp"

namespace hetal {

namespace {

int log2_exact(int x, const char* what) {
  int r = 0;
  while ((1 << r) < x) ++r;
  if ((1 << r) != x) fail(HETAL_E_SHAPE, std::string(what) + " must be a power of two");
  return r;
}

void check_block_shape(const Context& c, int s0, int s1) {
  if (s0 < 1 || s1 < 1 || (long)s0 * s1 != c.slots) fail(HETAL_E_SHAPE, "s0 * s1 must equal the slot count N/2");
  log2_exact(s0, "s0");
  log2_exact(s1, "s1");
}

BView one(CtView x) { return BView{x.d, x.level, 1, x.scale, 0}; }

// CS on every item of a batch.
Batch col_sum(Context& c, const KeySet& k, MaskCache& mc, Batch x, int s0, int s1) {
  const int lg = log2_exact(s1, "s1");
  for (int m = 0; m < lg; ++m) x = b_rotate_add(c, k, x.v(), 1 << m);
  Batch masked = b_cmult_masks(c, mc, x.v(), {MaskSpec{MASK_FIRST_COL, 0, 0, s0, s1, 1.0}});
  x = b_rescale(c, masked.v());
  for (int m = 0; m < lg; ++m) x = b_rotate_add(c, k, x.v(), -(1 << m));
  return x;
}

// RS on every item of a batch.
Batch row_sum(Context& c, const KeySet& k, Batch x, int s0, int s1) {
  const int lg = log2_exact(s0, "s0");
  for (int m = 0; m < lg; ++m) x = b_rotate_add(c, k, x.v(), (1 << m) * s1);
  return x;
}

// Completes RL (Alg. 2) from A1 = Lrot(A, k_i) (item i): A2 = rescale(A1 * D_{k_i}),
// RL = A2 + Rrot(A1 - A2, s1).  One level.
Batch rot_left_finish(Context& c, const KeySet& k, MaskCache& mc, const Batch& a1, const std::vector<int>& ks, int s0,
                      int s1) {
  std::vector<MaskSpec> masks;
  for (int kk : ks) masks.push_back(MaskSpec{MASK_LEFT_COLS, kk, 0, s0, s1, 1.0});
  Batch a2m = b_cmult_masks(c, mc, a1.v(), masks);
  Batch a2 = b_rescale(c, a2m.v());
  Batch a1d = b_mod_drop(c, a1.v(), a2.level);
  Batch rest = b_sub(c, a1d.v(), a2.v());
  BView a2v = a2.v();
  return b_rotate_add(c, k, rest.v(), -s1, &a2v);
}

// PRU (Alg. 3) of one ciphertext b for k = ks[i]: B' = rescale(b * D_k),
// PRU = B' + Lrot(b - B', s1).  One level.
Batch partial_rot_up(Context& c, const KeySet& k, MaskCache& mc, CtView b, const std::vector<int>& ks, int s0, int s1) {
  const int m = (int)ks.size();
  std::vector<MaskSpec> masks;
  for (int kk : ks) masks.push_back(MaskSpec{MASK_LEFT_COLS, kk, 0, s0, s1, 1.0});
  BView bc = BView{b.d, b.level, m, b.scale, 0};
  Batch bpm = b_cmult_masks(c, mc, bc, masks);
  Batch bp = b_rescale(c, bpm.v());
  Batch bd = b_mod_drop(c, one(b), bp.level);
  Batch rest = b_sub(c, BView{bd.d, bd.level, m, bd.scale, 0}, bp.v());
  BView bpv = bp.v();
  return b_rotate_add(c, k, rest.v(), s1, &bpv);
}

// A view at `level`: the input itself, or a copy with the upper limbs dropped (kept in `hold`).
CtView at_level(Context& c, CtView x, int level, std::vector<Batch>& hold) {
  if (x.level == level) return x;
  hold.push_back(b_mod_drop(c, one(x), level));
  return hold.back().item(0);
}

}  // namespace

std::vector<int> required_rot_steps(const Context& c, int op, int cc, int s0) {
  const int s1 = c.slots / s0;
  check_block_shape(c, s0, s1);
  const int half = cc / 2;
  std::vector<int> steps;
  if (op == 0) {
    for (int k = 1; k <= half; ++k) steps.push_back(k * s1);
    for (int m = 0; (1 << m) < s1; ++m) {
      steps.push_back(1 << m);
      steps.push_back(-(1 << m));
    }
  } else if (op == 1 || op == 2) {
    for (int k = 1; k <= half; ++k) steps.push_back(k);
    steps.push_back(-s1);
    for (int m = 0; (1 << m) < s0; ++m) steps.push_back((1 << m) * s1);
    if (op == 2) steps.push_back(s1);
  } else {
    fail(HETAL_E_INVALID_ARG, "op must be 0 (ABT), 1 (ATB RotLeft) or 2 (ATB PRotUp)");
  }
  std::sort(steps.begin(), steps.end());
  steps.erase(std::unique(steps.begin(), steps.end()), steps.end());
  return steps;
}

std::vector<Cipher> to_ciphers(Context& c, const Batch& b) {
  std::vector<Cipher> out;
  for (int i = 0; i < b.count; ++i) {
    Cipher x(c, b.level);
    HCHECK(hipMemcpyAsync(x.d, b.item(i).d, c.ct_words(b.level) * 8, hipMemcpyDeviceToDevice, c.stream));
    x.scale = b.scale;
    out.push_back(std::move(x));
  }
  return out;
}

Batch diag_abt_batch(Context& c, const KeySet& k, MaskCache& mc, const std::vector<std::vector<CtView>>& A,
                     const std::vector<CtView>& Bbar, int cc, int s0, int s1, double t) {
  check_block_shape(c, s0, s1);
  if (cc < 2 || cc > s0 || s1 % cc || (cc & (cc - 1))) fail(HETAL_E_SHAPE, "need 1 < c <= s0, c a power of two dividing s1");
  const int n_a = (int)A.size(), n_b = (int)Bbar.size();
  if (n_a < 1 || n_b < 1) fail(HETAL_E_SHAPE, "empty block matrix");
  int lv = 1 << 30;
  for (auto& row : A) {
    if ((int)row.size() != n_b) fail(HETAL_E_SHAPE, "A and Bbar block columns differ");
    for (auto& x : row) lv = std::min(lv, x.level);
  }
  for (auto& x : Bbar) lv = std::min(lv, x.level);
  if (lv < 3) fail(HETAL_E_LEVEL, "DiagABT needs three levels");
  const int half = cc / 2;
  std::vector<Batch> hold;
  std::vector<std::vector<CtView>> a(n_a);
  for (int i = 0; i < n_a; ++i)
    for (int j = 0; j < n_b; ++j) a[i].push_back(at_level(c, A[i][j], lv, hold));
  std::vector<CtView> bv;
  for (int j = 0; j < n_b; ++j) bv.push_back(at_level(c, Bbar[j], lv, hold));
  Batch bp = b_pack(c, bv);

  // B_cplx = Bbar + i RU(Bbar, c/2)
  Batch rb = b_rotate(c, k, bp.v(), {half * s1});
  Batch rbi = b_mul_i(c, rb.v());
  Batch bc = b_add(c, bp.v(), rbi.v());

  // RU(B_cplx, k) for k = 1 .. c/2 - 1, hoisted per block
  std::vector<Batch> bk(n_b);
  if (half > 1) {
    std::vector<int> steps;
    for (int kk = 1; kk < half; ++kk) steps.push_back(kk * s1);
    for (int j = 0; j < n_b; ++j) bk[j] = b_rotate_hoisted(c, k, bc.item(j), steps);
  }

  // products A_ij * B_kj in the order (i, k, j): sums over j are contiguous groups
  std::vector<CtView> pa, pb;
  for (int i = 0; i < n_a; ++i)
    for (int kk = 0; kk < half; ++kk)
      for (int j = 0; j < n_b; ++j) {
        pa.push_back(a[i][j]);
        pb.push_back(kk == 0 ? bc.item(j) : bk[j].item(kk - 1));
      }
  Batch prod = b_hmult(c, k, pa, pb);
  Batch r = b_sum_groups(c, prod.v(), n_a * half);
  prod = Batch();
  r = b_rescale(c, r.v());

  r = col_sum(c, k, mc, std::move(r), s0, s1);

  std::vector<MaskSpec> masks;
  for (int i = 0; i < n_a; ++i)
    for (int kk = 0; kk < half; ++kk) masks.push_back(MaskSpec{MASK_OFFDIAG_CPLX, kk, cc, s0, s1, t});
  Batch rm = b_cmult_masks(c, mc, r.v(), masks);
  r = b_rescale(c, rm.v());
  Batch x = b_sum_groups(c, r.v(), n_a);
  return b_conj_add(c, k, x.v());
}

Batch diag_atb_batch(Context& c, const KeySet& k, MaskCache& mc, const std::vector<CtView>& Abar,
                     const std::vector<std::vector<CtView>>& B, int cc, int s0, int s1, double t) {
  check_block_shape(c, s0, s1);
  if (cc < 2 || cc > s1 || s1 % cc || (cc & (cc - 1))) fail(HETAL_E_SHAPE, "need 1 < c, c a power of two dividing s1");
  const int n_a = (int)Abar.size();
  if (n_a < 1 || (int)B.size() != n_a || B[0].empty()) fail(HETAL_E_SHAPE, "Abar and B block rows differ");
  const int n_b = (int)B[0].size();
  int lA = 1 << 30, lB = 1 << 30;
  for (auto& x : Abar) lA = std::min(lA, x.level);
  for (auto& row : B) {
    if ((int)row.size() != n_b) fail(HETAL_E_SHAPE, "ragged B");
    for (auto& x : row) lB = std::min(lB, x.level);
  }
  const bool use_pru = lA < lB;
  const int lstar = use_pru ? std::min(lA - 1, lB - 1) : std::min(lA - 2, lB);
  if (lstar < 2) fail(HETAL_E_LEVEL, "DiagATB needs more levels");
  const int half = cc / 2;
  std::vector<Batch> hold;
  std::vector<CtView> av;
  for (int i = 0; i < n_a; ++i) av.push_back(at_level(c, Abar[i], lA, hold));
  Batch ap = b_pack(c, av);
  std::vector<std::vector<CtView>> bview(n_a);
  for (int i = 0; i < n_a; ++i)
    for (int j = 0; j < n_b; ++j) bview[i].push_back(at_level(c, B[i][j], lB, hold));

  // A_cplx = Abar + i RL(Abar, c/2)
  Batch a1 = b_rotate(c, k, ap.v(), {half});
  Batch rl = rot_left_finish(c, k, mc, a1, std::vector<int>(n_a, half), s0, s1);
  Batch apd = b_mod_drop(c, ap.v(), rl.level);
  Batch rli = b_mul_i(c, rl.v());
  Batch ac = b_add(c, apd.v(), rli.v());
  a1 = Batch();

  std::vector<int> ks, steps;
  for (int kk = 1; kk < half; ++kk) {
    ks.push_back(kk);
    steps.push_back(kk);
  }
  // A_k[i][kk] and B_k[i][j][kk] at lstar
  std::vector<std::vector<CtView>> ak(n_a, std::vector<CtView>(half));
  std::vector<std::vector<std::vector<CtView>>> bk(n_a, std::vector<std::vector<CtView>>(n_b, std::vector<CtView>(half)));
  for (int i = 0; i < n_a; ++i) {
    ak[i][0] = at_level(c, ac.item(i), lstar, hold);
    if (half > 1) {
      Batch rk = b_rotate_hoisted(c, k, ac.item(i), steps);
      if (!use_pru) rk = rot_left_finish(c, k, mc, rk, ks, s0, s1);
      hold.push_back(rk.level == lstar ? std::move(rk) : b_mod_drop(c, rk.v(), lstar));
      for (int kk = 1; kk < half; ++kk) ak[i][kk] = hold.back().item(kk - 1);
    }
    for (int j = 0; j < n_b; ++j) {
      CtView bd = at_level(c, bview[i][j], lstar, hold);
      bk[i][j][0] = bd;
      if (half > 1) {
        if (use_pru) {
          Batch pr = partial_rot_up(c, k, mc, bview[i][j], ks, s0, s1);
          hold.push_back(pr.level == lstar ? std::move(pr) : b_mod_drop(c, pr.v(), lstar));
          for (int kk = 1; kk < half; ++kk) bk[i][j][kk] = hold.back().item(kk - 1);
        } else {
          for (int kk = 1; kk < half; ++kk) bk[i][j][kk] = bd;
        }
      }
    }
  }

  // products in the order (j, k, i): sums over i are contiguous groups
  std::vector<CtView> pa, pb;
  for (int j = 0; j < n_b; ++j)
    for (int kk = 0; kk < half; ++kk)
      for (int i = 0; i < n_a; ++i) {
        pa.push_back(ak[i][kk]);
        pb.push_back(bk[i][j][kk]);
      }
  Batch prod = b_hmult(c, k, pa, pb);
  Batch r = b_sum_groups(c, prod.v(), n_b * half);
  prod = Batch();
  hold.clear();
  r = b_rescale(c, r.v());

  r = row_sum(c, k, std::move(r), s0, s1);

  std::vector<MaskSpec> masks;
  for (int j = 0; j < n_b; ++j)
    for (int kk = 0; kk < half; ++kk) masks.push_back(MaskSpec{MASK_OFFDIAG_CPLX, -kk, cc, s0, s1, t});
  Batch rm = b_cmult_masks(c, mc, r.v(), masks);
  r = b_rescale(c, rm.v());
  Batch x = b_sum_groups(c, r.v(), n_b);
  return b_conj_add(c, k, x.v());
}

std::vector<Cipher> diag_abt(Context& c, const KeySet& k, MaskCache& mc, const std::vector<std::vector<CtView>>& A,
                             const std::vector<CtView>& Bbar, int cc, int s0, int s1, double t) {
  return to_ciphers(c, diag_abt_batch(c, k, mc, A, Bbar, cc, s0, s1, t));
}

std::vector<Cipher> diag_atb(Context& c, const KeySet& k, MaskCache& mc, const std::vector<CtView>& Abar,
                             const std::vector<std::vector<CtView>>& B, int cc, int s0, int s1, double t) {
  return to_ciphers(c, diag_atb_batch(c, k, mc, Abar, B, cc, s0, s1, t));
}

}  // namespace hetal
