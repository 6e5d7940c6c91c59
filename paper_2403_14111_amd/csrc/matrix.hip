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

namespace {

int common_level(std::initializer_list<const std::vector<CtView>*> parts) {
  int lv = 1 << 30;
  for (auto* v : parts)
    for (auto& x : *v) lv = std::min(lv, x.level);
  return lv;
}

}  // namespace

Batch diag_abt_multi(Context& c, const KeySet& k, MaskCache& mc, const std::vector<AbtRequest>& reqs, int cc, int s0,
                     int s1) {
  check_block_shape(c, s0, s1);
  if (cc < 2 || cc > s0 || s1 % cc || (cc & (cc - 1))) fail(HETAL_E_SHAPE, "need 1 < c <= s0, c a power of two dividing s1");
  if (reqs.empty()) fail(HETAL_E_INVALID_ARG, "no requests");
  int lv = -1;
  for (const AbtRequest& r : reqs) {
    const int n_a = (int)r.A.size(), n_b = (int)r.Bbar.size();
    if (n_a < 1 || n_b < 1) fail(HETAL_E_SHAPE, "empty block matrix");
    int l = common_level({&r.Bbar});
    for (auto& row : r.A) {
      if ((int)row.size() != n_b) fail(HETAL_E_SHAPE, "A and Bbar block columns differ");
      l = std::min(l, common_level({&row}));
    }
    if (lv >= 0 && l != lv) fail(HETAL_E_LEVEL, "requests in one lockstep group at different levels");
    lv = l;
  }
  if (lv < 3) fail(HETAL_E_LEVEL, "DiagABT needs three levels");
  const int half = cc / 2;
  std::vector<Batch> hold;
  // every request's blocks at the common level; the Bbar blocks of all requests in one batch
  std::vector<std::vector<std::vector<CtView>>> a(reqs.size());
  std::vector<CtView> bv;
  std::vector<int> boff;
  for (size_t r = 0; r < reqs.size(); ++r) {
    for (auto& row : reqs[r].A) {
      a[r].emplace_back();
      for (auto& x : row) a[r].back().push_back(at_level(c, x, lv, hold));
    }
    boff.push_back((int)bv.size());
    for (auto& x : reqs[r].Bbar) bv.push_back(at_level(c, x, lv, hold));
  }
  Batch bp = b_pack(c, bv);

  // B_cplx = Bbar + i RU(Bbar, c/2)
  Batch rb = b_rotate(c, k, bp.v(), {half * s1});
  Batch rbi = b_mul_i(c, rb.v());
  Batch bc = b_add(c, bp.v(), rbi.v());

  // RU(B_cplx, k) for k = 1 .. c/2 - 1, hoisted per block
  std::vector<Batch> bk(bv.size());
  if (half > 1) {
    std::vector<int> steps;
    for (int kk = 1; kk < half; ++kk) steps.push_back(kk * s1);
    for (size_t g = 0; g < bv.size(); ++g) bk[g] = b_rotate_hoisted(c, k, bc.item((int)g), steps);
  }

  // products A_ij * B_kj in the order (request, i, k, j): each sum over j is a contiguous run
  std::vector<CtView> pa, pb;
  std::vector<int> runs_j, runs_k;
  std::vector<MaskSpec> masks;
  for (size_t r = 0; r < reqs.size(); ++r) {
    const int n_b = (int)reqs[r].Bbar.size();
    for (auto& row : a[r]) {
      for (int kk = 0; kk < half; ++kk) {
        for (int j = 0; j < n_b; ++j) {
          pa.push_back(row[j]);
          pb.push_back(kk == 0 ? bc.item(boff[r] + j) : bk[boff[r] + j].item(kk - 1));
        }
        runs_j.push_back(n_b);
        masks.push_back(MaskSpec{MASK_OFFDIAG_CPLX, kk, cc, s0, s1, reqs[r].t});
      }
      runs_k.push_back(half);
    }
  }
  Batch prod = b_hmult(c, k, pa, pb);
  Batch x = b_sum_segments(c, prod.v(), runs_j);
  prod = Batch();
  x = b_rescale(c, x.v());

  x = col_sum(c, k, mc, std::move(x), s0, s1);

  Batch xm = b_cmult_masks(c, mc, x.v(), masks);
  x = b_rescale(c, xm.v());
  Batch y = b_sum_segments(c, x.v(), runs_k);
  return b_conj_add(c, k, y.v());
}

Batch diag_abt_batch(Context& c, const KeySet& k, MaskCache& mc, const std::vector<std::vector<CtView>>& A,
                     const std::vector<CtView>& Bbar, int cc, int s0, int s1, double t) {
  return diag_abt_multi(c, k, mc, {AbtRequest{A, Bbar, t}}, cc, s0, s1);
}

Batch diag_atb_multi(Context& c, const KeySet& k, MaskCache& mc, const std::vector<AtbRequest>& reqs, int cc, int s0,
                     int s1) {
  check_block_shape(c, s0, s1);
  if (cc < 2 || cc > s1 || s1 % cc || (cc & (cc - 1))) fail(HETAL_E_SHAPE, "need 1 < c, c a power of two dividing s1");
  if (reqs.empty()) fail(HETAL_E_INVALID_ARG, "no requests");
  int lA = -1, lB = -1;
  for (const AtbRequest& r : reqs) {
    const int n_a = (int)r.Abar.size();
    if (n_a < 1 || (int)r.B.size() != n_a || r.B[0].empty()) fail(HETAL_E_SHAPE, "Abar and B block rows differ");
    const int n_b = (int)r.B[0].size();
    const int la = common_level({&r.Abar});
    int lb = 1 << 30;
    for (auto& row : r.B) {
      if ((int)row.size() != n_b) fail(HETAL_E_SHAPE, "ragged B");
      lb = std::min(lb, common_level({&row}));
    }
    if (lA >= 0 && (la != lA || lb != lB)) fail(HETAL_E_LEVEL, "requests in one lockstep group at different levels");
    lA = la;
    lB = lb;
  }
  const bool use_pru = lA < lB;
  const int lstar = use_pru ? std::min(lA - 1, lB - 1) : std::min(lA - 2, lB);
  if (lstar < 2) fail(HETAL_E_LEVEL, "DiagATB needs more levels");
  const int half = cc / 2;
  std::vector<Batch> hold;
  // the Abar blocks of all requests in one batch
  std::vector<CtView> av;
  std::vector<int> aoff;
  for (const AtbRequest& r : reqs) {
    aoff.push_back((int)av.size());
    for (auto& x : r.Abar) av.push_back(at_level(c, x, lA, hold));
  }
  Batch ap = b_pack(c, av);

  // A_cplx = Abar + i RL(Abar, c/2)
  Batch a1 = b_rotate(c, k, ap.v(), {half});
  Batch rl = rot_left_finish(c, k, mc, a1, std::vector<int>(av.size(), half), s0, s1);
  Batch apd = b_mod_drop(c, ap.v(), rl.level);
  Batch rli = b_mul_i(c, rl.v());
  Batch ac = b_add(c, apd.v(), rli.v());
  a1 = Batch();

  std::vector<int> ks, steps;
  for (int kk = 1; kk < half; ++kk) {
    ks.push_back(kk);
    steps.push_back(kk);
  }
  // per request: A_k[i][kk] and B_k[i][j][kk] at lstar
  std::vector<std::vector<std::vector<CtView>>> ak(reqs.size());
  std::vector<std::vector<std::vector<std::vector<CtView>>>> bk(reqs.size());
  for (size_t r = 0; r < reqs.size(); ++r) {
    const int n_a = (int)reqs[r].Abar.size(), n_b = (int)reqs[r].B[0].size();
    ak[r].assign(n_a, std::vector<CtView>(half));
    bk[r].assign(n_a, std::vector<std::vector<CtView>>(n_b, std::vector<CtView>(half)));
    for (int i = 0; i < n_a; ++i) {
      const CtView aci = ac.item(aoff[r] + i);
      ak[r][i][0] = at_level(c, aci, lstar, hold);
      if (half > 1) {
        Batch rk = b_rotate_hoisted(c, k, aci, steps);
        if (!use_pru) rk = rot_left_finish(c, k, mc, rk, ks, s0, s1);
        hold.push_back(rk.level == lstar ? std::move(rk) : b_mod_drop(c, rk.v(), lstar));
        for (int kk = 1; kk < half; ++kk) ak[r][i][kk] = hold.back().item(kk - 1);
      }
      for (int j = 0; j < n_b; ++j) {
        const CtView bij = at_level(c, reqs[r].B[i][j], lB, hold);
        const CtView bd = at_level(c, bij, lstar, hold);
        bk[r][i][j][0] = bd;
        if (half > 1) {
          if (use_pru) {
            Batch pr = partial_rot_up(c, k, mc, bij, ks, s0, s1);
            hold.push_back(pr.level == lstar ? std::move(pr) : b_mod_drop(c, pr.v(), lstar));
            for (int kk = 1; kk < half; ++kk) bk[r][i][j][kk] = hold.back().item(kk - 1);
          } else {
            for (int kk = 1; kk < half; ++kk) bk[r][i][j][kk] = bd;
          }
        }
      }
    }
  }

  // products in the order (request, j, k, i): each sum over i is a contiguous run
  std::vector<CtView> pa, pb;
  std::vector<int> runs_i, runs_k;
  std::vector<MaskSpec> masks;
  for (size_t r = 0; r < reqs.size(); ++r) {
    const int n_a = (int)reqs[r].Abar.size(), n_b = (int)reqs[r].B[0].size();
    for (int j = 0; j < n_b; ++j) {
      for (int kk = 0; kk < half; ++kk) {
        for (int i = 0; i < n_a; ++i) {
          pa.push_back(ak[r][i][kk]);
          pb.push_back(bk[r][i][j][kk]);
        }
        runs_i.push_back(n_a);
        masks.push_back(MaskSpec{MASK_OFFDIAG_CPLX, -kk, cc, s0, s1, reqs[r].t});
      }
      runs_k.push_back(half);
    }
  }
  Batch prod = b_hmult(c, k, pa, pb);
  Batch x = b_sum_segments(c, prod.v(), runs_i);
  prod = Batch();
  hold.clear();
  x = b_rescale(c, x.v());

  x = row_sum(c, k, std::move(x), s0, s1);

  Batch xm = b_cmult_masks(c, mc, x.v(), masks);
  x = b_rescale(c, xm.v());
  Batch y = b_sum_segments(c, x.v(), runs_k);
  return b_conj_add(c, k, y.v());
}

Batch diag_atb_batch(Context& c, const KeySet& k, MaskCache& mc, const std::vector<CtView>& Abar,
                     const std::vector<std::vector<CtView>>& B, int cc, int s0, int s1, double t) {
  return diag_atb_multi(c, k, mc, {AtbRequest{Abar, B, t}}, cc, s0, s1);
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
