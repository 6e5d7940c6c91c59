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
  x = b_cmult_masks_rescale(c, mc, x.v(), {MaskSpec{MASK_FIRST_COL, 0, 0, s0, s1, 1.0}});
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
  Batch a2 = b_cmult_masks_rescale(c, mc, a1.v(), masks);
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
  Batch bp = b_cmult_masks_rescale(c, mc, bc, masks);
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

// The most ciphertexts at `level` that one stage of a product holds at once: the transient rotations and
// products of one chunk, and the run sums of one group of requests (the class's tuned value, else 2 GiB worth).
int work_limit(const Context& c, int level) {
  if (c.tune.work_cts > 0) return c.tune.work_cts;
  return std::max(8, (int)((size_t(2) << 30) / (c.ct_words(level) * 8)));
}

namespace {

// Consecutive requests whose sizes add up to at most `limit` (a larger one alone): [first, last) ranges.
std::vector<std::pair<int, int>> split_by_size(const std::vector<long>& sizes, long limit) {
  std::vector<std::pair<int, int>> parts;
  int first = 0;
  long used = 0;
  for (int r = 0; r < (int)sizes.size(); ++r) {
    if (r > first && used + sizes[r] > limit) {
      parts.push_back({first, r});
      first = r;
      used = 0;
    }
    used += sizes[r];
  }
  parts.push_back({first, (int)sizes.size()});
  return parts;
}

// The parts' results back to back (all at one level and scale).
Batch concat(Context& c, std::vector<Batch>& parts) {
  if (parts.size() == 1) return std::move(parts[0]);
  int total = 0;
  for (auto& p : parts) total += p.count;
  Batch o(c, parts[0].level, total);
  const size_t w = c.ct_words(o.level);
  int at = 0;
  for (auto& p : parts) {
    HCHECK(hipMemcpyAsync(o.d + (size_t)at * w, p.d, (size_t)p.count * w * 8, hipMemcpyDeviceToDevice, c.stream));
    at += p.count;
  }
  o.scale = parts[0].scale;
  return o;
}

// One slice of a request's products: a range [lo, hi) of the loop variable a chunk covers (DiagABT: k; DiagATB:
// the block column j).
struct Slice {
  int r, lo, hi;
};

// Consecutive slices of every request (unit u of request r costs cost[r] ciphertexts; units[r] of them), packed
// into chunks of at most `limit` ciphertexts (at least one unit each).
std::vector<std::vector<Slice>> chunk_slices(const std::vector<int>& units, const std::vector<long>& cost, long limit) {
  std::vector<std::vector<Slice>> chunks(1);
  long used = 0;
  for (int r = 0; r < (int)units.size(); ++r) {
    int lo = 0;
    while (lo < units[r]) {
      const long room = limit - used;
      int take = (int)std::min<long>(units[r] - lo, room / std::max(1L, cost[r]));
      if (take == 0) {
        if (used > 0) {
          chunks.emplace_back();
          used = 0;
          continue;
        }
        take = 1;
      }
      chunks.back().push_back(Slice{r, lo, lo + take});
      used += take * cost[r];
      lo += take;
    }
  }
  return chunks;
}

Batch abt_group(Context& c, const KeySet& k, MaskCache& mc, const std::vector<AbtRequest>& reqs, int cc, int s0, int s1,
                int lv) {
  const int half = cc / 2;
  std::vector<Batch> hold;
  // every request's blocks at the common level; the Bbar blocks of all requests in one batch
  std::vector<std::vector<std::vector<CtView>>> a(reqs.size());
  std::vector<CtView> bv;
  std::vector<int> boff, roff;
  int total_runs = 0;
  for (size_t r = 0; r < reqs.size(); ++r) {
    for (auto& row : reqs[r].A) {
      a[r].emplace_back();
      for (auto& x : row) a[r].back().push_back(at_level(c, x, lv, hold));
    }
    boff.push_back((int)bv.size());
    for (auto& x : reqs[r].Bbar) bv.push_back(at_level(c, x, lv, hold));
    roff.push_back(total_runs);
    total_runs += (int)reqs[r].A.size() * half;
  }
  Batch bc;
  {
    Batch bp = b_pack(c, bv);
    // B_cplx = Bbar + i RU(Bbar, c/2)
    Batch rb = b_rotate(c, k, bp.v(), {half * s1});
    Batch rbi = b_mul_i(c, rb.v());
    bc = b_add(c, bp.v(), rbi.v());
  }

  // The run sums xs[(r, i, k)] = sum over j of A_ij * RU(B_cplx, k)_j, in the order (request, i, k).  The products
  // are made a chunk of k-ranges at a time: RU(B_cplx_j, k) for the chunk's k (hoisted per block), the products,
  // and their sums over j written into place.
  Batch xs(c, lv, total_runs);
  std::vector<int> units(reqs.size(), half);
  std::vector<long> cost(reqs.size());
  for (size_t r = 0; r < reqs.size(); ++r) cost[r] = (long)reqs[r].Bbar.size() * ((long)reqs[r].A.size() + 1);
  for (const auto& chunk : chunk_slices(units, cost, work_limit(c, lv))) {
    std::vector<Batch> rot;
    std::vector<std::vector<int>> rot_at(chunk.size());  // per slice: index into rot of its block j (or -1)
    for (size_t q = 0; q < chunk.size(); ++q) {
      const Slice& sl = chunk[q];
      std::vector<int> steps;
      for (int kk = std::max(1, sl.lo); kk < sl.hi; ++kk) steps.push_back(kk * s1);
      const int n_b = (int)reqs[sl.r].Bbar.size();
      rot_at[q].assign(n_b, -1);
      if (steps.empty()) continue;
      for (int j = 0; j < n_b; ++j) {
        rot_at[q][j] = (int)rot.size();
        rot.push_back(b_rotate_hoisted(c, k, bc.item(boff[sl.r] + j), steps));
      }
    }
    std::vector<CtView> pa, pb;
    std::vector<int> runs_j, dst;
    for (size_t q = 0; q < chunk.size(); ++q) {
      const Slice& sl = chunk[q];
      const int n_b = (int)reqs[sl.r].Bbar.size();
      const int first_rot = std::max(1, sl.lo);
      for (int i = 0; i < (int)a[sl.r].size(); ++i) {
        for (int kk = sl.lo; kk < sl.hi; ++kk) {
          for (int j = 0; j < n_b; ++j) {
            pa.push_back(a[sl.r][i][j]);
            pb.push_back(kk == 0 ? bc.item(boff[sl.r] + j) : rot[rot_at[q][j]].item(kk - first_rot));
          }
          runs_j.push_back(n_b);
          dst.push_back(roff[sl.r] + i * half + kk);
        }
      }
    }
    Batch prod = b_hmult(c, k, pa, pb);
    b_sum_segments_into(c, prod.v(), runs_j, dst, xs);
  }
  bc = Batch();
  hold.clear();
  Batch x = b_rescale(c, xs.v());
  xs = Batch();

  x = col_sum(c, k, mc, std::move(x), s0, s1);

  std::vector<int> runs_k;
  std::vector<MaskSpec> masks;
  for (size_t r = 0; r < reqs.size(); ++r)
    for (size_t i = 0; i < reqs[r].A.size(); ++i) {
      for (int kk = 0; kk < half; ++kk) masks.push_back(MaskSpec{MASK_OFFDIAG_CPLX, kk, cc, s0, s1, reqs[r].t});
      runs_k.push_back(half);
    }
  x = b_cmult_masks_rescale(c, mc, x.v(), masks);
  Batch y = b_sum_segments(c, x.v(), runs_k);
  return b_conj_add(c, k, y.v());
}

Batch atb_group(Context& c, const KeySet& k, MaskCache& mc, const std::vector<AtbRequest>& reqs, int cc, int s0, int s1,
                int lA, int lB) {
  const bool use_pru = lA < lB;
  const int lstar = use_pru ? std::min(lA - 1, lB - 1) : std::min(lA - 2, lB);
  const int half = cc / 2;
  std::vector<Batch> hold;
  // the Abar blocks of all requests in one batch
  std::vector<CtView> av;
  std::vector<int> aoff, roff;
  int total_runs = 0;
  for (const AtbRequest& r : reqs) {
    aoff.push_back((int)av.size());
    for (auto& x : r.Abar) av.push_back(at_level(c, x, lA, hold));
    roff.push_back(total_runs);
    total_runs += (int)r.B[0].size() * half;
  }
  Batch ac;
  {
    Batch ap = b_pack(c, av);
    // A_cplx = Abar + i RL(Abar, c/2)
    Batch a1 = b_rotate(c, k, ap.v(), {half});
    Batch rl = rot_left_finish(c, k, mc, a1, std::vector<int>(av.size(), half), s0, s1);
    Batch apd = b_mod_drop(c, ap.v(), rl.level);
    Batch rli = b_mul_i(c, rl.v());
    ac = b_add(c, apd.v(), rli.v());
  }

  std::vector<int> ks, steps;
  for (int kk = 1; kk < half; ++kk) {
    ks.push_back(kk);
    steps.push_back(kk);
  }
  // per request: A_k[i][kk] at lstar (RotLeft of A_cplx by k, hoisted per block)
  std::vector<std::vector<std::vector<CtView>>> ak(reqs.size());
  for (size_t r = 0; r < reqs.size(); ++r) {
    const int n_a = (int)reqs[r].Abar.size();
    ak[r].assign(n_a, std::vector<CtView>(half));
    for (int i = 0; i < n_a; ++i) {
      const CtView aci = ac.item(aoff[r] + i);
      ak[r][i][0] = at_level(c, aci, lstar, hold);
      if (half > 1) {
        Batch rk = b_rotate_hoisted(c, k, aci, steps);
        if (!use_pru) rk = rot_left_finish(c, k, mc, rk, ks, s0, s1);
        hold.push_back(rk.level == lstar ? std::move(rk) : b_mod_drop(c, rk.v(), lstar));
        for (int kk = 1; kk < half; ++kk) ak[r][i][kk] = hold.back().item(kk - 1);
      }
    }
  }

  // The run sums xs[(r, j, k)] = sum over i of A_k[i] * B_k[i][j], in the order (request, j, k), made a chunk of
  // block columns j at a time: B_k[i][j] for the chunk's j (PRotUp, or B itself on the RotLeft branch), the
  // products, and their sums over i written into place.
  Batch xs(c, lstar, total_runs);
  std::vector<int> units(reqs.size());
  std::vector<long> cost(reqs.size());
  for (size_t r = 0; r < reqs.size(); ++r) {
    units[r] = (int)reqs[r].B[0].size();
    cost[r] = (long)reqs[r].Abar.size() * (half + (use_pru ? 2L * (half - 1) + 2 : 2));
  }
  for (const auto& chunk : chunk_slices(units, cost, work_limit(c, lstar))) {
    std::vector<Batch> held;
    std::vector<CtView> pa, pb;
    std::vector<int> runs_i, dst;
    for (const Slice& sl : chunk) {
      const AtbRequest& rq = reqs[sl.r];
      const int n_a = (int)rq.Abar.size();
      for (int j = sl.lo; j < sl.hi; ++j) {
        std::vector<std::vector<CtView>> bk(n_a, std::vector<CtView>(half));
        for (int i = 0; i < n_a; ++i) {
          const CtView bij = at_level(c, rq.B[i][j], lB, held);
          const CtView bd = at_level(c, bij, lstar, held);
          bk[i][0] = bd;
          if (half > 1) {
            if (use_pru) {
              Batch pr = partial_rot_up(c, k, mc, bij, ks, s0, s1);
              held.push_back(pr.level == lstar ? std::move(pr) : b_mod_drop(c, pr.v(), lstar));
              for (int kk = 1; kk < half; ++kk) bk[i][kk] = held.back().item(kk - 1);
            } else {
              for (int kk = 1; kk < half; ++kk) bk[i][kk] = bd;
            }
          }
        }
        for (int kk = 0; kk < half; ++kk) {
          for (int i = 0; i < n_a; ++i) {
            pa.push_back(ak[sl.r][i][kk]);
            pb.push_back(bk[i][kk]);
          }
          runs_i.push_back(n_a);
          dst.push_back(roff[sl.r] + j * half + kk);
        }
      }
    }
    Batch prod = b_hmult(c, k, pa, pb);
    b_sum_segments_into(c, prod.v(), runs_i, dst, xs);
  }
  hold.clear();
  ac = Batch();
  Batch x = b_rescale(c, xs.v());
  xs = Batch();

  x = row_sum(c, k, std::move(x), s0, s1);

  std::vector<int> runs_k;
  std::vector<MaskSpec> masks;
  for (size_t r = 0; r < reqs.size(); ++r)
    for (size_t j = 0; j < reqs[r].B[0].size(); ++j) {
      for (int kk = 0; kk < half; ++kk) masks.push_back(MaskSpec{MASK_OFFDIAG_CPLX, -kk, cc, s0, s1, reqs[r].t});
      runs_k.push_back(half);
    }
  x = b_cmult_masks_rescale(c, mc, x.v(), masks);
  Batch y = b_sum_segments(c, x.v(), runs_k);
  return b_conj_add(c, k, y.v());
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
  // requests in lockstep while their run sums fit the working-set limit
  std::vector<long> runs;
  for (const AbtRequest& r : reqs) runs.push_back((long)r.A.size() * (cc / 2));
  std::vector<Batch> parts;
  for (auto [first, last] : split_by_size(runs, work_limit(c, lv)))
    parts.push_back(abt_group(c, k, mc, std::vector<AbtRequest>(reqs.begin() + first, reqs.begin() + last), cc, s0,
                              s1, lv));
  return concat(c, parts);
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
  // requests in lockstep while their run sums and rotated A blocks fit the working-set limit
  std::vector<long> size;
  for (const AtbRequest& r : reqs) size.push_back(((long)r.B[0].size() + (long)r.Abar.size()) * (cc / 2));
  std::vector<Batch> parts;
  for (auto [first, last] : split_by_size(size, work_limit(c, lstar)))
    parts.push_back(atb_group(c, k, mc, std::vector<AtbRequest>(reqs.begin() + first, reqs.begin() + last), cc, s0,
                              s1, lA, lB));
  return concat(c, parts);
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
