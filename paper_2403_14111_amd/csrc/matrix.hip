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
// Every step runs as device kernels; the sequence of rounding operations
// (key switches, rescales) is fixed by the algorithm, so reordering
// independent work cannot change a single bit of the result.
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

Cipher col_sum(Context& c, const KeySet& k, MaskCache& mc, Cipher x, int s0, int s1) {
  const int lg = log2_exact(s1, "s1");
  for (int m = 0; m < lg; ++m) {
    Cipher r = rotate(c, k, view(x), 1 << m);
    x = add(c, view(x), view(r));
  }
  Cipher masked = cmult_mask(c, mc, view(x), MASK_FIRST_COL, 0, 0, s0, s1, 1.0);
  x = rescale(c, view(masked));
  for (int m = 0; m < lg; ++m) {
    Cipher r = rotate(c, k, view(x), -(1 << m));
    x = add(c, view(x), view(r));
  }
  return x;
}

Cipher row_sum(Context& c, const KeySet& k, Cipher x, int s0, int s1) {
  const int lg = log2_exact(s0, "s0");
  for (int m = 0; m < lg; ++m) {
    Cipher r = rotate(c, k, view(x), (1 << m) * s1);
    x = add(c, view(x), view(r));
  }
  return x;
}

// RL(A, k) (Alg. 2): columns rotated left by k within each row; one level.
Cipher rot_left_cols(Context& c, const KeySet& k, MaskCache& mc, CtView a, int kk, int s0, int s1) {
  Cipher a1 = rotate(c, k, a, kk);
  Cipher a2m = cmult_mask(c, mc, view(a1), MASK_LEFT_COLS, kk, 0, s0, s1, 1.0);
  Cipher a2 = rescale(c, view(a2m));
  Cipher a1d = mod_drop(c, view(a1), a2.level);
  Cipher rest = sub(c, view(a1d), view(a2));
  Cipher back = rotate(c, k, view(rest), -s1);
  return add(c, view(a2), view(back));
}

// PRU(B, k) (Alg. 3): the last k columns move up by one row; one level.
Cipher partial_rot_up(Context& c, const KeySet& k, MaskCache& mc, CtView b, int kk, int s0, int s1) {
  Cipher bpm = cmult_mask(c, mc, b, MASK_LEFT_COLS, kk, 0, s0, s1, 1.0);
  Cipher bp = rescale(c, view(bpm));
  Cipher bd = mod_drop(c, b, bp.level);
  Cipher rest = sub(c, view(bd), view(bp));
  Cipher up = rotate(c, k, view(rest), s1);
  return add(c, view(bp), view(up));
}

void check_block_shape(const Context& c, int s0, int s1) {
  if (s0 < 1 || s1 < 1 || (long)s0 * s1 != c.slots) fail(HETAL_E_SHAPE, "s0 * s1 must equal the slot count N/2");
  log2_exact(s0, "s0");
  log2_exact(s1, "s1");
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

std::vector<Cipher> diag_abt(Context& c, const KeySet& k, MaskCache& mc, const std::vector<std::vector<CtView>>& A,
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
  std::vector<std::vector<Cipher>> a(n_a);
  for (int i = 0; i < n_a; ++i)
    for (int j = 0; j < n_b; ++j) a[i].push_back(mod_drop(c, A[i][j], lv));
  std::vector<Cipher> bc;
  for (int j = 0; j < n_b; ++j) {
    Cipher b = mod_drop(c, Bbar[j], lv);
    Cipher r = rotate(c, k, view(b), half * s1);
    Cipher ri = mul_i(c, view(r));
    bc.push_back(add(c, view(b), view(ri)));
  }
  std::vector<Cipher> X(n_a);
  for (int kk = 0; kk < half; ++kk) {
    std::vector<Cipher> bk;
    if (kk > 0)
      for (int j = 0; j < n_b; ++j) bk.push_back(rotate(c, k, view(bc[j]), kk * s1));
    for (int i = 0; i < n_a; ++i) {
      Cipher r;
      for (int j = 0; j < n_b; ++j) {
        Cipher p = hmult(c, k, view(a[i][j]), kk == 0 ? view(bc[j]) : view(bk[j]));
        r = j == 0 ? std::move(p) : add(c, view(r), view(p));
      }
      r = rescale(c, view(r));
      r = col_sum(c, k, mc, std::move(r), s0, s1);
      Cipher rm = cmult_mask(c, mc, view(r), MASK_OFFDIAG_CPLX, kk, cc, s0, s1, t);
      r = rescale(c, view(rm));
      X[i] = kk == 0 ? std::move(r) : add(c, view(X[i]), view(r));
    }
  }
  std::vector<Cipher> out;
  for (int i = 0; i < n_a; ++i) {
    Cipher cj = conjugate(c, k, view(X[i]));
    out.push_back(add(c, view(X[i]), view(cj)));
  }
  return out;
}

std::vector<Cipher> diag_atb(Context& c, const KeySet& k, MaskCache& mc, const std::vector<CtView>& Abar,
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
  std::vector<Cipher> ac;
  for (int i = 0; i < n_a; ++i) {
    Cipher a = mod_drop(c, Abar[i], lA);
    Cipher rl = rot_left_cols(c, k, mc, view(a), half, s0, s1);
    Cipher ad = mod_drop(c, view(a), rl.level);
    Cipher rli = mul_i(c, view(rl));
    ac.push_back(add(c, view(ad), view(rli)));
  }
  std::vector<std::vector<Cipher>> bd(n_a);
  for (int i = 0; i < n_a; ++i)
    for (int j = 0; j < n_b; ++j) bd[i].push_back(mod_drop(c, B[i][j], lB));
  std::vector<Cipher> X(n_b);
  for (int kk = 0; kk < half; ++kk) {
    std::vector<Cipher> ak;
    std::vector<std::vector<Cipher>> bk(n_a);
    for (int i = 0; i < n_a; ++i) {
      if (use_pru) {
        if (kk == 0) ak.push_back(mod_drop(c, view(ac[i]), lstar));
        else {
          Cipher r = rotate(c, k, view(ac[i]), kk);
          ak.push_back(mod_drop(c, view(r), lstar));
        }
        for (int j = 0; j < n_b; ++j) {
          if (kk == 0) bk[i].push_back(mod_drop(c, view(bd[i][j]), lstar));
          else {
            Cipher p = partial_rot_up(c, k, mc, view(bd[i][j]), kk, s0, s1);
            bk[i].push_back(mod_drop(c, view(p), lstar));
          }
        }
      } else {
        if (kk == 0) ak.push_back(mod_drop(c, view(ac[i]), lstar));
        else {
          Cipher r = rot_left_cols(c, k, mc, view(ac[i]), kk, s0, s1);
          ak.push_back(mod_drop(c, view(r), lstar));
        }
        for (int j = 0; j < n_b; ++j) bk[i].push_back(mod_drop(c, view(bd[i][j]), lstar));
      }
    }
    for (int j = 0; j < n_b; ++j) {
      Cipher r;
      for (int i = 0; i < n_a; ++i) {
        Cipher p = hmult(c, k, view(ak[i]), view(bk[i][j]));
        r = i == 0 ? std::move(p) : add(c, view(r), view(p));
      }
      r = rescale(c, view(r));
      r = row_sum(c, k, std::move(r), s0, s1);
      Cipher rm = cmult_mask(c, mc, view(r), MASK_OFFDIAG_CPLX, -kk, cc, s0, s1, t);
      r = rescale(c, view(rm));
      X[j] = kk == 0 ? std::move(r) : add(c, view(X[j]), view(r));
    }
  }
  std::vector<Cipher> out;
  for (int j = 0; j < n_b; ++j) {
    Cipher cj = conjugate(c, k, view(X[j]));
    out.push_back(add(c, view(X[j]), view(cj)));
  }
  return out;
}

}  // namespace hetal
