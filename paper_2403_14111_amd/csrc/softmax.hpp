// Constant operations and the row-wise softmax approximation (App. softmax) on device ciphertexts.
#pragma once
#include <vector>

#include "hetal.h"
#include "ops.hpp"

namespace hetal {

// round(v) (ties to even) as a signed 62-bit integer; E_OVERFLOW beyond.
i64 round_const(double v);

// x * K for the integer K = round(value * sigma) (both polynomials, every limb); scale * sigma.
Batch b_mul_const(Context& c, BView a, double value, double sigma);
// rescale(x taken at `level` (mod-dropped) times round(value sigma)), in the rescale's three launches: the same
// words as b_mod_drop, b_mul_const and b_rescale one after the other (and, with an addend, b_add(addend, that)).
Batch b_mul_const_rescale(Context& c, BView a, int level, double value, double sigma,
                          const BView* addend = nullptr);
// x + value in every slot: K = round(value * scale) added to c0's constant term (every NTT-domain word).
Batch b_add_const(Context& c, BView a, double value);
// x + pt (c0 + pt), pt at the batch's level in the NTT domain.
Batch b_add_plain(Context& c, BView a, const u64* pt);

// Refresh by the key holder: called with a ciphertext (the library's buffer, room for the top level) that it must
// replace, in place, by an encryption of the same message at the top level; the new scale is read back.
struct Refresher {
  hetal_refresh_fn fn = nullptr;
  void* user = nullptr;
  int count = 0;
};

// sum_k coeffs[k] x^k, power basis (x^k = x^a x^b, a the largest power of two below k, or k/2 twice), each product
// relinearised and rescaled; terms brought to the common level and multiplied by coeffs[k] at the scale that lands
// on x's scale; the constant term added last.  Operands below the depth needed are refreshed first.
Batch poly_eval(Context& c, const KeySet& k, BView x, const std::vector<double>& coeffs, Refresher& rf);

struct SoftmaxArgs {
  double R, L;
  int n, precise, extend, comp_g, exp_B;
  std::vector<double> exp_coeffs;  // p(x / B), degree exp_B's polynomial
  double inv_R;
  int inv_iters;
};

// Alg. "Row-wise softmax approximation" on the row blocks of a horizontally tiled a x c matrix.
Batch softmax_approx(Context& c, const KeySet& k, MaskCache& mc, BView m, int cc, int s0, int s1,
                     const SoftmaxArgs& a, Refresher& rf);

std::vector<int> softmax_rot_steps(int cc, int s1);

// One step of the encrypted training loop (NAG, Sec. 3): P = ASoftmax(X V^T) (DiagABT, then the softmax),
// W' = V - lr (P - Y)^T X (DiagATB with t = -lr), V' = (1 - gamma) W' + gamma W.  X: n_rb x n_cb untiled blocks; Y:
// n_rb one-hot blocks tiled horizontally; W, V: n_cb blocks tiled vertically.  X and V are refreshed below 3
// levels, P - Y below 4.
struct NagResult {
  Batch W, V;
};
NagResult nag_step(Context& c, const KeySet& k, MaskCache& mc, BView X, int n_rb, int n_cb, BView Y, BView W,
                   BView V, int cls, int s0, int s1, double lr, double gamma, const SoftmaxArgs& a, Refresher& rf);

// Default AExp polynomial: the L^2 projection of e^t on [-1, 1] onto degree `degree`, as monomial coefficients of
// p(x / B).
std::vector<double> default_exp_coeffs(int degree, int B);

// Client-side refresh: decrypt, lift the plaintext from q_0 (centred; E_OVERFLOW when another limb disagrees),
// re-encode it at `scale` (rint(m * scale / ct.scale); scale <= 0 keeps it), re-encrypt at the top level with the
// caller's randomness (a_ntt, e_ntt: NTT form over q_0..q_{num_q-1}).
void refresh_encrypt(Context& c, const u64* s, CtView ct, double scale, const u64* a_ntt, const u64* e_ntt,
                     u64* out);

}  // namespace hetal
