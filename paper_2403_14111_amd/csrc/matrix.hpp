// Encrypted matrix products (DiagABT, DiagATB) on device ciphertexts.
#pragma once
#include <vector>

#include "ops.hpp"

namespace hetal {

std::vector<int> required_rot_steps(const Context& c, int op, int cc, int s0);

// The most ciphertexts at `level` that one stage of DiagABT / DiagATB holds at once (Tune::work_cts, else 2 GiB
// worth): the products are made in chunks of this size and summed into place, and a lockstep group whose run
// sums exceed it runs as consecutive smaller groups.  Results do not depend on it.
int work_limit(const Context& c, int level);

// One product of a lockstep group: DiagABT <t A Bbar^T> (A: n_a x n_b blocks, Bbar: n_b blocks) or DiagATB
// <t Abar^T B> (Abar: n_a blocks, B: n_a x n_b blocks).
struct AbtRequest {
  std::vector<std::vector<CtView>> A;
  std::vector<CtView> Bbar;
  double t;
};
struct AtbRequest {
  std::vector<CtView> Abar;
  std::vector<std::vector<CtView>> B;
  double t;
};

// Several products that share (c, s0, s1), their input levels and scales, run in lockstep: every step of the
// algorithm is one batched operation over all requests' ciphertexts (rotations by one step share the key), and
// each ciphertext goes through exactly the operations of its own product, so every result is bit-identical to
// the product computed alone.  Result: the requests' output blocks back to back, in request order.
Batch diag_abt_multi(Context& c, const KeySet& k, MaskCache& mc, const std::vector<AbtRequest>& reqs, int cc, int s0,
                     int s1);
Batch diag_atb_multi(Context& c, const KeySet& k, MaskCache& mc, const std::vector<AtbRequest>& reqs, int cc, int s0,
                     int s1);

// Batched forms: the result blocks packed in one batch.
Batch diag_abt_batch(Context& c, const KeySet& k, MaskCache& mc, const std::vector<std::vector<CtView>>& A,
                     const std::vector<CtView>& Bbar, int cc, int s0, int s1, double t);
Batch diag_atb_batch(Context& c, const KeySet& k, MaskCache& mc, const std::vector<CtView>& Abar,
                     const std::vector<std::vector<CtView>>& B, int cc, int s0, int s1, double t);

// A: n_a x n_b blocks, Bbar: n_b blocks.  Returns n_a blocks.
std::vector<Cipher> diag_abt(Context& c, const KeySet& k, MaskCache& mc, const std::vector<std::vector<CtView>>& A,
                             const std::vector<CtView>& Bbar, int cc, int s0, int s1, double t);
// Abar: n_a blocks (one block column), B: n_a x n_b blocks.  Returns n_b blocks.
std::vector<Cipher> diag_atb(Context& c, const KeySet& k, MaskCache& mc, const std::vector<CtView>& Abar,
                             const std::vector<std::vector<CtView>>& B, int cc, int s0, int s1, double t);

}  // namespace hetal
