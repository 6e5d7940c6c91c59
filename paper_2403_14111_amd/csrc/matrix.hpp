// Encrypted matrix products (DiagABT, DiagATB) on device ciphertexts.
#pragma once
#include <vector>

#include "ops.hpp"

namespace hetal {

std::vector<int> required_rot_steps(const Context& c, int op, int cc, int s0);

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
