// Seeded sampling of the client's randomness (see sampler.hip for the streams and distributions).
#pragma once
#include "hetal_internal.hpp"

namespace hetal {

constexpr u32 PURPOSE_SECRET = 1, PURPOSE_KSK_A = 2, PURPOSE_KSK_E = 3, PURPOSE_ENC_A = 4, PURPOSE_ENC_E = 5;
constexpr int GAUSS_ENTRIES = 19;   // thresholds of |x| <= 0 .. 18 (|x| <= 19 in all)
constexpr int SECRET_HAMMING = 192;  // nonzero coefficients of a sampled secret

// T_j = floor(2^63 P(|x| <= j)) for the rounded Gaussian of standard deviation 3.2 on |x| <= 19.
void gaussian_table(u64 (&out)[GAUSS_ENTRIES]);
// The ternary secret of `seed` with h nonzero coefficients (host), out[N].
void sample_ternary(u64 seed, int log_n, int h, i64* out);
// `rows` rows of uniform residues (device, [rows][N], coefficient form): row r is the stream of sub
// (r / group) * 64 + r % group, modulo the prime of index r % group.
void sample_uniform(Context& c, u64 seed, u32 purpose, u32 index, int rows, int group, u64* out);
// `count` rows of errors (device, signed, [count][N]): row r is the stream of sub r.
void sample_gaussian(Context& c, u64 seed, u32 purpose, u32 index, int count, i64* out);

}  // namespace hetal
