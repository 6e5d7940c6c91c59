// Seeded sampling of the client's randomness (Sec. 3.1: the client generates the secret key and the public
// operation keys, and encrypts): a counter-based generator, so that every word of every stream can be drawn by
// its own thread, and the three distributions the scheme uses.
//
//  * Generator: the ChaCha20 block function of RFC 8439 (four constants, a 256-bit key, a 32-bit block counter
//    and a 96-bit nonce; ten double rounds of quarter rounds on the columns and the diagonals; the input state
//    added back).  Stream (seed, purpose, index, sub): key = the 64-bit seed, low word first, then zeros;
//    nonce = (purpose, index, sub); counter = block number.  Word p of the stream is the little-endian 64-bit
//    word p mod 8 of block p / 8.
//  * Uniform residues modulo q (coefficient k): the first of words k, N + k, 2N + k, ... below
//    floor(2^64 / q) q, reduced modulo q.
//  * Errors: the rounded Gaussian of standard deviation 3.2 on |x| <= 19, coefficient k from word k: the top
//    bit is the sign, the low 63 bits u give the magnitude #{j < 19 : T_j <= u} for the cumulative thresholds
//    T_j = floor(2^63 P(|x| <= j)) (gaussian_table, computed in double-double arithmetic).
//  * The secret: ternary with exactly h nonzero coefficients: word p names position (w mod N) and sign (top
//    bit), taken in order, skipping positions already set.
//  * Purposes: secret 1; switching key masks 2 (index = key id: 0 for relinearisation, else the Galois element;
//    sub = digit * 64 + prime) and errors 3 (sub = digit); encryption masks 4 (index = the encryption's number,
//    sub = prime) and errors 5 (sub = 0).
#include <cmath>
#include <vector>

#include "sampler.hpp"

namespace hetal {

namespace {

constexpr int STPB = 128;

__host__ __device__ inline u32 rotl32(u32 v, int c) { return (v << c) | (v >> (32 - c)); }

__host__ __device__ inline void qround(u32& a, u32& b, u32& c, u32& d) {
  a += b; d ^= a; d = rotl32(d, 16);
  c += d; b ^= c; b = rotl32(b, 12);
  a += b; d ^= a; d = rotl32(d, 8);
  c += d; b ^= c; b = rotl32(b, 7);
}

// The 16 words of block `counter` of stream (seed, nonce).
__host__ __device__ inline void chacha_block(u64 seed, u32 counter, u32 n0, u32 n1, u32 n2, u32 (&out)[16]) {
  const u32 init[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, (u32)seed, (u32)(seed >> 32), 0u, 0u,
                        0u, 0u, 0u, 0u, counter, n0, n1, n2};
  u32 x[16];
  for (int i = 0; i < 16; ++i) x[i] = init[i];
  for (int r = 0; r < 10; ++r) {
    qround(x[0], x[4], x[8], x[12]);
    qround(x[1], x[5], x[9], x[13]);
    qround(x[2], x[6], x[10], x[14]);
    qround(x[3], x[7], x[11], x[15]);
    qround(x[0], x[5], x[10], x[15]);
    qround(x[1], x[6], x[11], x[12]);
    qround(x[2], x[7], x[8], x[13]);
    qround(x[3], x[4], x[9], x[14]);
  }
  for (int i = 0; i < 16; ++i) out[i] = x[i] + init[i];
}

__host__ __device__ inline u64 stream_word(u64 seed, u32 purpose, u32 index, u32 sub, u64 p) {
  u32 blk[16];
  chacha_block(seed, (u32)(p >> 3), purpose, index, sub, blk);
  const int w = (int)(p & 7);
  return (u64)blk[2 * w] | ((u64)blk[2 * w + 1] << 32);
}

// Rows r of `rows` streams: sub = (r / group) * 64 + r % group, prime = primes[r % group].  Each thread draws one
// block (8 coefficients) of layer 0 and redraws the rejected ones from the later layers.
__global__ void __launch_bounds__(STPB) uniform_kernel(u64 seed, u32 purpose, u32 index, int group,
                                                      const ModInfo* __restrict__ mods, u64* __restrict__ out,
                                                      int log_n) {
  const u64 n = 1ull << log_n;
  const u64 blk = (u64)blockIdx.x * STPB + threadIdx.x;
  const int r = blockIdx.y;
  const int t = r % group;
  const u32 sub = (u32)((r / group) * 64 + t);
  const u64 q = mods[t].q;
  const u64 bound = (~0ull / q) * q;  // floor(2^64 / q) q: q is odd, so it does not divide 2^64
  u32 w32[16];
  chacha_block(seed, (u32)blk, purpose, index, sub, w32);
  u64* __restrict__ o = out + (size_t)r * n;
  for (int i = 0; i < 8; ++i) {
    const u64 k = blk * 8 + i;
    u64 w = (u64)w32[2 * i] | ((u64)w32[2 * i + 1] << 32);
    for (u64 layer = 1; w >= bound; ++layer) w = stream_word(seed, purpose, index, sub, layer * n + k);
    o[k] = w % q;
  }
}

// `count` streams of errors, stream r at sub = r, written as signed coefficients [count][N].
__global__ void __launch_bounds__(STPB) gaussian_kernel(u64 seed, u32 purpose, u32 index,
                                                       const u64* __restrict__ table, i64* __restrict__ out,
                                                       int log_n) {
  const u64 n = 1ull << log_n;
  const u64 blk = (u64)blockIdx.x * STPB + threadIdx.x;
  const int r = blockIdx.y;
  u32 w32[16];
  chacha_block(seed, (u32)blk, purpose, index, (u32)r, w32);
  i64* __restrict__ o = out + (size_t)r * n;
  for (int i = 0; i < 8; ++i) {
    const u64 w = (u64)w32[2 * i] | ((u64)w32[2 * i + 1] << 32);
    const u64 u = w & 0x7fffffffffffffffull;
    i64 mag = 0;
    for (int j = 0; j < GAUSS_ENTRIES; ++j) mag += table[j] <= u ? 1 : 0;
    o[blk * 8 + i] = (w >> 63) ? -mag : mag;
  }
}

// ---- double-double arithmetic for the table (Dekker / Knuth error-free transforms)
struct DD {
  double hi, lo;
};
DD two_sum(double a, double b) {
  const double s = a + b, bb = s - a;
  return DD{s, (a - (s - bb)) + (b - bb)};
}
DD dd_add(DD a, DD b) {
  DD s = two_sum(a.hi, b.hi);
  const double lo = s.lo + a.lo + b.lo;
  return two_sum(s.hi, lo);
}
DD dd_mul(DD a, DD b) {
  const double p = a.hi * b.hi;
  const double e = std::fma(a.hi, b.hi, -p);
  return two_sum(p, e + (a.hi * b.lo + a.lo * b.hi));
}
DD dd_div(DD a, DD b) {
  const double q1 = a.hi / b.hi;
  DD r = dd_add(a, dd_mul(DD{-q1, 0.0}, b));
  const double q2 = r.hi / b.hi;
  r = dd_add(r, dd_mul(DD{-q2, 0.0}, b));
  const double q3 = r.hi / b.hi;
  return dd_add(two_sum(q1, q2), DD{q3, 0.0});
}

}  // namespace

void gaussian_table(u64 (&out)[GAUSS_ENTRIES]) {
  // rho(i) = exp(-i^2 / (2 sigma^2)) = r^(i^2), r = exp(-25/512) (2 sigma^2 = 512/25 for sigma = 3.2): r by its
  // Taylor series (terms below 2^-110 dropped), the powers by products.  About 60 double-double operations in
  // all, each exact to about 2^-104 relative, so every threshold below is within 2^-30 of its true value.
  const double x = 25.0 / 512.0;  // exact
  DD r{1.0, 0.0}, term{1.0, 0.0};
  for (int k = 1; k < 30; ++k) {
    term = dd_div(dd_mul(term, DD{-x, 0.0}), DD{(double)k, 0.0});
    r = dd_add(r, term);
  }
  const DD r2 = dd_mul(r, r);
  DD rho[GAUSS_ENTRIES + 1];
  rho[0] = DD{1.0, 0.0};
  DD step = r;  // r^(2i - 1) for i = 1, 2, ...
  for (int i = 1; i <= GAUSS_ENTRIES; ++i) {
    rho[i] = dd_mul(rho[i - 1], step);
    step = dd_mul(step, r2);
  }
  DD total = rho[0];
  for (int i = 1; i <= GAUSS_ENTRIES; ++i) total = dd_add(total, dd_mul(DD{2.0, 0.0}, rho[i]));
  DD acc = rho[0];
  for (int j = 0; j < GAUSS_ENTRIES; ++j) {
    DD v = dd_div(acc, total);
    v.hi *= 9223372036854775808.0;  // 2^63, exact
    v.lo *= 9223372036854775808.0;
    // v.hi >= 2^59 is an integer: the fraction is in v.lo
    const double fl = std::floor(v.lo);
    const double frac = v.lo - fl;
    if (!(frac > 0x1p-20 && frac < 1.0 - 0x1p-20)) fail(HETAL_E_DEVICE, "Gaussian threshold too close to an integer");
    out[j] = (u64)v.hi + (u64)(i64)fl;
    acc = dd_add(acc, dd_mul(DD{2.0, 0.0}, rho[j + 1]));
  }
}

void sample_ternary(u64 seed, int log_n, int h, i64* out) {
  const u64 n = 1ull << log_n;
  if ((u64)h > n) fail(HETAL_E_INVALID_ARG, "Hamming weight above N");
  for (u64 k = 0; k < n; ++k) out[k] = 0;
  u64 p = 0;
  for (int set = 0; set < h; ++p) {
    const u64 w = stream_word(seed, PURPOSE_SECRET, 0, 0, p);
    const u64 pos = w & (n - 1);
    if (out[pos] != 0) continue;
    out[pos] = (w >> 63) ? -1 : 1;
    ++set;
  }
}

void sample_uniform(Context& c, u64 seed, u32 purpose, u32 index, int rows, int group, u64* out) {
  c.begin_launch();
  hipLaunchKernelGGL(uniform_kernel, dim3((unsigned)(c.n / 8 / STPB), (unsigned)rows), dim3(STPB), 0, c.stream, seed,
                     purpose, index, group, c.d_mod, out, c.log_n);
  c.end_launch(KC_ELEMWISE, 8.0 * c.n * rows);
}

void sample_gaussian(Context& c, u64 seed, u32 purpose, u32 index, int count, i64* out) {
  if (!c.d_gauss) {
    u64 t[GAUSS_ENTRIES];
    gaussian_table(t);
    HCHECK(hipMalloc(&c.d_gauss, sizeof(t)));
    HCHECK(hipMemcpy(c.d_gauss, t, sizeof(t), hipMemcpyHostToDevice));
  }
  c.begin_launch();
  hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)(c.n / 8 / STPB), (unsigned)count), dim3(STPB), 0, c.stream, seed,
                     purpose, index, c.d_gauss, out, c.log_n);
  c.end_launch(KC_ELEMWISE, 8.0 * c.n * count);
}

}  // namespace hetal
