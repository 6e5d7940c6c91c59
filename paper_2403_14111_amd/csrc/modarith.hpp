// Exact 64-bit modular arithmetic for gfx950 (device side).
//
// All moduli are primes below 2^50.  Residues stored in memory are always
// reduced to [0, q).  Two multiplication forms are used:
//   * Shoup multiplication by a constant w (with w' = floor(w 2^64 / q)):
//     for any a < 2^64, a*w - floor(a*w'/2^64)*q lies in [0, 2q);
//   * Barrett reduction of a 128-bit value x < 2^(b+64), b = bitlen(q) - 1,
//     with mu = floor(2^(b+64) / q): the estimate floor((x >> b) * mu / 2^64)
//     is at most 2 below floor(x / q), so two conditional subtractions finish.
// Integer multiplies (v_mul_lo_u32, v_mul_hi_u32, v_mad_u64_u32) issue at
// full rate on gfx950, so these are VALU sequences of ~20 instructions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

struct ModInfo {
  u64 q;
  u64 mu;       // floor(2^(b+64) / q)
  u64 one_sh;   // floor(2^64 / q): Shoup companion of 1, for lazy final reductions
  int b;        // bitlen(q) - 1
  int pad;
};

struct U128 {
  u64 lo, hi;
};

__device__ __forceinline__ u32 lo32(u64 x) { return (u32)x; }
__device__ __forceinline__ u32 hi32(u64 x) { return (u32)(x >> 32); }

// High 64 bits of a * b, from 32-bit halves:
//   x = a0 b1 + hi(a0 b0), y = a1 b0 + lo(x), hi = a1 b1 + hi(x) + hi(y)
// (each partial sum fits in 64 bits; one v_mul_hi_u32, three v_mad_u64_u32).
__device__ __forceinline__ u64 mulhi64(u64 a, u64 b) {
  const u32 a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
  const u64 x = (u64)a0 * b1 + __umulhi(a0, b0);
  const u64 y = (u64)a1 * b0 + lo32(x);
  return (u64)a1 * b1 + ((u64)hi32(x) + hi32(y));
}

// floor(a * b / 2^64) - e with e in {0, 1, 2}: the high word without the
// carries out of the low partial products (a1 b1 + hi(a0 b1) + hi(a1 b0)).
__device__ __forceinline__ u64 mulhi64_lazy(u64 a, u64 b) {
  const u32 a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
  return (u64)a1 * b1 + ((u64)__umulhi(a0, b1) + __umulhi(a1, b0));
}

// Low 64 bits of a * b: a0 b0 + ((a0 b1 + a1 b0) mod 2^32) 2^32.
__device__ __forceinline__ u64 mullo64(u64 a, u64 b) {
  const u32 a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
  const u32 cross = a0 * b1 + a1 * b0;
  return (u64)a0 * b0 + ((u64)cross << 32);
}

__device__ __forceinline__ U128 mul_wide(u64 a, u64 b) {
  U128 r;
  r.lo = mullo64(a, b);
  r.hi = mulhi64(a, b);
  return r;
}

__device__ __forceinline__ void acc_wide(U128& acc, U128 x) {
  u64 lo = acc.lo + x.lo;
  acc.hi += x.hi + (lo < x.lo ? 1ull : 0ull);
  acc.lo = lo;
}

// a*w mod q lazily: result in [0, 2q) for any a < 2^64.
__device__ __forceinline__ u64 mul_shoup_lazy(u64 a, u64 w, u64 wp, u64 q) {
  const u64 h = mulhi64(a, wp);
  return mullo64(a, w) - mullo64(h, q);
}

// a*w mod q, lazier: with the quotient estimate of mulhi64_lazy (at most 3
// below floor(a w / q)) the result lies in [0, 4q), for any a < 2^64.
__device__ __forceinline__ u64 mul_shoup_lazy4(u64 a, u64 w, u64 wp, u64 q) {
  const u64 h = mulhi64_lazy(a, wp);
  return mullo64(a, w) - mullo64(h, q);
}

// The same product with the subtraction folded into multiply-adds: a*w - h*q = a*w + h*nq (mod 2^64)
// with nq = 2^64 - q, so both low partial products chain into one 64-bit multiply-add and the four
// cross products into the high word.  Result in [0, 4q) for any a < 2^64.
__device__ __forceinline__ u64 mul_shoup_lazy4n(u64 a, u64 w, u64 wp, u64 nq) {
  const u32 a0 = lo32(a), a1 = hi32(a);
  const u64 h = mulhi64_lazy(a, wp);
  const u32 h0 = lo32(h), h1 = hi32(h);
  const u64 lo = (u64)a0 * lo32(w) + (u64)h0 * lo32(nq);
  const u32 hi = hi32(lo) + a0 * hi32(w) + a1 * lo32(w) + h0 * hi32(nq) + h1 * lo32(nq);
  return ((u64)hi << 32) | lo32(lo);
}

// x mod q lazily, in [0, 4q) for any x < 2^64 (Shoup multiplication by 1).
__device__ __forceinline__ u64 reduce_lazy4(u64 x, u64 one_sh, u64 nq) {
  const u64 h = mulhi64_lazy(x, one_sh);
  const u32 h0 = lo32(h), h1 = hi32(h);
  const u64 lo = (u64)lo32(x) + (u64)h0 * lo32(nq);
  const u32 hi = hi32(lo) + hi32(x) + h0 * hi32(nq) + h1 * lo32(nq);
  return ((u64)hi << 32) | lo32(lo);
}

__device__ __forceinline__ u64 csub(u64 x, u64 q) { return x >= q ? x - q : x; }

__device__ __forceinline__ u64 mul_shoup(u64 a, u64 w, u64 wp, u64 q) { return csub(mul_shoup_lazy(a, w, wp, q), q); }

// x mod q for x < 2^64, through Shoup multiplication by 1.
__device__ __forceinline__ u64 reduce64(u64 x, const ModInfo& m) { return csub(x - mullo64(mulhi64(x, m.one_sh), m.q), m.q); }

// x mod q for x < 2^(b+64).
__device__ __forceinline__ u64 reduce128(U128 x, const ModInfo& m) {
  u64 t = (x.hi << (64 - m.b)) | (x.lo >> m.b);
  u64 qh = mulhi64(t, m.mu);
  u64 r = x.lo - mullo64(qh, m.q);
  r = csub(r, m.q);
  return csub(r, m.q);
}

__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const ModInfo& m) { return reduce128(mul_wide(a, b), m); }

__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) { return csub(a + b, q); }
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
__device__ __forceinline__ u64 neg_mod(u64 a, u64 q) { return a ? q - a : 0; }

// 16-bit bit reversal helper for NTT-domain index maps.
__device__ __forceinline__ u32 bit_reverse(u32 x, int bits) { return __builtin_bitreverse32(x) >> (32 - bits); }

// Position in the NTT domain (bit-reversed order of the odd exponents 2k+1)
// that holds the value at exponent g*e, for the automorphism X -> X^g.
__device__ __forceinline__ u32 galois_source(u32 k, u32 g, int log_n) {
  u32 e = 2u * bit_reverse(k, log_n) + 1u;
  u32 e2 = (g * e) & ((2u << log_n) - 1u);  // only the low log_n + 1 bits matter
  return bit_reverse((e2 - 1u) >> 1, log_n);
}

// Slot of the word at NTT-domain position pos in a stored switching key: the key inner product's 16 threads of a
// 256-word chunk own element 16 j + u of the chunk (thread j, element u < 16) and read it from slot 16 u + j.
__device__ __forceinline__ u32 key_slot(u32 pos) { return (pos & ~255u) | ((pos & 15u) << 4) | ((pos >> 4) & 15u); }
