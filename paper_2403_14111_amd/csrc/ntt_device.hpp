// Device helpers shared by the NTT passes (ntt.hip) and the fused key-switch kernels (keyswitch.hip): the
// workgroup shape, conversions between stored 64-bit residues and exact doubles, and the LDS transpose that
// switches which thread owns which elements of a sub-transform.
#pragma once
#include "hetal_internal.hpp"
#include "ntt_fp64.hpp"

namespace hetal {

constexpr int NTT_THREADS = 256;
constexpr int NTT_R = 16;  // residues per thread

__device__ __forceinline__ int pad_idx(int v) { return v + (v >> 4); }

// u64 below 2^53 -> double, exactly.
__device__ __forceinline__ double u2d(u64 v) {
#pragma clang fp contract(off)
  return __builtin_fma((double)hi32(v), 4294967296.0, (double)lo32(v));
}

// Integer-valued double in [0, 2^53) -> u64.
__device__ __forceinline__ u64 d2u(double v) {
#pragma clang fp contract(off)
  const double h = __builtin_floor(v * (1.0 / 4294967296.0));
  const double l = __builtin_fma(-h, 4294967296.0, v);
  return ((u64)(u32)h << 32) | (u64)(u32)l;
}

// Intermediate rows that only these kernels read hold the bit patterns of the (integer-valued) doubles, so
// that neither side converts.  Such rows are never residues in [0, q) as 64-bit integers: only a reader that
// takes them through mid_ld may read them.
__device__ __forceinline__ u64 mid_st(double v) { return (u64)__double_as_longlong(v); }
__device__ __forceinline__ double mid_ld(u64 w) { return __longlong_as_double((long long)w); }

// Waits until the calling wavefront's LDS accesses so far have completed; the compiler moves no memory access
// across it.
__device__ __forceinline__ void wave_lds_wait() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Transpose through LDS: x[u] is stored at word widx(u) of the workgroup's buffer, then x[u] is
// loaded from word ridx(u).  The 64-bit values travel as two 32-bit halves through a 32-bit
// buffer, which halves the LDS a workgroup holds.  LEAD_SYNC: the buffer was read before.  WAVE: every
// lane that reads a word written here belongs to the writer's wavefront (the 16 threads of a contiguous
// sub-transform are consecutive lanes, with a slice of the buffer of their own), so waiting for the wavefront's
// own LDS accesses is enough and no workgroup barrier is taken.
template <bool LEAD_SYNC, bool WAVE = false, class W, class R>
__device__ __forceinline__ void lds_exchange(double (&x)[NTT_R], u32* __restrict__ ls, W widx, R ridx) {
  auto sync = [] {
    if (WAVE)
      wave_lds_wait();
    else
      __syncthreads();
  };
  if (LEAD_SYNC) sync();
#pragma unroll
  for (int u = 0; u < NTT_R; ++u) ls[widx(u)] = lo32((u64)__double_as_longlong(x[u]));
  sync();
  u32 lo[NTT_R];
#pragma unroll
  for (int u = 0; u < NTT_R; ++u) lo[u] = ls[ridx(u)];
  sync();
#pragma unroll
  for (int u = 0; u < NTT_R; ++u) ls[widx(u)] = hi32((u64)__double_as_longlong(x[u]));
  sync();
#pragma unroll
  for (int u = 0; u < NTT_R; ++u) x[u] = __longlong_as_double((long long)(((u64)ls[ridx(u)] << 32) | lo[u]));
}

// Workgroups are numbered so that the batch items sharing one (row, chunk) group -- and so one twiddle and key
// range -- run back to back on the same XCD (workgroups are dealt to the 8 XCDs round robin), where those
// stay in its L2: workgroup wg covers item wg_item(wg, batch) of group wg_group(wg, batch).
__device__ __forceinline__ int wg_item(int wg, int batch) { return (wg % (8 * batch)) >> 3; }
__device__ __forceinline__ int wg_group(int wg, int batch) { return (wg / (8 * batch)) * 8 + (wg & 7); }

}  // namespace hetal
