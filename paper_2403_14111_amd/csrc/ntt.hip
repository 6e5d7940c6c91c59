// Negacyclic NTT / inverse NTT for gfx950, 64-bit residues, N = 2^12 .. 2^16.
//
// Forward transform: Cooley-Tukey butterflies with the negacyclic twist merged
// into the twiddles (psi_rev[x] = psi^brev(x)); the output at position k is
// the evaluation at psi^(2 brev(k) + 1), i.e. bit-reversed order.  Inverse:
// Gentleman-Sande butterflies with psi^-brev(x), N^-1 merged into the last
// stage.  These are the textbook structures; the gfx950 specifics are:
//
//  * A 2^16 limb (512 KiB) exceeds the 160 KiB LDS of a CU, so the log N
//    stages run as two passes of independent sub-transforms: pass A covers
//    stages 0 .. L1-1 on 2^L1-point columns of stride 256, pass B covers the
//    last 8 stages on contiguous 256-point chunks.  Each pass reads and
//    writes the limb once (2 x 1 MiB of HBM traffic per limb and transform).
//  * 256 threads per workgroup, 16 residues per thread in registers: four
//    stages run in registers, one LDS transpose (padded by one word per 16 to
//    keep the strided reads conflict-free) switches the ownership, the
//    remaining stages run in registers again.
//  * Loads and stores are arranged so that the 16 threads of a sub-transform
//    (contiguous pass) or 16 neighbouring columns (strided pass) touch 128
//    contiguous bytes.
//  * Forward butterflies are lazy: X' = X + T, Y' = X + 2q - T with
//    T = Shoup(Y * W) in [0, 2q); values stay below (1 + 2 log N) q < 2^56
//    and one Shoup reduction by 1 finishes.  Inverse butterflies keep [0, 2q).
#include "hetal_internal.hpp"

namespace hetal {

namespace {

constexpr int NTT_THREADS = 256;
constexpr int NTT_R = 16;

__device__ __forceinline__ int pad_idx(int v) { return v + (v >> 4); }

__device__ __forceinline__ void fwd_bfly(u64& x, u64& y, ulonglong2 w, u64 q, u64 q2) {
  u64 t = mul_shoup_lazy(y, w.x, w.y, q);
  y = x + q2 - t;
  x = x + t;
}

__device__ __forceinline__ void inv_bfly(u64& x, u64& y, ulonglong2 w, u64 q, u64 q2) {
  u64 s = x + y;
  s = s >= q2 ? s - q2 : s;
  u64 d = x + q2 - y;
  y = mul_shoup_lazy(d, w.x, w.y, q);
  x = s;
}

template <int L, bool INV>
__global__ void __launch_bounds__(NTT_THREADS) ntt_pass_kernel(u64* __restrict__ base, size_t batch_stride,
                                                              const int2* __restrict__ rows,
                                                              const ulonglong2* __restrict__ tw,
                                                              const ModInfo* __restrict__ mods,
                                                              const PrimeConsts* __restrict__ pc, int log_n, int s0,
                                                              int final_pass) {
  constexpr int SUB = 1 << L;
  constexpr int T = SUB / NTT_R;        // threads per sub-transform
  constexpr int S = NTT_THREADS / T;    // sub-transforms per workgroup
  constexpr int PAD = SUB + SUB / 16;
  __shared__ u64 lds[S * PAD];

  const int n = 1 << log_n;
  const int log_stride = log_n - s0 - L;
  const int stride = 1 << log_stride;
  const int2 rj = rows[blockIdx.y];
  u64* __restrict__ a = base + (size_t)blockIdx.z * batch_stride + (size_t)rj.x * n;
  const u64 q = mods[rj.y].q;
  const u64 q2 = 2 * q;
  const ulonglong2* __restrict__ w = tw + (size_t)rj.y * n;

  const int tid = threadIdx.x;
  const bool contiguous = (stride == 1);
  const int sl = contiguous ? tid / T : tid % S;
  const int j = contiguous ? tid % T : tid / S;
  const int sub = blockIdx.x * S + sl;
  const int hi = sub >> log_stride;
  const int lo = sub & (stride - 1);
  u64* __restrict__ p = a + ((size_t)hi << (log_stride + L)) + lo;
  u64* __restrict__ ls = lds + sl * PAD;
  u64 x[NTT_R];

  if (!INV) {
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) x[u] = p[(size_t)(j + T * u) << log_stride];
    // stages 0..3: element v = j + T u is held in x[u]
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int hu = 8 >> l;
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) {
        if (u & hu) continue;
        const int v = j + T * u;
        const int blk = (hi << l) | (v >> (L - l));
        fwd_bfly(x[u], x[u + hu], w[(1 << (s0 + l)) + blk], q, q2);
      }
    }
    if (L > 4) {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) ls[pad_idx(j + T * u)] = x[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = ls[pad_idx(16 * j + u)];
      // stages 4..L-1: element v = 16 j + u is held in x[u]
#pragma unroll
      for (int l = 4; l < L; ++l) {
        const int half = 1 << (L - 1 - l);
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) {
          if (u & half) continue;
          const int v = 16 * j + u;
          const int blk = (hi << l) | (v >> (L - l));
          fwd_bfly(x[u], x[u + half], w[(1 << (s0 + l)) + blk], q, q2);
        }
      }
    }
    if (final_pass) {
      const ModInfo m = mods[rj.y];
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = reduce64(x[u], m);
    }
    if (L > 4) {
      if (contiguous) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) ls[pad_idx(16 * j + u)] = x[u];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) p[(size_t)(j + T * u) << log_stride] = ls[pad_idx(j + T * u)];
      } else {
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) p[(size_t)(16 * j + u) << log_stride] = x[u];
      }
    } else {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) p[(size_t)(j + T * u) << log_stride] = x[u];
    }
  } else {
    // ownership v = 16 j + u for stages L-1 .. 4
    if (L > 4 && contiguous) {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) ls[pad_idx(j + T * u)] = p[(size_t)(j + T * u) << log_stride];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = ls[pad_idx(16 * j + u)];
    } else {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = p[(size_t)(16 * j + u) << log_stride];
    }
    if (L > 4) {
#pragma unroll
      for (int l = L - 1; l >= 4; --l) {
        const int half = 1 << (L - 1 - l);
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) {
          if (u & half) continue;
          const int v = 16 * j + u;
          const int blk = (hi << l) | (v >> (L - l));
          inv_bfly(x[u], x[u + half], w[(1 << (s0 + l)) + blk], q, q2);
        }
      }
      if (contiguous) __syncthreads();
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) ls[pad_idx(16 * j + u)] = x[u];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = ls[pad_idx(j + T * u)];
    }
    // stages 3..0: element v = j + T u is held in x[u]
    const bool merge_ninv = final_pass && s0 == 0;
#pragma unroll
    for (int l = 3; l >= 0; --l) {
      const int hu = 8 >> l;
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) {
        if (u & hu) continue;
        const int v = j + T * u;
        const int blk = (hi << l) | (v >> (L - l));
        if (l == 0 && merge_ninv) {
          const PrimeConsts k = pc[rj.y];
          u64 s = x[u] + x[u + hu];
          u64 d = x[u] + q2 - x[u + hu];
          x[u] = mul_shoup_lazy(s, k.ninv, k.ninv_sh, q);
          x[u + hu] = mul_shoup_lazy(d, k.w1ninv, k.w1ninv_sh, q);
        } else {
          inv_bfly(x[u], x[u + hu], w[(1 << (s0 + l)) + blk], q, q2);
        }
      }
    }
    if (final_pass) {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = csub(x[u], q);
    }
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) p[(size_t)(j + T * u) << log_stride] = x[u];
  }
}

template <bool INV>
void launch_pass(Context& c, int L, u64* base, size_t batch_stride, int batch, RowsRef rows, int s0, int final_pass) {
  const int sub = 1 << L;
  const int per_wg = NTT_THREADS * NTT_R / sub;  // sub-transforms per workgroup
  const int nsub = c.n / sub;
  dim3 grid(nsub / per_wg, rows.count, batch), block(NTT_THREADS);
  const ulonglong2* tw = INV ? c.d_tw_inv : c.d_tw_fwd;
  c.begin_launch();
  switch (L) {
#define HETAL_NTT_CASE(LL)                                                                                      \
  case LL:                                                                                                    \
    hipLaunchKernelGGL((ntt_pass_kernel<LL, INV>), grid, block, 0, c.stream, base, batch_stride, rows.d, tw, \
                       c.d_mod, c.d_pc, c.log_n, s0, final_pass);                                            \
    break;
    HETAL_NTT_CASE(4)
    HETAL_NTT_CASE(5)
    HETAL_NTT_CASE(6)
    HETAL_NTT_CASE(7)
    HETAL_NTT_CASE(8)
#undef HETAL_NTT_CASE
    default:
      fail(HETAL_E_PARAMS, "unsupported NTT pass size");
  }
  c.end_launch(KC_NTT, 16.0 * c.n * rows.count * batch);  // every residue read and written once
}

}  // namespace

void ntt_forward(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows) {
  if (rows.count == 0 || batch == 0) return;
  const int l1 = c.log_n - 8;
  launch_pass<false>(c, l1, base, batch_stride, batch, rows, 0, 0);
  launch_pass<false>(c, 8, base, batch_stride, batch, rows, l1, 1);
  c.counters[6] += (int64_t)rows.count * batch;
}

void ntt_inverse(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows) {
  if (rows.count == 0 || batch == 0) return;
  const int l1 = c.log_n - 8;
  launch_pass<true>(c, 8, base, batch_stride, batch, rows, l1, 0);
  launch_pass<true>(c, l1, base, batch_stride, batch, rows, 0, 1);
  c.counters[6] += (int64_t)rows.count * batch;
}

}  // namespace hetal
