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
//    stages run in registers, one LDS transpose (padded by one word per 16,
//    and with an odd slice length per sub-transform, so that both access
//    patterns are free of bank conflicts) switches the ownership, the
//    remaining stages run in registers again.
//  * Loads and stores are arranged so that the 16 threads of a sub-transform
//    (contiguous pass) or 16 neighbouring columns (strided pass) touch 128
//    contiguous bytes.
//  * Butterflies are lazy.  T = Y * W mod q comes from Shoup's method with a
//    quotient estimate that skips the carries of the low partial products
//    (3 integer multiplies fewer, and no 64-bit register shuffles): it is at
//    most 3 below the exact quotient, so T lies in [0, 4q).  Forward:
//    X' = X + T, Y' = X + 4q - T; values stay below (1 + 4 log N) q < 2^57
//    and one exact Shoup reduction by 1 finishes.  Inverse: values kept in
//    [0, 4q) by one conditional subtraction of 4q on the sum.
#include "hetal_internal.hpp"

namespace hetal {

namespace {

constexpr int NTT_THREADS = 256;
constexpr int NTT_R = 16;

__device__ __forceinline__ int pad_idx(int v) { return v + (v >> 4); }

__device__ __forceinline__ void fwd_bfly(u64& x, u64& y, ulonglong2 w, u64 q, u64 q4) {
  u64 t = mul_shoup_lazy4(y, w.x, w.y, q);
  y = x + q4 - t;
  x = x + t;
}

__device__ __forceinline__ void inv_bfly(u64& x, u64& y, ulonglong2 w, u64 q, u64 q4) {
  u64 s = x + y;
  s = s >= q4 ? s - q4 : s;
  u64 d = x + q4 - y;
  y = mul_shoup_lazy4(d, w.x, w.y, q);
  x = s;
}

// Workgroups are numbered so that the batch items sharing one (row, chunk) --
// and so one twiddle range -- run back to back on the same XCD (workgroups
// are dealt to the 8 XCDs round robin), where the twiddles stay in its L2.
struct PassArgs {
  u64* base;
  size_t batch_stride;
  const u64* src;       // input of this pass (null: in place)
  size_t src_batch_stride;
  int src_row_mul, src_row_add;  // input row = row * mul + add
  int groups;           // (row, chunk) pairs
  int batch;
  int wg_per_poly;
};

template <int L, bool INV, bool CONTIG>
__global__ void __launch_bounds__(NTT_THREADS) ntt_pass_kernel(PassArgs pa, const int2* __restrict__ rows,
                                                              const ulonglong2* __restrict__ tw,
                                                              const ModInfo* __restrict__ mods,
                                                              const PrimeConsts* __restrict__ pc, int log_n, int s0,
                                                              int final_pass) {
  constexpr int SUB = 1 << L;
  constexpr int T = SUB / NTT_R;        // threads per sub-transform
  constexpr int S = NTT_THREADS / T;    // sub-transforms per workgroup
  // one word of padding per 16 keeps strided reads of a sub-transform on distinct banks; the odd
  // slice length spreads neighbouring sub-transforms (read in lockstep by the strided pass) as well
  constexpr int PAD = SUB + SUB / 16 + 1;
  __shared__ u64 lds[S * PAD];

  const int n = 1 << log_n;
  const int log_stride = log_n - s0 - L;
  const int stride = 1 << log_stride;
  const int wg = blockIdx.x;
  const int per_block = 8 * pa.batch;
  const int item = (wg % per_block) >> 3;
  const int group = (wg / per_block) * 8 + (wg & 7);
  if (group >= pa.groups) return;
  const int rowi = group / pa.wg_per_poly;
  const int chunk = group - rowi * pa.wg_per_poly;
  const int2 rj = rows[rowi];
  u64* __restrict__ a = pa.base + (size_t)item * pa.batch_stride + (size_t)rj.x * n;
  const u64* __restrict__ ain =
      pa.src ? pa.src + (size_t)item * pa.src_batch_stride + (size_t)(rj.x * pa.src_row_mul + pa.src_row_add) * n : a;
  const u64 q = mods[rj.y].q;
  const u64 q4 = 4 * q;
  const ulonglong2* __restrict__ w = tw + (size_t)rj.y * n;

  const int tid = threadIdx.x;
  constexpr bool contiguous = CONTIG;  // stride == 1
  const int sl = contiguous ? tid / T : tid % S;
  const int j = contiguous ? tid % T : tid / S;
  const int sub = chunk * S + sl;
  const int hi = sub >> log_stride;
  const int lo = sub & (stride - 1);
  u64* __restrict__ p = a + ((size_t)hi << (log_stride + L)) + lo;
  const u64* __restrict__ pin = ain + ((size_t)hi << (log_stride + L)) + lo;
  u64* __restrict__ ls = lds + sl * PAD;
  u64 x[NTT_R];

  if (!INV) {
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) x[u] = pin[(size_t)(j + T * u) << log_stride];
    // stages 0..3: element v = j + T u is held in x[u]
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int hu = 8 >> l;
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) {
        if (u & hu) continue;
        const int v = j + T * u;
        const int blk = (hi << l) | (v >> (L - l));
        fwd_bfly(x[u], x[u + hu], w[(1 << (s0 + l)) + blk], q, q4);
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
          fwd_bfly(x[u], x[u + half], w[(1 << (s0 + l)) + blk], q, q4);
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
      for (int u = 0; u < NTT_R; ++u) ls[pad_idx(j + T * u)] = pin[(size_t)(j + T * u) << log_stride];
      __syncthreads();
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = ls[pad_idx(16 * j + u)];
    } else {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = pin[(size_t)(16 * j + u) << log_stride];
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
          inv_bfly(x[u], x[u + half], w[(1 << (s0 + l)) + blk], q, q4);
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
          u64 d = x[u] + q4 - x[u + hu];
          x[u] = mul_shoup_lazy4(s, k.ninv, k.ninv_sh, q);
          x[u + hu] = mul_shoup_lazy4(d, k.w1ninv, k.w1ninv_sh, q);
        } else {
          inv_bfly(x[u], x[u + hu], w[(1 << (s0 + l)) + blk], q, q4);
        }
      }
    }
    if (final_pass) {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = csub(csub(x[u], 2 * q), q);
    }
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) p[(size_t)(j + T * u) << log_stride] = x[u];
  }
}

template <bool INV>
void launch_pass(Context& c, int L, u64* base, size_t batch_stride, int batch, RowsRef rows, int s0, int final_pass,
                 const NttSrc& src) {
  const int sub = 1 << L;
  const int per_wg = NTT_THREADS * NTT_R / sub;  // sub-transforms per workgroup
  const int nsub = c.n / sub;
  PassArgs pa;
  pa.base = base;
  pa.batch_stride = batch_stride;
  pa.src = src.p;
  pa.src_batch_stride = src.batch_stride;
  pa.src_row_mul = src.row_mul;
  pa.src_row_add = src.row_add;
  pa.wg_per_poly = nsub / per_wg;
  pa.groups = pa.wg_per_poly * rows.count;
  pa.batch = batch;
  const int padded = (pa.groups + 7) / 8 * 8;
  dim3 grid((unsigned)(padded * batch)), block(NTT_THREADS);
  const ulonglong2* tw = INV ? c.d_tw_inv : c.d_tw_fwd;
  c.begin_launch();
  const bool contiguous = s0 + L == c.log_n;
  switch (L * 2 + (contiguous ? 1 : 0)) {
#define HETAL_NTT_CASE(LL, CC)                                                                           \
  case LL * 2 + CC:                                                                                    \
    hipLaunchKernelGGL((ntt_pass_kernel<LL, INV, CC>), grid, block, 0, c.stream, pa, rows.d, tw, c.d_mod, \
                       c.d_pc, c.log_n, s0, final_pass);                                               \
    break;
    HETAL_NTT_CASE(4, 0)
    HETAL_NTT_CASE(5, 0)
    HETAL_NTT_CASE(6, 0)
    HETAL_NTT_CASE(7, 0)
    HETAL_NTT_CASE(8, 0)
    HETAL_NTT_CASE(8, 1)
#undef HETAL_NTT_CASE
    default:
      fail(HETAL_E_PARAMS, "unsupported NTT pass size");
  }
  c.end_launch(KC_NTT, 16.0 * c.n * rows.count * batch);  // every residue read and written once
}

}  // namespace

void ntt_forward(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src) {
  if (rows.count == 0 || batch == 0) return;
  const int l1 = c.log_n - 8;
  launch_pass<false>(c, l1, base, batch_stride, batch, rows, 0, 0, src);
  launch_pass<false>(c, 8, base, batch_stride, batch, rows, l1, 1, NttSrc{});
  c.counters[6] += (int64_t)rows.count * batch;
}

void ntt_inverse(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src) {
  if (rows.count == 0 || batch == 0) return;
  const int l1 = c.log_n - 8;
  launch_pass<true>(c, 8, base, batch_stride, batch, rows, l1, 0, src);
  launch_pass<true>(c, l1, base, batch_stride, batch, rows, 0, 1, NttSrc{});
  c.counters[6] += (int64_t)rows.count * batch;
}

}  // namespace hetal
