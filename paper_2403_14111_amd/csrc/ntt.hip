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
//    stages run in registers, one LDS transpose (in two 32-bit halves, padded
//    against bank conflicts) switches the ownership, the remaining stages run
//    in registers again.
//  * Loads and stores are arranged so that the 16 threads of a sub-transform
//    (contiguous pass) or 16 neighbouring columns (strided pass) touch 128
//    contiguous bytes.
//  * The arithmetic is FP64, which gfx950 issues at the full vector rate while
//    64-bit integer products take several half- and quarter-rate 32-bit
//    multiplies.  Residues (all moduli are below 2^50) are exact integers in
//    doubles between the loads and the stores, which stay 64-bit integers:
//      - a*w mod q for |a| <= 2^51, 0 <= w < q: p = fl(a w) and its exact
//        error e = fma(a, w, -p); f = floor(fl(p * fl(1/q))) is within one of
//        floor(a w / q) (relative error below 3 * 2^-53), so
//        r = fma(-f, q, p) + e = a w - f q is exact and lies in (-0.75q, 1.75q);
//      - v mod q for an integer |v| < 2^52: r = fma(-floor(fl(v * fl(1/q))), q, v)
//        is exact and lies in [0, q] (the quotient is off by less than 1/q,
//        and r is an integer).
//    Every butterfly output is reduced that way, so each stage takes and gives
//    values in [0, q]; stored results are mapped to [0, q).  Rows of moduli
//    below 2^42 (most of the chain) skip those reductions within a pass (see
//    fwd_bfly / inv_bfly).  Twiddles are doubles (8 bytes, no Shoup companion).
#include <type_traits>

#include "ntt_device.hpp"

namespace hetal {

namespace {

using namespace fp64;

// Arguments of one pass over `groups` (row, chunk) pairs of `batch` items (numbered as wg_item / wg_group).
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

// One pass of 2^L-point sub-transforms.  Two shapes occur:
//  * strided (pass A, CONTIG false): the 256 columns of the limb seen as a 2^L x 256 matrix, stages
//    0 .. L-1 (s0 == 0); element v of column c sits at c + 256 v;
//  * contiguous (pass B, CONTIG true): the 2^(log_n - 8) chunks of 256, stages log_n - 8 .. log_n - 1
//    (L == 8); element v of chunk c sits at 256 c + v.
// Forward passes run A then B, inverse passes B then A; the second pass of either is the final one
// (stored in [0, q); the first pass stores [0, q] as doubles, read only by the second).  Inputs are in [0, q].
//
// Each thread holds 16 elements of one sub-transform: in stages 0..3 of the pass element
// v = j + T u ("spread"), in stages 4..L-1 element v = 16 j + u ("block").  The twiddle of stage l
// for element v is psi_rev[2^(s0 + l) + (c 2^l) + (v >> (L - l))] (c = 0 in the strided pass, where
// in the spread stages it does not depend on the lane at all), stored at ntt_twiddle_slot of that.
// EPI (forward contiguous pass only): the combine epilogue of NttEpilogue replaces the plain store.  X & NTT_TOP
// (with EPI): the rows of NttEpilogue::top_prime then also run the inverse contiguous pass (a rescale's first
// launch).  X & NTT_TENSOR: a Mult's tensor product is read where it is needed (NttEpilogue::tensor).
// (The key switch's strided passes, which compute their input by a basis conversion, are in keyswitch.hip.)
constexpr int NTT_TOP = 1;     // (with EPI) the top rows also run the inverse contiguous pass
constexpr int NTT_TENSOR = 2;  // a Mult's tensor product computed where it is read (NttEpilogue::tensor)
constexpr int NTT_PTMUL = 4;   // a plaintext product applied where the rows are read (NttEpilogue::pt_mul)

template <int L, bool INV, bool CONTIG, bool EPI, int X = 0>
__global__ void __launch_bounds__(NTT_THREADS) ntt_pass_kernel(PassArgs pa, const int2* __restrict__ rows,
                                                              const double* __restrict__ tw,
                                                              const FpMod* __restrict__ fpm,
                                                              const PrimeConsts* __restrict__ pc, int log_n, int s0,
                                                              NttEpilogue epi) {
#pragma clang fp contract(off)
  constexpr int SUB = 1 << L;
  constexpr int T = SUB / NTT_R;        // threads per sub-transform
  constexpr int S = NTT_THREADS / T;    // sub-transforms per workgroup
  constexpr bool FINAL = INV != CONTIG;
  static_assert(!CONTIG || L == 8, "the contiguous pass covers the last 8 stages");
  static_assert(!EPI || (CONTIG && !INV), "the epilogue belongs to the last forward pass");
  constexpr bool TOP = (X & NTT_TOP) != 0;
  constexpr bool TENSOR = (X & NTT_TENSOR) != 0;
  constexpr bool PTMUL = (X & NTT_PTMUL) != 0;
  static_assert(!TENSOR || CONTIG, "the tensor product is read by the contiguous passes");
  // Words per sub-transform slice.  Within a slice one word of padding per 16 spreads the strided
  // reads; the slice length is chosen so that the 16-lane groups of a wave reading or writing
  // neighbouring slices in lockstep fall on distinct banks.
  constexpr int PAD = SUB + SUB / 16 + (CONTIG ? 0 : 2);
  __shared__ u32 lds[S * PAD];

  const int n = 1 << log_n;
  const int wg = blockIdx.x;
  const int item = wg_item(wg, pa.batch);
  const int group = wg_group(wg, pa.batch);
  if (group >= pa.groups) return;
  const int rowi = group / pa.wg_per_poly;
  const int chunk = group - rowi * pa.wg_per_poly;
  const int2 rj = rows[rowi];
  u64* __restrict__ a = pa.base + (size_t)item * pa.batch_stride + (size_t)rj.x * n;
  const u64* __restrict__ ain =
      pa.src ? pa.src + (size_t)item * pa.src_batch_stride + (size_t)(rj.x * pa.src_row_mul + pa.src_row_add) * n : a;
  const FpMod fm = fpm[rj.y];
  const double q = fm.q, qi = fm.qinv;
  const double* __restrict__ w = tw + (size_t)rj.y * n;

  const int tid = threadIdx.x;
  const int sl = CONTIG ? tid / T : tid % S;
  const int j = CONTIG ? tid % T : tid / S;
  const int sub = chunk * S + sl;
  // limb offsets of this thread's elements: spread u at sp_off + sp_step u, block u at bl_off + bl_step u
  const u32 sp_off = CONTIG ? (u32)(sub * SUB + j) : (u32)(sub + (j << 8));
  const u32 bl_off = CONTIG ? (u32)(sub * SUB + 16 * j) : (u32)(sub + (j << 12));
  constexpr u32 sp_step = CONTIG ? T : T * 256;
  constexpr u32 bl_step = CONTIG ? 1 : 256;
  u32* __restrict__ ls = lds + sl * PAD;
  auto spread = [&](int u) { return pad_idx(j + T * u); };
  auto block = [&](int u) { return pad_idx(16 * j + u); };
  auto tw_spread = [&](int l, int u) {
    return CONTIG ? w[(1 << (s0 + l)) + (sub << l) + (u >> (4 - l))] : w[(1 << l) + (u >> (4 - l))];
  };
  auto tw_block = [&](int l, int u) {
    // contiguous pass: entry (16 j + u) >> (8 - l) = j 2^(l-4) + i of the chunk's block, stored at 16 i + j
    return CONTIG ? w[(1 << (s0 + l)) + (sub << l) + (((u >> (8 - l)) << 4) | j)]
                  : w[(1 << l) + ((16 * j + u) >> (L - l))];
  };
  double x[NTT_R];

  if (!INV) {
    // LZ: the lazy butterflies and conversion sums of moduli below 2^42 (see fwd_bfly)
    auto transform = [&](auto lazy) {
      constexpr bool LZ = decltype(lazy)::value;
      // keeps the two instances' identical loads from being merged above the branch (which would hold every
      // twiddle of the pass in registers at once)
      asm volatile("" ::: "memory");
      {
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) {
          const u64 w = (ain + sp_step * u)[sp_off];
          x[u] = FINAL ? mid_ld(w) : u2d(w);  // the final pass reads the first pass's doubles
        }
      }
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int hu = 8 >> l;
#pragma unroll
        for (int u = 0; u < NTT_R; ++u)
          if (!(u & hu)) fwd_bfly<LZ>(x[u], x[u + hu], tw_spread(l, u), q, qi);
      }
      if (L > 4) {
        lds_exchange<false, CONTIG>(x, ls, spread, block);
#pragma unroll
        for (int l = 4; l < L; ++l) {
          const int half = 1 << (L - 1 - l);
#pragma unroll
          for (int u = 0; u < NTT_R; ++u)
            if (!(u & half)) fwd_bfly<LZ>(x[u], x[u + half], tw_block(l, u), q, qi);
        }
      }
      if (LZ) {
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) x[u] = fred(x[u], q, qi);
      }
    };
    // (the epilogue pass keeps to the reduced butterflies: the lazy copy's registers cost it a wave per SIMD)
    if (!EPI && q < LAZY_MODULUS)
      transform(std::true_type{});
    else
      transform(std::false_type{});
    if (FINAL && !EPI) {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = ffix(x[u], q);
    }
    if (CONTIG && EPI) {
      // (a - x) c + addends: a - x in [-q, q] (with a_mul in (-1.75 q, 1.75 q)), its product in (-0.75q, 1.75q),
      // plus two residues: below 3.75q < 2^52 before the reduction
      lds_exchange<true, true>(x, ls, block, spread);
      const int p = rj.x >= epi.l ? 1 : 0;
      const int i = rj.y;
      const double cst = u2d(epi.cst[i]);
      const u64* __restrict__ ea = epi.a + item * epi.a_stride + ((size_t)p * epi.a_poly_rows + i) * n;
      u64* __restrict__ eo = epi.out + item * epi.out_stride + (size_t)rj.x * n;
      const u64* __restrict__ own = p == 0 ? (epi.add0 ? epi.add0 + item * epi.add0_stride + (size_t)i * n : nullptr)
                                           : (epi.add1 ? epi.add1 + item * epi.add1_stride + (size_t)i * n : nullptr);
      const u64* __restrict__ both = epi.addx ? epi.addx + item * epi.addx_stride + (size_t)rj.x * n : nullptr;
      const u32 g = epi.g[item];
      const bool perm = g != 1;                           // a key switch by tau_g: x and a precede tau_g
      const bool own_before = perm && p == 0 && epi.gather;  // tau_g's input c0: added before the permutation
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) {
        const u32 k = sp_off + sp_step * u;
        double av = epi.a_dbl ? mid_ld(ea[k]) : u2d(ea[k]);
        if (epi.a_mul) av = fmul(av, u2d(epi.a_k[i]), q, qi);  // in (-0.75 q, 1.75 q)
        if (PTMUL) av = fmul(av, u2d(epi.ta[item][(size_t)i * n + k]), q, qi);
        double v = fmul(av - x[u], cst, q, qi);
        if (own_before) v = v + u2d(own[k]);
        x[u] = v;
      }
      // tau_g moves the value at position k to galois_source(k, g^-1): this chunk's 256 words all land in one
      // chunk, so the move is an exchange through the chunk's LDS slice, and the stores stay coalesced
      u32 out_chunk = (u32)sub << 8;
      if (perm) {
        const u32 gi = epi.ginv[item];
        out_chunk = galois_source(out_chunk, gi, log_n) & ~255u;
        auto dest = [&](int u) { return pad_idx((int)(galois_source(sp_off + sp_step * u, gi, log_n) & 255u)); };
        lds_exchange<true, true>(x, ls, dest, spread);
      }
      const u32 o_off = out_chunk + (u32)j;
      // the tensor product's row i of c_p: a0 b0 (p = 0), a0 b1 + a1 b0 (p = 1), reduced to [0, q]
      const u64* __restrict__ ta0 = TENSOR ? epi.ta[item] + (size_t)i * n : nullptr;
      const u64* __restrict__ tb0 = TENSOR ? epi.tb[item] + (size_t)i * n : nullptr;
      const u64* __restrict__ ta1 = TENSOR ? ta0 + (size_t)epi.l * n : nullptr;
      const u64* __restrict__ tb1 = TENSOR ? tb0 + (size_t)epi.l * n : nullptr;
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) {
        const u32 k = o_off + sp_step * u;
        double v = x[u];
        if (TENSOR) {
          const double d = p == 0 ? fmul(u2d(ta0[k]), u2d(tb0[k]), q, qi)
                                  : fmul(u2d(ta0[k]), u2d(tb1[k]), q, qi) + fmul(u2d(ta1[k]), u2d(tb0[k]), q, qi);
          v = v + fred(d, q, qi);
        } else if (own && !own_before) {
          v = v + u2d(own[k]);
        }
        if (both) v = v + u2d(both[k]);
        x[u] = ffix(fred(v, q, qi), q);
        eo[k] = d2u(x[u]);
      }
      if (TOP && i == epi.top_prime) {
        // the inverse transform's contiguous pass on the result, as ntt_inverse_first_pass would run it on the
        // stored row (the host asks for this only without a permutation, so the chunk is the workgroup's own)
        const double* __restrict__ wi = epi.tw_inv + (size_t)i * n;
        auto twi_spread = [&](int l, int u) { return wi[(1 << (s0 + l)) + (sub << l) + (u >> (4 - l))]; };
        auto twi_block = [&](int l, int u) { return wi[(1 << (s0 + l)) + (sub << l) + (((u >> (8 - l)) << 4) | j)]; };
        auto inverse = [&](auto lazy) {
          constexpr bool LZ = decltype(lazy)::value;
          lds_exchange<true, true>(x, ls, spread, block);
#pragma unroll
          for (int l = 7; l >= 4; --l) {
            const int half = 1 << (7 - l);
#pragma unroll
            for (int u = 0; u < NTT_R; ++u)
              if (!(u & half)) inv_bfly<LZ>(x[u], x[u + half], twi_block(l, u), q, qi);
          }
          if (LZ) {
#pragma unroll
            for (int u = 0; u < NTT_R; ++u) x[u] = fred(x[u], q, qi);
          }
          lds_exchange<true, true>(x, ls, block, spread);
#pragma unroll
          for (int l = 3; l >= 0; --l) {
            const int hu = 8 >> l;
#pragma unroll
            for (int u = 0; u < NTT_R; ++u)
              if (!(u & hu)) inv_bfly<LZ>(x[u], x[u + hu], twi_spread(l, u), q, qi);
          }
          if (LZ) {
#pragma unroll
            for (int u = 0; u < NTT_R; ++u) x[u] = fred(x[u], q, qi);
          }
        };
        if (q < LAZY_MODULUS)
          inverse(std::true_type{});
        else
          inverse(std::false_type{});
        u64* __restrict__ to = epi.top_out + item * epi.top_out_stride + (size_t)p * n;
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) (to + sp_step * u)[sp_off] = mid_st(x[u]);
      }
    } else if (CONTIG) {
      lds_exchange<true, true>(x, ls, block, spread);
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) (a + sp_step * u)[sp_off] = d2u(x[u]);
    } else if (L > 4) {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) (a + bl_step * u)[bl_off] = mid_st(x[u]);
    } else {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) (a + sp_step * u)[sp_off] = mid_st(x[u]);
    }
  } else {
    auto transform = [&](auto lazy) {
      constexpr bool LZ = decltype(lazy)::value;
      asm volatile("" ::: "memory");  // as in the forward branch
      if (CONTIG) {
        if (TENSOR) {
          // row i of a Mult's a1 b1: computed from the pair, stored in NTT form, and transformed
          const int i = rj.y;
          const u64* __restrict__ a1 = epi.ta[item] + (size_t)(epi.l + i) * n;
          const u64* __restrict__ b1 = epi.tb[item] + (size_t)(epi.l + i) * n;
          u64* __restrict__ d2 = epi.t_out + item * epi.t_out_stride + (size_t)i * n;
#pragma unroll
          for (int u = 0; u < NTT_R; ++u) {
            const u32 k = sp_off + sp_step * u;
            x[u] = ffix(fred(fmul(u2d(a1[k]), u2d(b1[k]), q, qi), q, qi), q);
            d2[k] = d2u(x[u]);
          }
        } else if (PTMUL) {
          // times the item's plaintext, row of this prime
          const u64* __restrict__ pt = epi.ta[item] + (size_t)rj.y * n;
#pragma unroll
          for (int u = 0; u < NTT_R; ++u) {
            const u32 k = sp_off + sp_step * u;
            x[u] = fred(fmul(u2d(ain[k]), u2d(pt[k]), q, qi), q, qi);  // [0, q]
          }
        } else {
#pragma unroll
          for (int u = 0; u < NTT_R; ++u) x[u] = u2d((ain + sp_step * u)[sp_off]);
        }
        lds_exchange<false, true>(x, ls, spread, block);
      } else if (L > 4) {
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) x[u] = mid_ld((ain + bl_step * u)[bl_off]);
      } else {
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) x[u] = mid_ld((ain + sp_step * u)[sp_off]);
      }
      if (L > 4) {
#pragma unroll
        for (int l = L - 1; l >= 4; --l) {
          const int half = 1 << (L - 1 - l);
#pragma unroll
          for (int u = 0; u < NTT_R; ++u)
            if (!(u & half)) inv_bfly<LZ>(x[u], x[u + half], tw_block(l, u), q, qi);
        }
        if (LZ) {  // halfway: back to [0, q]
#pragma unroll
          for (int u = 0; u < NTT_R; ++u) x[u] = fred(x[u], q, qi);
        }
        if (CONTIG)
          lds_exchange<true, true>(x, ls, block, spread);
        else
          lds_exchange<false>(x, ls, block, spread);
      }
#pragma unroll
      for (int l = 3; l >= 0; --l) {
        const int hu = 8 >> l;
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) {
          if (u & hu) continue;
          if (l == 0 && FINAL) {
            // last stage of the transform, N^-1 (or the row's replacement) merged into both outputs
            const double k0 = u2d(pc[rj.y].ninv);
            const double k1 = u2d(pc[rj.y].w1ninv);
            const double s = x[u] + x[u + hu];  // [0, 2q] (lazy: below 16q)
            const double d = x[u] - x[u + hu];
            x[u] = ffix(fred(fmul(s, k0, q, qi), q, qi), q);
            x[u + hu] = ffix(fred(fmul(d, k1, q, qi), q, qi), q);
          } else {
            inv_bfly<LZ>(x[u], x[u + hu], tw_spread(l, u), q, qi);
          }
        }
      }
      if (LZ && !FINAL) {
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) x[u] = fred(x[u], q, qi);
      }
    };
    if (q < LAZY_MODULUS)
      transform(std::true_type{});
    else
      transform(std::false_type{});
#pragma unroll
    for (int u = 0; u < NTT_R; ++u)
      (a + sp_step * u)[sp_off] = !FINAL ? mid_st(x[u]) : d2u(x[u]);
  }
}

template <bool INV>
void launch_pass(Context& c, int L, u64* base, size_t batch_stride, int batch, RowsRef rows, int s0,
                 const NttSrc& src, const NttEpilogue* epi = nullptr) {
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
  const double* tw = INV ? c.d_twd_inv : c.d_twd_fwd;
  // the strided pass is the 2^L x 256 column view (s0 == 0), the contiguous one the last 8 stages
  const bool contiguous = s0 + L == c.log_n;
  if (contiguous ? (L != 8) : (s0 != 0 || L + 8 != c.log_n)) fail(HETAL_E_PARAMS, "unsupported NTT pass shape");
  if (epi && !contiguous) fail(HETAL_E_PARAMS, "NTT epilogue outside the contiguous pass");
  if (epi && INV && !epi->tensor && !epi->pt_mul) fail(HETAL_E_PARAMS, "NTT epilogue outside the last forward pass");
  if (epi && batch > MAX_BATCH) fail(HETAL_E_INVALID_ARG, "NTT epilogue batch");
  const NttEpilogue no_epi{};
  c.begin_launch();
  if (epi && INV && epi->tensor) {
    hipLaunchKernelGGL((ntt_pass_kernel<8, true, true, false, NTT_TENSOR>), grid, block, 0, c.stream, pa, rows.d, tw,
                       c.d_fpm, c.d_pc, c.log_n, s0, *epi);
  } else if (epi && INV) {
    hipLaunchKernelGGL((ntt_pass_kernel<8, true, true, false, NTT_PTMUL>), grid, block, 0, c.stream, pa, rows.d, tw,
                       c.d_fpm, c.d_pc, c.log_n, s0, *epi);
  } else if (epi) {
    if (epi->pt_mul && (epi->top_out || epi->tensor)) fail(HETAL_E_PARAMS, "unsupported epilogue combination");
    switch ((epi->top_out ? NTT_TOP : 0) | (epi->tensor ? NTT_TENSOR : 0) | (epi->pt_mul ? NTT_PTMUL : 0)) {
#define HETAL_EPI_CASE(XX)                                                                                       \
  case XX:                                                                                                     \
    hipLaunchKernelGGL((ntt_pass_kernel<8, false, true, true, XX>), grid, block, 0, c.stream, pa, rows.d, tw,     \
                       c.d_fpm, c.d_pc, c.log_n, s0, *epi);                                                    \
    break;
      HETAL_EPI_CASE(0)
      HETAL_EPI_CASE(1)
      HETAL_EPI_CASE(2)
      HETAL_EPI_CASE(3)
      HETAL_EPI_CASE(4)
#undef HETAL_EPI_CASE
    }
  } else {
    switch (L * 2 + (contiguous ? 1 : 0)) {
#define HETAL_NTT_CASE(LL, CC)                                                                                 \
  case LL * 2 + CC:                                                                                          \
    hipLaunchKernelGGL((ntt_pass_kernel<LL, INV, CC, false>), grid, block, 0, c.stream, pa, rows.d, tw, c.d_fpm, \
                       c.d_pc, c.log_n, s0, no_epi);                                                         \
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
  }
  const double words = (double)c.n * rows.count * batch;
  if (epi && INV) {
    // the pair's two rows (or the row and the plaintext's) read; the pass output (and a tensor's product) written
    c.end_launch(KC_NTT_INV_CONTIG, (epi->tensor ? 32.0 : 24.0) * words);
  } else if (epi) {
    // per word: the pass input and a read, out written; addx on every row, add0 / add1 on half of them (the
    // tensor product: the pair's rows, 3 of 4 on average)
    const double per_word = 24.0 + (epi->addx ? 8.0 : 0.0) + (epi->add0 ? 4.0 : 0.0) + (epi->add1 ? 4.0 : 0.0) +
                            (epi->tensor ? 24.0 : 0.0) + (epi->pt_mul ? 8.0 : 0.0);
    c.end_launch(KC_NTT_FWD_EPILOGUE, per_word * words);
  } else {
    const int cls = INV ? (contiguous ? KC_NTT_INV_CONTIG : KC_NTT_INV_STRIDED)
                        : (contiguous ? KC_NTT_FWD_CONTIG : KC_NTT_FWD_STRIDED);
    c.end_launch(cls, 16.0 * words);  // every residue read and written once
  }
}

}  // namespace

void ntt_forward(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src,
                 const NttEpilogue* epi) {
  if (rows.count == 0 || batch == 0) return;
  const int l1 = c.log_n - 8;
  launch_pass<false>(c, l1, base, batch_stride, batch, rows, 0, src);
  launch_pass<false>(c, 8, base, batch_stride, batch, rows, l1, NttSrc{}, epi);
  c.counters[6] += (int64_t)rows.count * batch;
}

void ntt_inverse_first_pass(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src) {
  if (rows.count == 0 || batch == 0) return;
  launch_pass<true>(c, 8, base, batch_stride, batch, rows, c.log_n - 8, src);
}

void ntt_inverse_first_pass_tensor(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows,
                                   const NttEpilogue& t) {
  if (rows.count == 0 || batch == 0) return;
  if (!t.tensor || !t.t_out) fail(HETAL_E_INVALID_ARG, "tensor pass without its pairs");
  launch_pass<true>(c, 8, base, batch_stride, batch, rows, c.log_n - 8, NttSrc{}, &t);
}

void ntt_inverse_first_pass_pt(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src,
                               const NttEpilogue& t) {
  if (rows.count == 0 || batch == 0) return;
  if (!t.pt_mul) fail(HETAL_E_INVALID_ARG, "plaintext pass without its plaintexts");
  launch_pass<true>(c, 8, base, batch_stride, batch, rows, c.log_n - 8, src, &t);
}

void ntt_forward_last_pass(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows,
                           const NttEpilogue& epi) {
  if (rows.count == 0 || batch == 0) return;
  launch_pass<false>(c, 8, base, batch_stride, batch, rows, c.log_n - 8, NttSrc{}, &epi);
}

void ntt_inverse(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src) {
  if (rows.count == 0 || batch == 0) return;
  const int l1 = c.log_n - 8;
  launch_pass<true>(c, 8, base, batch_stride, batch, rows, l1, src);
  launch_pass<true>(c, l1, base, batch_stride, batch, rows, 0, NttSrc{});
  c.counters[6] += (int64_t)rows.count * batch;
}

}  // namespace hetal
