// Hybrid key switching (Sec. 2.2: the switch behind HRot, Conj and Mult's relinearisation) on gfx950, in five
// launches per batch of key switches at one level (l limbs, K special primes, beta digits of alpha primes):
//
//  1. the inverse NTT's contiguous pass over the input c1 (ntt.hip);
//  2. modconv<MODUP>: one workgroup per (item, digit, column group, subset of target primes): the inverse
//     NTT's strided pass over the digit's rows, whose last stage also multiplies by (D_j/d_i)^-1, giving
//     y_i = [x_i (D_j/d_i)^-1]_{d_i}; then for every target prime t of the subset the fast basis conversion
//     sum_i y_i (D_j/d_i) mod t and the forward NTT's strided pass;
//  3. ks_inner: one workgroup per (item, extended row t, chunk group): for every digit the forward NTT's
//     contiguous pass of its row t (the digit's own rows are the input, already in NTT form) times the key's
//     rows, summed into the b and a accumulators; the rows of q_0..q_l store the sums, the special rows go on
//     through the inverse NTT's contiguous pass (the start of ModDown);
//  4. modconv<MODDOWN>: one workgroup per (item, polynomial, column group, subset of target primes): the
//     inverse strided pass over the K special rows (times (P/p_k)^-1), each value centred, then the conversion
//     sum_k y_k (P/p_k) mod q_i and the forward strided pass;
//  5. the forward contiguous pass with the combine epilogue (acc - conv) P^-1 + addends (ntt.hip).
//
// Every intermediate lives in HBM once: the extended digits are written by (2) and read by (3), the special
// rows of the inner product are written by (3) in coefficient order's first half-transform and read by (4).
//
// The automorphism.  tau_g (X -> X^g) permutes the NTT domain, and in this library's bit-reversed order it maps
// every aligned chunk of 256 words onto a whole chunk.  It is a ring automorphism, so
//   sum_j tau_g(d_j) k_j = tau_g(sum_j d_j tau_g^-1(k_j)):
// the switching keys are stored permuted by tau_g^-1 (keygen_kernel), which makes the inner product pointwise
// in the digits' own frame.  ModDown's conversion is centred, so it commutes with the signed permutation of the
// coefficients that tau_g is in coefficient form; the epilogue therefore applies tau_g once, to the combined
// result, through its LDS exchange.  The residues are the same, word for word, as those of applying tau_g to
// the extended digits after ModUp (the order that fixes the result).
//
// Keys are stored as the bit patterns of exact doubles (every residue is below 2^50), and inside each chunk of
// 256 words in the order the inner product's threads own them (key_slot): the 16 threads of a sub-transform
// then read 128 contiguous bytes per load.
#include <algorithm>
#include <memory>
#include <type_traits>

#include "ntt_device.hpp"

namespace hetal {

namespace {

using namespace fp64;

constexpr int KIND_MODUP = 0;
constexpr int KIND_MODDOWN = 1;
constexpr int KIND_RESCALE = 2;  // one source, the top prime q_level of each polynomial; conversion factor 1
constexpr int MAX_CONV = 4;  // terms of a fused conversion: alpha and K are at most this

// A read of a table that no kernel writes while this one runs, through the constant address space: a uniform
// address then takes the scalar memory path, whose waits (lgkmcnt) are independent of the vector memory
// counter.  A vector load inside the conversion's loop over targets would make each target wait for the
// previous target's stores, since that counter completes in order.
template <class T>
__device__ __forceinline__ T cload(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}

// ------------------------------------------------------------------ basis conversion passes (launches 2 and 4)
struct ConvArgs {
  const u64* src;        // per item: the rows the inverse strided pass reads (doubles)
  size_t src_stride;
  u64* dst;              // per item: the rows the forward strided pass writes (doubles)
  size_t dst_stride;
  const int2* targets;   // (destination row, prime) of every conversion target, grouped by source group
  int first[2 * MAX_CONV];  // per source group: its first entry in `targets`, and its count (MODUP: digits,
  int count[2 * MAX_CONV];  // MODDOWN: the two polynomials)
  int nsrc[2 * MAX_CONV];   // MODUP: rows of each digit (a short last digit has fewer)
  int src_row0[2 * MAX_CONV];  // first source row of each group (MODUP: the digit's first limb; MODDOWN: p ext + l;
                               // RESCALE: p)
  const NttScale* scale;   // per source row (MODUP: indexed by limb; MODDOWN: by p K + k; RESCALE: one)
  int src_prime;           // RESCALE: the source prime's index (the level)
  NttScale scale_v;        // RESCALE: the scaling of the inverse transform's last stage (by value)
  const ModUpTab* modup;   // MODUP: the level's digit tables
  const ModDownTab* moddown;
  int num_q;
  int tpt;                 // targets per task
  int tasks_per_group;
  int groups;              // (task, column group) pairs
  int colgroups;
  int batch;
};

template <int L, int KIND, int CNT>
__global__ void __launch_bounds__(NTT_THREADS) modconv_kernel(ConvArgs a, const double* __restrict__ tw_fwd,
                                                             const double* __restrict__ tw_inv,
                                                             const FpMod* __restrict__ fpm, int log_n) {
#pragma clang fp contract(off)
  constexpr int SUB = 1 << L;
  constexpr int T = SUB / NTT_R;       // threads per column
  constexpr int S = NTT_THREADS / T;   // columns per workgroup
  constexpr int PAD = SUB + SUB / 16 + 2;
  __shared__ u32 lds[S * PAD];
  const int n = 1 << log_n;
  const int wg = blockIdx.x;
  const int item = wg_item(wg, a.batch);
  const int group = wg_group(wg, a.batch);
  if (group >= a.groups) return;
  const int task = group / a.colgroups;
  const int colgroup = group - task * a.colgroups;
  const int sg = task / a.tasks_per_group;              // source group: digit (MODUP) or polynomial (MODDOWN)
  const int t_begin = (task - sg * a.tasks_per_group) * a.tpt;
  const int t_end = min(t_begin + a.tpt, a.count[sg]);
  if (t_begin >= t_end) return;

  const int tid = threadIdx.x;
  const int sl = tid % S;
  const int j = tid / S;
  const int sub = colgroup * S + sl;
  const u32 sp_off = (u32)(sub + (j << 8)), bl_off = (u32)(sub + (j << 12));
  constexpr u32 sp_step = T * 256, bl_step = 256;
  u32* __restrict__ ls = lds + sl * PAD;
  auto spread = [&](int u) { return pad_idx(j + T * u); };
  auto block = [&](int u) { return pad_idx(16 * j + u); };

  // ---- the inverse strided pass of every source row, kept in registers: y[i] in [0, p_i)
  double y[CNT][NTT_R];
  const int nsrc = KIND == KIND_MODUP ? a.nsrc[sg] : CNT;
  const u64* __restrict__ srcb = a.src + (size_t)item * a.src_stride;
  // every source row's loads first, so that their latencies overlap
#pragma unroll
  for (int i = 0; i < CNT; ++i) {
    const u64* __restrict__ in = srcb + (size_t)(a.src_row0[sg] + (i < nsrc ? i : 0)) * n;
#pragma unroll
    for (int u = 0; u < NTT_R; ++u)
      y[i][u] = i >= nsrc ? 0.0 : mid_ld(L > 4 ? (in + bl_step * u)[bl_off] : (in + sp_step * u)[sp_off]);
  }
#pragma unroll
  for (int i = 0; i < CNT; ++i) {
    if (i >= nsrc) {  // a short last digit: zero terms (its constants beyond the length are zero too)
      // (set here, not only by the load's select, so that no source register enters the target loop with a
      // load in flight: the loop would then wait for all vector memory on every target)
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) y[i][u] = 0.0;
      continue;
    }
    const int row = a.src_row0[sg] + i;
    const int prime = KIND == KIND_MODUP ? row : KIND == KIND_MODDOWN ? a.num_q + i : a.src_prime;
    const NttScale sc = KIND == KIND_RESCALE ? a.scale_v : a.scale[KIND == KIND_MODUP ? row : sg * CNT + i];
    const FpMod fm = fpm[prime];
    const double q = fm.q, qi = fm.qinv;
    const double* __restrict__ w = tw_inv + (size_t)prime * n;
    double (&x)[NTT_R] = y[i];
    auto stages = [&](auto lazy) {
      constexpr bool LZ = decltype(lazy)::value;
      if (L > 4) {
#pragma unroll
        for (int l = L - 1; l >= 4; --l) {
          const int half = 1 << (L - 1 - l);
#pragma unroll
          for (int u = 0; u < NTT_R; ++u)
            if (!(u & half)) inv_bfly<LZ>(x[u], x[u + half], w[(1 << l) + ((16 * j + u) >> (L - l))], q, qi);
        }
        if (LZ) {
#pragma unroll
          for (int u = 0; u < NTT_R; ++u) x[u] = fred(x[u], q, qi);
        }
        lds_exchange<true>(x, ls, block, spread);
      }
      const double k0 = u2d(sc.s0), k1 = u2d(sc.s1);
#pragma unroll
      for (int l = 3; l >= 0; --l) {
        const int hu = 8 >> l;
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) {
          if (u & hu) continue;
          if (l == 0) {
            // the transform's last stage, N^-1 times the conversion's first factor merged into both outputs
            const double s = x[u] + x[u + hu];
            const double d = x[u] - x[u + hu];
            x[u] = ffix(fred(fmul(s, k0, q, qi), q, qi), q);
            x[u + hu] = ffix(fred(fmul(d, k1, q, qi), q, qi), q);
          } else {
            inv_bfly<LZ>(x[u], x[u + hu], w[(1 << l) + (u >> (4 - l))], q, qi);
          }
        }
      }
    };
    if (q < LAZY_MODULUS)
      stages(std::true_type{});
    else
      stages(std::false_type{});
    if (KIND != KIND_MODUP) {
      const double ph = __builtin_floor(q * 0.5);  // (p - 1) / 2: values above it are taken as negative
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) x[u] = x[u] > ph ? x[u] - q : x[u];
    }
  }

  // ---- each target: the conversion sum, then the forward strided pass
  u64* __restrict__ dstb = a.dst + (size_t)item * a.dst_stride;
  for (int tt = t_begin; tt < t_end; ++tt) {
    const u64 rt2 = cload((const u64*)(a.targets + a.first[sg] + tt));  // (destination row, prime)
    const int2 rt = make_int2((int)lo32(rt2), (int)hi32(rt2));
    const FpMod fm = fpm[rt.y];
    const double q = fm.q, qi = fm.qinv;
    const double* __restrict__ w = tw_fwd + (size_t)rt.y * n;
    double cc[CNT];
#pragma unroll
    for (int i = 0; i < CNT; ++i)
      cc[i] = KIND == KIND_RESCALE ? 1.0
                                   : u2d(KIND == KIND_MODUP ? cload(&a.modup[sg].dhat[i][rt.y])
                                                            : cload(&a.moddown->phat[i][rt.y]));
    double x[NTT_R];
    auto stages = [&](auto lazy) {
      constexpr bool LZ = decltype(lazy)::value;
      asm volatile("" ::: "memory");
      // MODUP: y_i < 2^50, each product in (-0.375 t, 1.375 t); MODDOWN and RESCALE: |y_k| < 2^49, in
      // (-0.19 q, 1.19 q).
      // The reducing form reduces after two terms and at the end (below 3.75 q < 2^52 in between); the lazy
      // one leaves the sum of at most four terms below 5.5 q, which the lazy butterflies take.
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) {
        double s = fmul(y[0][u], cc[0], q, qi);
#pragma unroll
        for (int i = 1; i < CNT; ++i) {
          s = s + fmul(y[i][u], cc[i], q, qi);
          if (!LZ && i == 1 && CNT > 2) s = fred(s, q, qi);
        }
        x[u] = LZ ? s : fred(s, q, qi);
      }
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        const int hu = 8 >> l;
#pragma unroll
        for (int u = 0; u < NTT_R; ++u)
          if (!(u & hu)) fwd_bfly<LZ>(x[u], x[u + hu], w[(1 << l) + (u >> (4 - l))], q, qi);
      }
      if (L > 4) {
        lds_exchange<true>(x, ls, spread, block);
#pragma unroll
        for (int l = 4; l < L; ++l) {
          const int half = 1 << (L - 1 - l);
#pragma unroll
          for (int u = 0; u < NTT_R; ++u)
            if (!(u & half)) fwd_bfly<LZ>(x[u], x[u + half], w[(1 << l) + ((16 * j + u) >> (L - l))], q, qi);
        }
      }
      if (LZ) {
#pragma unroll
        for (int u = 0; u < NTT_R; ++u) x[u] = fred(x[u], q, qi);
      }
    };
    if (q < LAZY_MODULUS)
      stages(std::true_type{});
    else
      stages(std::false_type{});
    u64* __restrict__ out = dstb + (size_t)rt.x * n;
    if (L > 4) {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) (out + bl_step * u)[bl_off] = mid_st(x[u]);
    } else {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) (out + sp_step * u)[sp_off] = mid_st(x[u]);
    }
  }
}

// ------------------------------------------------------------------ key inner product (launch 3)
struct InnerArgs {
  const u64* dt;        // per item: [beta][ext][N], the ModUp rows after the strided pass (doubles)
  size_t dt_stride;     // 0: one set shared by every item (hoisting)
  const u64* in;        // per item: the input polynomial [l][N] in NTT form (the digits' own rows)
  size_t in_stride;
  u64* acc;             // per item: [2][ext][N]
  size_t acc_stride;
  const double* key[MAX_BATCH];  // per item: [dnum][2][nprimes][N], permuted and in key_slot order
  int groups, batch, wg_per_row;
  int l, ext, alpha, beta, num_q, nprimes;
};

// ntt_pass_kernel's contiguous pass, stages s0 .. s0 + 7 on 256-point chunks: element v of chunk `sub` sits at
// 256 sub + v; the 16 threads j of a chunk own v = j + 16 u ("spread") or v = 16 j + u ("block").
__global__ void __launch_bounds__(NTT_THREADS) ks_inner_kernel(InnerArgs a, const double* __restrict__ tw_fwd,
                                                              const double* __restrict__ tw_inv,
                                                              const FpMod* __restrict__ fpm, int log_n) {
#pragma clang fp contract(off)
  constexpr int PAD = 256 + 16;
  __shared__ u32 lds[16 * PAD];
  const int n = 1 << log_n;
  const int s0 = log_n - 8;
  const int wg = blockIdx.x;
  const int item = wg_item(wg, a.batch);
  const int group = wg_group(wg, a.batch);
  if (group >= a.groups) return;
  const int t = group / a.wg_per_row;                       // extended row: q_0 .. q_{l-1}, then p_0 .. p_{K-1}
  const int chunk = group - t * a.wg_per_row;
  const int prime = t < a.l ? t : a.num_q + (t - a.l);
  const FpMod fm = fpm[prime];
  const double q = fm.q, qi = fm.qinv;
  const bool lazy = q < LAZY_MODULUS;

  const int tid = threadIdx.x;
  const int sl = tid >> 4;
  const int j = tid & 15;
  const int sub = chunk * 16 + sl;
  const u32 sp_off = (u32)(sub * 256 + j);
  const u32 bl_off = (u32)(sub * 256 + 16 * j);
  const u32 key_off = (u32)(sub * 256 + j);  // key_slot of block element (j, u) is 16 u + j
  u32* __restrict__ ls = lds + sl * PAD;
  auto spread = [&](int u) { return pad_idx(j + 16 * u); };
  auto block = [&](int u) { return pad_idx(16 * j + u); };
  const double* __restrict__ wf = tw_fwd + (size_t)prime * n;
  auto twf_spread = [&](int l, int u) { return wf[(1 << (s0 + l)) + (sub << l) + (u >> (4 - l))]; };
  auto twf_block = [&](int l, int u) { return wf[(1 << (s0 + l)) + (sub << l) + (((u >> (8 - l)) << 4) | j)]; };

  const double* __restrict__ key = a.key[item];
  const size_t kstride = (size_t)a.nprimes * n;  // between the b and a rows of a digit
  const int own_digit = t < a.l ? t / a.alpha : -1;
  double accb[NTT_R], acca[NTT_R];
#pragma unroll
  for (int u = 0; u < NTT_R; ++u) accb[u] = acca[u] = 0.0;

  // the row of digit jd: the input itself for the digit's own row (residues, NTT form), else the ModUp row
  // after the strided pass (doubles)
  auto row_of = [&](int jd) {
    return jd == own_digit ? a.in + (size_t)item * a.in_stride + (size_t)t * n
                           : a.dt + (size_t)item * a.dt_stride + ((size_t)jd * a.ext + t) * n;
  };
  // software pipelining: the next digit's row is loaded while this one is transformed and multiplied
  u64 nxt[NTT_R];
  {
    const u64* __restrict__ r = row_of(0);
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) nxt[u] = (r + 16 * u)[sp_off];
  }
  for (int jd = 0; jd < a.beta; ++jd) {
    double x[NTT_R];
    const bool own = jd == own_digit;
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) x[u] = own ? u2d(nxt[u]) : mid_ld(nxt[u]);
    if (jd + 1 < a.beta) {
      asm volatile("" ::: "memory");
      const u64* __restrict__ r = row_of(jd + 1);
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) nxt[u] = (r + 16 * u)[sp_off];
      asm volatile("" ::: "memory");
    }
    if (own) {
      lds_exchange<true, true>(x, ls, spread, block);
    } else {
      auto stages = [&](auto lz) {
        constexpr bool LZ = decltype(lz)::value;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const int hu = 8 >> l;
#pragma unroll
          for (int u = 0; u < NTT_R; ++u)
            if (!(u & hu)) fwd_bfly<LZ>(x[u], x[u + hu], twf_spread(l, u), q, qi);
        }
        lds_exchange<true, true>(x, ls, spread, block);
#pragma unroll
        for (int l = 4; l < 8; ++l) {
          const int half = 1 << (7 - l);
#pragma unroll
          for (int u = 0; u < NTT_R; ++u)
            if (!(u & half)) fwd_bfly<LZ>(x[u], x[u + half], twf_block(l, u), q, qi);
        }
        // lazily the values stay below 13.9 q < 2^46: fmul takes them as they are
      };
      if (lazy)
        stages(std::true_type{});
      else
        stages(std::false_type{});
    }
    asm volatile("" ::: "memory");  // the key loads start after the transform (held early they cost registers)
    const double* __restrict__ kb = key + ((size_t)(2 * jd) * a.nprimes + prime) * n;
    const double* __restrict__ ka = kb + kstride;
    // products in (-0.75 q, 1.75 q): lazily (q < 2^42) at most 8 of them are summed (below 14 q), else every
    // term is folded in with a reduction (below 2.75 q before it)
    if (lazy) {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) {
        accb[u] = accb[u] + fmul(x[u], (kb + 16 * u)[key_off], q, qi);
        acca[u] = acca[u] + fmul(x[u], (ka + 16 * u)[key_off], q, qi);
      }
    } else {
#pragma unroll
      for (int u = 0; u < NTT_R; ++u) {
        accb[u] = fred(accb[u] + fmul(x[u], (kb + 16 * u)[key_off], q, qi), q, qi);
        acca[u] = fred(acca[u] + fmul(x[u], (ka + 16 * u)[key_off], q, qi), q, qi);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < NTT_R; ++u) {
    accb[u] = fred(accb[u], q, qi);  // [0, q]
    acca[u] = fred(acca[u], q, qi);
  }

  u64* __restrict__ accp = a.acc + (size_t)item * a.acc_stride;
  if (t < a.l) {
    // rows of q_0 .. q_{l-1}: the sums, read by the epilogue of launch 5
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) {
      accb[u] = ffix(accb[u], q);
      acca[u] = ffix(acca[u], q);
    }
    u64* __restrict__ ob = accp + (size_t)t * n;
    u64* __restrict__ oa = accp + (size_t)(a.ext + t) * n;
    lds_exchange<true, true>(accb, ls, block, spread);
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) (ob + 16 * u)[sp_off] = mid_st(accb[u]);
    lds_exchange<true, true>(acca, ls, block, spread);
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) (oa + 16 * u)[sp_off] = mid_st(acca[u]);
    return;
  }
  // special rows: the inverse NTT's contiguous pass (stages s0 + 7 .. s0) on the sums, which are already in the
  // block ownership its first stages use
  const double* __restrict__ wi = tw_inv + (size_t)prime * n;
  auto twi_spread = [&](int l, int u) { return wi[(1 << (s0 + l)) + (sub << l) + (u >> (4 - l))]; };
  auto twi_block = [&](int l, int u) { return wi[(1 << (s0 + l)) + (sub << l) + (((u >> (8 - l)) << 4) | j)]; };
  auto inverse = [&](double (&x)[NTT_R], u64* __restrict__ out) {
    auto stages = [&](auto lz) {
      constexpr bool LZ = decltype(lz)::value;
      asm volatile("" ::: "memory");
#pragma unroll
      for (int l = 7; l >= 4; --l) {
        const int half = 1 << (7 - l);
#pragma unroll
        for (int u = 0; u < NTT_R; ++u)
          if (!(u & half)) inv_bfly<LZ>(x[u], x[u + half], twi_block(l, u), q, qi);
      }
      if (LZ) {  // halfway: back to [0, q]
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
    if (lazy)
      stages(std::true_type{});
    else
      stages(std::false_type{});
#pragma unroll
    for (int u = 0; u < NTT_R; ++u) (out + 16 * u)[sp_off] = mid_st(x[u]);
  };
  inverse(accb, accp + (size_t)t * n);
  inverse(acca, accp + (size_t)(a.ext + t) * n);
}

// ------------------------------------------------------------------ host side
dim3 ks_grid(int groups, int batch) {
  const int padded = (groups + 7) / 8 * 8;
  return dim3((unsigned)(padded * batch));
}

// Targets per conversion task.  A task transforms its sources once and then each target, so the fewer tasks per
// source group the less is recomputed, but the launch needs about two workgroups per CU to fill the chip: the
// largest count that still gives 512 workgroups, else 2 (measured at N = 2^16, level 11: one task per digit at 8
// items, 2-3 targets per task at 1 item).
int targets_per_task(const Context& c, int targets, int sources, int items) {
  const int colgroups = std::max(1, c.n / 4096);
  for (int tpt = targets; tpt > 2; --tpt)
    if (sources * ((targets + tpt - 1) / tpt) * colgroups * items >= 512) return tpt;
  return std::min(targets, 2);
}

template <int KIND>
void launch_conv(Context& c, ConvArgs& a, int cnt, int items) {
  const int L = c.log_n - 8;
  dim3 grid = ks_grid(a.groups, items), block(NTT_THREADS);
  c.begin_launch();
  if constexpr (KIND == KIND_RESCALE) {
    if (cnt != 1 || L < 4 || L > 8) fail(HETAL_E_PARAMS, "unsupported rescale shape");
    switch (L) {
#define HETAL_RESCALE_CASE(LL)                                                                                   \
  case LL:                                                                                                     \
    hipLaunchKernelGGL((modconv_kernel<LL, KIND, 1>), grid, block, 0, c.stream, a, c.d_twd_fwd, c.d_twd_inv,    \
                       c.d_fpm, c.log_n);                                                                      \
    break;
      HETAL_RESCALE_CASE(4)
      HETAL_RESCALE_CASE(5)
      HETAL_RESCALE_CASE(6)
      HETAL_RESCALE_CASE(7)
      HETAL_RESCALE_CASE(8)
#undef HETAL_RESCALE_CASE
    }
    return;
  }
  switch (L * 10 + cnt) {
#define HETAL_CONV_CASE(LL, C)                                                                                  \
  case LL * 10 + C:                                                                                           \
    hipLaunchKernelGGL((modconv_kernel<LL, KIND, C>), grid, block, 0, c.stream, a, c.d_twd_fwd, c.d_twd_inv,   \
                       c.d_fpm, c.log_n);                                                                     \
    break;
#define HETAL_CONV_L(LL) HETAL_CONV_CASE(LL, 1) HETAL_CONV_CASE(LL, 2) HETAL_CONV_CASE(LL, 3) HETAL_CONV_CASE(LL, 4)
    HETAL_CONV_L(4)
    HETAL_CONV_L(5)
    HETAL_CONV_L(6)
    HETAL_CONV_L(7)
    HETAL_CONV_L(8)
#undef HETAL_CONV_L
#undef HETAL_CONV_CASE
    default:
      fail(HETAL_E_PARAMS, "unsupported key-switch shape");
  }
}

}  // namespace

size_t key_switch_scratch_words(const Context& c, int level, int count) {
  const size_t n = c.n;
  const size_t l = level + 1, ext = l + c.num_p, beta = c.beta(level);
  // the input's first inverse pass, the extended digits, the accumulators, the ModDown conversion rows
  return Pool::arena_round(count * l * n) + Pool::arena_round(count * beta * ext * n) +
         Pool::arena_round(count * 2 * ext * n) + Pool::arena_round(count * 2 * l * n);
}

void key_switch(Context& c, const KsJob& job) {
  const int level = job.level;
  const int l = level + 1;
  const int ext = l + c.num_p;
  const int beta = c.beta(level);
  const int m = job.count;
  if (m < 1 || m > MAX_BATCH) fail(HETAL_E_INVALID_ARG, "key switch batch size");
  if (c.alpha > MAX_CONV || c.num_p > MAX_CONV || beta > 2 * MAX_CONV) fail(HETAL_E_PARAMS, "key switch shape");
  const bool hoisted = !job.tensor && job.in_stride == 0;
  const int m_in = hoisted ? 1 : m;
  const size_t n = c.n;
  const size_t poly = (size_t)l * n;
  const size_t dt_words = (size_t)beta * ext * n;
  const size_t acc_words = 2 * (size_t)ext * n;
  const size_t conv_words = 2 * poly;
  const int colgroups = std::max(1, c.n / 4096);

  // 1. the inverse NTT's contiguous pass over the input (its strided pass runs inside launch 2); for a Mult the
  // input a1 b1 is computed here, and stored for the inner product's own rows
  Tmp coef(c.pool, m_in * poly);
  RowsRef ct_rows = c.rows(ROWS_CT, level);
  if (job.tensor && hoisted) fail(HETAL_E_INVALID_ARG, "a Mult's key switch has one input per item");
  std::unique_ptr<Tmp> d2;
  const u64* in = job.in;
  size_t in_stride = job.in_stride;
  if (job.tensor) {
    d2.reset(new Tmp(c.pool, (size_t)m * poly));
    NttEpilogue t;
    t.tensor = 1;
    t.l = l;
    for (int i = 0; i < MAX_BATCH; ++i) {
      t.ta[i] = i < m ? job.ta[i] : nullptr;
      t.tb[i] = i < m ? job.tb[i] : nullptr;
    }
    t.t_out = d2->p;
    t.t_out_stride = poly;
    ntt_inverse_first_pass_tensor(c, coef, poly, m, RowsRef{ct_rows.d, l}, t);
    in = d2->p;
    in_stride = poly;
  } else {
    NttSrc src;
    src.p = job.in;
    src.batch_stride = hoisted ? 0 : job.in_stride;
    ntt_inverse_first_pass(c, coef, poly, m_in, RowsRef{ct_rows.d, l}, src);
  }

  // 2. ModUp: the strided passes around the conversion, one launch
  Tmp dt(c.pool, m_in * dt_words);
  {
    ConvArgs a{};
    a.src = coef.p;
    a.src_stride = poly;
    a.dst = dt.p;
    a.dst_stride = dt_words;
    a.targets = c.rows(ROWS_MODUP, level).d;
    int first = 0, maxcnt = 0;
    for (int jd = 0; jd < beta; ++jd) {
      const int lo = jd * c.alpha, hi = std::min(lo + c.alpha, l);
      a.first[jd] = first;
      a.count[jd] = ext - (hi - lo);
      a.nsrc[jd] = hi - lo;
      a.src_row0[jd] = lo;
      first += a.count[jd];
      maxcnt = std::max(maxcnt, a.count[jd]);
    }
    a.scale = c.d_modup_scale + (size_t)level * MAX_PRIMES;
    a.modup = c.d_modup + (size_t)level * c.dnum;
    a.num_q = c.num_q;
    a.tpt = c.tune.tpt_modup > 0 ? std::min(c.tune.tpt_modup, maxcnt) : targets_per_task(c, maxcnt, beta, m_in);
    a.tasks_per_group = (maxcnt + a.tpt - 1) / a.tpt;
    a.colgroups = colgroups;
    a.groups = beta * a.tasks_per_group * colgroups;
    a.batch = m_in;
    launch_conv<KIND_MODUP>(c, a, c.alpha, m_in);
    // reads the l coefficient-form limbs, writes the beta ext - l rows outside the digits
    c.end_launch(KC_KS_MODUP, 8.0 * n * m_in * ((double)beta * ext));
  }

  // 3. the inner product with the keys, after the contiguous pass of the extended digits
  Tmp acc(c.pool, m * acc_words);
  bool shared = !hoisted;
  for (int i = 1; i < m && shared; ++i) shared = job.item[i].key == job.item[0].key;
  {
    InnerArgs a{};
    a.dt = dt.p;
    a.dt_stride = hoisted ? 0 : dt_words;
    a.in = in;
    a.in_stride = hoisted ? 0 : in_stride;
    a.acc = acc.p;
    a.acc_stride = acc_words;
    for (int i = 0; i < MAX_BATCH; ++i) a.key[i] = reinterpret_cast<const double*>(i < m ? job.item[i].key : nullptr);
    a.wg_per_row = colgroups;
    a.groups = ext * colgroups;
    a.batch = m;
    a.l = l;
    a.ext = ext;
    a.alpha = c.alpha;
    a.beta = beta;
    a.num_q = c.num_q;
    a.nprimes = c.nprimes;
    c.begin_launch();
    hipLaunchKernelGGL(ks_inner_kernel, ks_grid(a.groups, m), dim3(NTT_THREADS), 0, c.stream, a,
                       c.d_twd_fwd, c.d_twd_inv, c.d_fpm, c.log_n);
    // reads the extended digits (beta ext rows per input) and 2 beta ext key rows per item (once for a shared
    // key), writes 2 ext rows per item
    c.end_launch(KC_KS_INNER, 8.0 * n * ((double)m_in * beta * ext + (shared ? 1.0 : (double)m) * 2.0 * beta * ext +
                                      (double)m * 2.0 * ext));
  }

  // 4. ModDown's conversion between the strided passes, one launch
  Tmp conv(c.pool, m * conv_words);
  {
    ConvArgs a{};
    a.src = acc.p;
    a.src_stride = acc_words;
    a.dst = conv.p;
    a.dst_stride = conv_words;
    a.targets = ct_rows.d;
    for (int p = 0; p < 2; ++p) {
      a.first[p] = p * l;
      a.count[p] = l;
      a.nsrc[p] = c.num_p;
      a.src_row0[p] = p * ext + l;
    }
    a.scale = c.d_moddown_scale;
    a.moddown = c.d_moddown;
    a.num_q = c.num_q;
    a.tpt = c.tune.tpt_moddown > 0 ? std::min(c.tune.tpt_moddown, l) : targets_per_task(c, l, 2, m);
    a.tasks_per_group = (l + a.tpt - 1) / a.tpt;
    a.colgroups = colgroups;
    a.groups = 2 * a.tasks_per_group * colgroups;
    a.batch = m;
    launch_conv<KIND_MODDOWN>(c, a, c.num_p, m);
    // reads the 2K special rows, writes 2l rows
    c.end_launch(KC_KS_MODDOWN, 8.0 * n * m * (2.0 * c.num_p + 2.0 * l));
  }

  // 5. the forward contiguous pass of the conversion rows, and the combine (acc_Q - conv) P^-1 + addends
  NttEpilogue epi;
  epi.a = acc.p;
  epi.a_stride = acc_words;
  epi.a_poly_rows = ext;
  epi.a_dbl = 1;
  epi.l = l;
  epi.cst = device_field<u64>(c.d_moddown, offsetof(ModDownTab, pinv));
  epi.out = job.out;
  epi.out_stride = job.out_stride;
  epi.add0 = job.add0;
  epi.add0_stride = job.add0_stride;
  epi.gather = job.add0_galois ? 1 : 0;
  epi.add1 = job.add1;
  epi.add1_stride = job.add1_stride;
  epi.addx = job.addx;
  epi.addx_stride = job.addx_stride;
  if (job.tensor) {
    epi.tensor = 1;
    for (int i = 0; i < MAX_BATCH; ++i) {
      epi.ta[i] = i < m ? job.ta[i] : nullptr;
      epi.tb[i] = i < m ? job.tb[i] : nullptr;
    }
  }
  const u32 two_n = 2u * (u32)c.n;
  for (int i = 0; i < MAX_BATCH; ++i) {
    const u32 g = i < m ? job.item[i].g : 1;
    epi.g[i] = g;
    epi.ginv[i] = galois_inverse(g, two_n);
    if (job.top_out && g != 1) fail(HETAL_E_INVALID_ARG, "the rescale's first pass needs items without a permutation");
  }
  if (job.top_out) {
    epi.top_out = job.top_out;
    epi.top_out_stride = 2 * n;
    epi.top_prime = level;
    epi.tw_inv = c.d_twd_inv;
  }
  ntt_forward_last_pass(c, conv, conv_words, m, ct_rows, epi);
  // limb transforms: c1 and the ModUp rows, the special rows and the ModDown rows
  c.counters[6] += (int64_t)m_in * beta * ext + (int64_t)m * 2 * (c.num_p + l);
  c.counters[5] += m;
  c.ks_items[level] += m;
  c.ks_key_reads[level] += shared ? 1 : m;
}

// A rescale (Sec. 2.2) of `batch` ciphertexts at `level`: out = (in - [in_level]_centred) q_level^-1 over
// q_0 .. q_{level-1} (with kconst: the same of in times the constant K, K in = [K_i in_i]_i; an input at a higher
// level is taken at `level`; with addx, plus that addend; with pts, of in times the item's plaintext), in three
// launches (two when a key switch's epilogue has run the first) -- ModDown's pipeline with the single source prime q_level: the inverse
// NTT's contiguous pass over the two top rows; one conversion launch (the inverse strided pass, the centred lift
// to every q_i, the forward strided pass); the forward contiguous pass with the combine epilogue.
void k_rescale(Context& c, const u64* in, u64* out, int level, int batch, size_t in_stride, size_t out_stride,
               const u64* kconst, int in_poly_rows, const u64* addx, size_t addx_stride, const u64* top_ready,
               const u64* const* pts) {
  if (pts && (kconst || top_ready)) fail(HETAL_E_INVALID_ARG, "rescale: a plaintext product with another fusion");
  const size_t n = c.n;
  const int prow = in_poly_rows > 0 ? in_poly_rows : level + 1;
  // the top row's inverse transform ends with N^-1 (times the constant's residue mod q_level)
  NttScale top_scale;
  {
    const u64 qt = c.primes[level];
    const u64 kt = kconst ? kconst[level] : 1;
    top_scale.s0 = (u64)((unsigned __int128)c.h_pc[level].ninv * kt % qt);
    top_scale.s1 = (u64)((unsigned __int128)c.h_pc[level].w1ninv * kt % qt);
    top_scale.s0_sh = top_scale.s1_sh = 0;  // the FP64 passes use no Shoup companions
  }
  const int colgroups = std::max(1, c.n / 4096);
  for (int first = 0; first < batch; first += MAX_BATCH) {
    const int m = std::min(MAX_BATCH, batch - first);
    const u64* in_m = in + (size_t)first * in_stride;
    u64* out_m = out + (size_t)first * out_stride;
    NttEpilogue ptm;  // the plaintexts of a fused CMult, if any
    if (pts) {
      ptm.pt_mul = 1;
      for (int i = 0; i < MAX_BATCH; ++i) ptm.ta[i] = i < m ? pts[first + i] : nullptr;
    }
    std::unique_ptr<Tmp> top;
    if (!top_ready) {
      top.reset(new Tmp(c.pool, (size_t)m * 2 * n));
      NttSrc src;
      src.p = in_m;
      src.batch_stride = in_stride;
      src.row_mul = prow;  // top row of poly p: p prow + level
      src.row_add = level;
      if (pts)
        ntt_inverse_first_pass_pt(c, top->p, 2 * n, m, c.rows(ROWS_TOP, level), src, ptm);
      else
        ntt_inverse_first_pass(c, top->p, 2 * n, m, c.rows(ROWS_TOP, level), src);
    }
    const size_t conv_words = 2 * (size_t)level * n;
    Tmp conv(c.pool, (size_t)m * conv_words);
    RowsRef out_rows = c.rows(ROWS_CT, level - 1);
    {
      ConvArgs a{};
      a.src = top_ready ? top_ready + (size_t)first * 2 * n : top->p;
      a.src_stride = 2 * n;
      a.dst = conv.p;
      a.dst_stride = conv_words;
      a.targets = out_rows.d;
      for (int p = 0; p < 2; ++p) {
        a.first[p] = p * level;
        a.count[p] = level;
        a.nsrc[p] = 1;
        a.src_row0[p] = p;
      }
      a.scale_v = top_scale;
      a.src_prime = level;
      a.num_q = c.num_q;
      a.tpt = c.tune.tpt_moddown > 0 ? std::min(c.tune.tpt_moddown, level) : targets_per_task(c, level, 2, m);
      // one source row: a task recomputes a single inverse pass per target, so where the heuristic settles for
      // the smallest tasks (small launches) one target per task spreads the launch over more workgroups
      if (c.tune.tpt_moddown <= 0 && a.tpt <= 2) a.tpt = 1;
      a.tasks_per_group = (level + a.tpt - 1) / a.tpt;
      a.colgroups = colgroups;
      a.groups = 2 * a.tasks_per_group * colgroups;
      a.batch = m;
      launch_conv<KIND_RESCALE>(c, a, 1, m);
      // reads the two top rows, writes 2 level rows
      c.end_launch(KC_RESCALE, 8.0 * n * m * (2.0 + 2.0 * level));
    }
    NttEpilogue epi;
    epi.a = in_m;
    epi.a_stride = in_stride;
    epi.a_poly_rows = prow;
    epi.l = level;
    epi.cst = device_field<u64>(c.d_rescale + level, offsetof(RescaleTab, inv));
    epi.out = out_m;
    epi.out_stride = out_stride;
    if (kconst) {
      epi.a_mul = 1;
      for (int i = 0; i < level; ++i) epi.a_k[i] = kconst[i];
    }
    if (addx) {
      epi.addx = addx + (size_t)first * addx_stride;
      epi.addx_stride = addx_stride;
    }
    if (pts) {
      epi.pt_mul = 1;
      for (int i = 0; i < MAX_BATCH; ++i) epi.ta[i] = ptm.ta[i];
    }
    for (int i = 0; i < MAX_BATCH; ++i) epi.g[i] = epi.ginv[i] = 1;
    ntt_forward_last_pass(c, conv, conv_words, m, out_rows, epi);
  }
  c.counters[4] += batch;
}

}  // namespace hetal
