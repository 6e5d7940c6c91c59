// Host-side set-up of a context: the primes, roots of unity and every
// constant table the kernels read, and the device memory pool.
#include <algorithm>
#include <cstring>

#include "hetal_internal.hpp"

namespace hetal {

void make_roots(Context& c);

namespace {

typedef unsigned __int128 u128;

u64 mulm(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }

u64 powm(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = mulm(r, a, q);
    a = mulm(a, a, q);
  }
  return r;
}

u64 invm(u64 a, u64 q) { return powm(a, q - 2, q); }

// Miller-Rabin with the prime bases up to 37: deterministic below 2^64.
bool is_prime(u64 n) {
  if (n < 2) return false;
  const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (u64 p : bases) {
    if (n % p == 0) return n == p;
  }
  u64 d = n - 1;
  int s = 0;
  while (!(d & 1)) {
    d >>= 1;
    ++s;
  }
  for (u64 a : bases) {
    u64 x = powm(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool witness = true;
    for (int r = 1; r < s && witness; ++r) {
      x = mulm(x, x, n);
      if (x == n - 1) witness = false;
    }
    if (witness) return false;
  }
  return true;
}

// Largest `count` primes p < bound with p = 1 mod m, descending.
std::vector<u64> primes_below(u64 bound, u64 m, int count) {
  std::vector<u64> out;
  u64 p = (bound - 1) - ((bound - 1) % m) + 1;
  if (p >= bound) p -= m;
  while ((int)out.size() < count && p > m) {
    if (is_prime(p)) out.push_back(p);
    p -= m;
  }
  if ((int)out.size() < count) fail(HETAL_E_PARAMS, "not enough NTT-friendly primes");
  return out;
}

// A primitive 2N-th root of unity: x^((q-1)/2N) for the first x whose N-th power of that is -1.
u64 root_2n(u64 q, int log_n) {
  const u64 m = 2ull << log_n;
  for (u64 x = 2;; ++x) {
    u64 r = powm(x, (q - 1) / m, q);
    if (powm(r, m / 2, q) == q - 1) return r;
  }
}

u64 shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

u32 brev(u32 x, int bits) {
  u32 r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

template <typename T>
T* upload(const T* h, size_t count, hipStream_t s) {
  T* d = nullptr;
  if (hipMalloc(&d, count * sizeof(T)) != hipSuccess) fail(HETAL_E_OOM, "device allocation of constant tables");
  HCHECK(hipMemcpyAsync(d, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}

}  // namespace

// ---------------------------------------------------------------- Pool

void Pool::arena_begin(u64* base, size_t words) {
  arena_ = base;
  arena_words_ = words;
  arena_top_ = 0;
  arena_marks_.clear();
}

void Pool::arena_end() {
  arena_ = nullptr;
  arena_words_ = 0;
  arena_top_ = 0;
  arena_marks_.clear();
}

// Buffers come in size classes (a multiple of an eighth of the size's power of two), and a request takes the
// smallest free buffer of at least its class and at most twice it (only its own class with exact_fit): the varied
// sizes of chunked work reuse each other's buffers instead of piling up in the free list.
static size_t size_class(size_t words) {
  size_t top = 1;
  while (top * 2 <= words) top *= 2;
  const size_t unit = std::max<size_t>(1, top / 8);
  return (words + unit - 1) / unit * unit;
}

u64* Pool::get(size_t words) {
  if (arena_) {
    const size_t need = arena_round(words);
    if (need > arena_words_ - arena_top_)
      fail(HETAL_E_INVALID_ARG, "scratch region exhausted: " + std::to_string(need * 8) + " more bytes needed, " +
                                    std::to_string((arena_words_ - arena_top_) * 8) + " left");
    u64* p = arena_ + arena_top_;
    arena_marks_.push_back(arena_top_);
    arena_top_ += need;
    return p;
  }
  words = size_class(words);
  auto it = exact_fit ? free_.find(words) : free_.lower_bound(words);
  if (it != free_.end() && (exact_fit || it->first <= 2 * words)) {
    u64* p = it->second;
    free_.erase(it);
    return p;
  }
  if (recording) fail(HETAL_E_DEVICE, "a recorded graph needs a buffer size the pool does not hold");
  u64* p = nullptr;
  if (hipMalloc(&p, words * sizeof(u64)) != hipSuccess) {
    (void)hipGetLastError();
    release_all();
    if (hipMalloc(&p, words * sizeof(u64)) != hipSuccess) {
      (void)hipGetLastError();
      fail(HETAL_E_OOM, "device pool allocation of " + std::to_string(words * 8) + " bytes");
    }
  }
  size_of_[p] = words;
  held_ += words * 8;
  return p;
}

void Pool::put(u64* p) {
  if (arena_) {
    if (!arena_marks_.empty() && p == arena_ + arena_marks_.back()) {
      arena_top_ = arena_marks_.back();
      arena_marks_.pop_back();
    }
    return;
  }
  auto it = size_of_.find(p);
  if (it == size_of_.end()) return;
  free_.emplace(it->second, p);
}

void Pool::release_all() {
  // Only buffers sitting in the free list are released; leased ones stay valid.
  (void)hipDeviceSynchronize();
  for (auto& kv : free_) {
    (void)hipFree(kv.second);
    held_ -= size_of_[kv.second] * 8;
    size_of_.erase(kv.second);
  }
  free_.clear();
}

Pool::~Pool() {
  for (auto& kv : size_of_) (void)hipFree(kv.first);
}

// ---------------------------------------------------------------- Context

void context_init(Context& c, const hetal_params& p, hipStream_t stream) {
  if (p.log_n < 12 || p.log_n > 16) fail(HETAL_E_PARAMS, "log_n must be in [12, 16]");
  if (p.num_q < 1 || p.num_p < 1 || p.num_p > MAX_K || p.dnum < 1 || p.num_q + p.num_p > MAX_PRIMES)
    fail(HETAL_E_PARAMS, "prime counts out of range");
  if (p.q0_bits < 20 || p.q0_bits > 50 || p.q_bits < 20 || p.q_bits > 50) fail(HETAL_E_PARAMS, "prime sizes out of range");
  c.log_n = p.log_n;
  c.n = 1 << p.log_n;
  c.slots = c.n / 2;
  c.num_q = p.num_q;
  c.num_p = p.num_p;
  c.dnum = p.dnum;
  c.alpha = (p.num_q + p.dnum - 1) / p.dnum;
  // the key switch's fused conversions hold one inverse-transformed row per term in registers (keyswitch.hip)
  if (c.alpha > MAX_FUSED_CONV || c.num_p > MAX_FUSED_CONV)
    fail(HETAL_E_PARAMS, "more than 4 primes per digit or special primes");
  if ((c.num_q + c.alpha - 1) / c.alpha > 8) fail(HETAL_E_PARAMS, "more than 8 digits");
  c.nprimes = p.num_q + p.num_p;
  c.stream = stream;

  const u64 m = 2ull << p.log_n;
  std::vector<u64> q0 = primes_below(1ull << p.q0_bits, m, 1);
  std::vector<u64> rest = p.num_q > 1 ? primes_below(1ull << p.q_bits, m, p.num_q - 1) : std::vector<u64>();
  std::vector<u64> sp = primes_below(q0[0], m, p.num_p);
  c.primes.clear();
  c.primes.push_back(q0[0]);
  c.primes.insert(c.primes.end(), rest.begin(), rest.end());
  c.primes.insert(c.primes.end(), sp.begin(), sp.end());
  for (size_t i = 0; i < c.primes.size(); ++i)
    for (size_t k = i + 1; k < c.primes.size(); ++k)
      if (c.primes[i] == c.primes[k]) fail(HETAL_E_PARAMS, "prime lists overlap (q0_bits == q_bits?)");

  const int np = c.nprimes, n = c.n;
  // modulus constants
  std::vector<ModInfo> mods(np);
  for (int i = 0; i < np; ++i) {
    const u64 q = c.primes[i];
    int b = 63 - __builtin_clzll(q);
    mods[i].q = q;
    mods[i].b = b;
    mods[i].mu = (u64)(((u128)1 << (b + 64)) / q);
    mods[i].one_sh = (u64)(((u128)1 << 64) / q);
    mods[i].pad = 0;
  }
  // twiddles and per-prime constants
  std::vector<double> twdf((size_t)np * n), twdi((size_t)np * n);
  c.h_pc.assign(np, PrimeConsts{});
  for (int i = 0; i < np; ++i) {
    const u64 q = c.primes[i];
    const u64 psi = root_2n(q, c.log_n);
    const u64 psi_inv = invm(psi, q);
    std::vector<u64> pw(n), pwi(n);
    pw[0] = pwi[0] = 1;
    for (int k = 1; k < n; ++k) {
      pw[k] = mulm(pw[k - 1], psi, q);
      pwi[k] = mulm(pwi[k - 1], psi_inv, q);
    }
    for (int x = 0; x < n; ++x) {
      const u64 wf = pw[brev((u32)x, c.log_n)], wi = pwi[brev((u32)x, c.log_n)];
      const size_t at = (size_t)i * n + ntt_twiddle_slot(x, c.log_n);
      twdf[at] = (double)wf;
      twdi[at] = (double)wi;
    }
    PrimeConsts& k = c.h_pc[i];
    k.ninv = invm((u64)n % q, q);
    k.ninv_sh = shoup(k.ninv, q);
    k.w1ninv = mulm(pwi[n / 2], k.ninv, q);  // psi^-brev(1) = psi^-(N/2)
    k.w1ninv_sh = shoup(k.w1ninv, q);
    k.iq = pw[n / 2];
    k.iq_sh = shoup(k.iq, q);
    u64 pm = 1;
    for (int t = 0; t < c.num_p; ++t) pm = mulm(pm, c.primes[c.num_q + t] % q, q);
    k.pmod = i < c.num_q ? pm : 0;
    k.pmod_sh = shoup(k.pmod, q);
  }

  // ModUp tables: [level][digit]
  c.h_modup.assign((size_t)c.num_q * c.dnum, ModUpTab{});
  for (int lv = 0; lv < c.num_q; ++lv) {
    const int l = lv + 1;
    for (int j = 0; j < c.dnum; ++j) {
      ModUpTab& tb = c.h_modup[(size_t)lv * c.dnum + j];
      std::memset(&tb, 0, sizeof(tb));
      tb.first = j * c.alpha;
      tb.nsrc = std::max(0, std::min(c.alpha, l - tb.first));
      for (int i = 0; i < tb.nsrc; ++i) {
        const u64 di = c.primes[tb.first + i];
        u64 prod = 1;
        for (int k = 0; k < tb.nsrc; ++k)
          if (k != i) prod = mulm(prod, c.primes[tb.first + k] % di, di);
        tb.dinv[i] = invm(prod, di);
        tb.dinv_sh[i] = shoup(tb.dinv[i], di);
        for (int t = 0; t < np; ++t) {
          const u64 qt = c.primes[t];
          u64 h = 1;
          for (int k = 0; k < tb.nsrc; ++k)
            if (k != i) h = mulm(h, c.primes[tb.first + k] % qt, qt);
          tb.dhat[i][t] = h;
          tb.dhat_sh[i][t] = shoup(h, qt);
        }
      }
    }
  }
  // ModDown table
  std::memset(&c.h_moddown, 0, sizeof(c.h_moddown));
  c.h_moddown.k = c.num_p;
  for (int k = 0; k < c.num_p; ++k) {
    const u64 pk = c.primes[c.num_q + k];
    u64 prod = 1;
    for (int t = 0; t < c.num_p; ++t)
      if (t != k) prod = mulm(prod, c.primes[c.num_q + t] % pk, pk);
    c.h_moddown.pkinv[k] = invm(prod, pk);
    c.h_moddown.pkinv_sh[k] = shoup(c.h_moddown.pkinv[k], pk);
    for (int i = 0; i < c.num_q; ++i) {
      const u64 qi = c.primes[i];
      u64 h = 1;
      for (int t = 0; t < c.num_p; ++t)
        if (t != k) h = mulm(h, c.primes[c.num_q + t] % qi, qi);
      c.h_moddown.phat[k][i] = h;
      c.h_moddown.phat_sh[k][i] = shoup(h, qi);
    }
  }
  for (int i = 0; i < c.num_q; ++i) {
    const u64 qi = c.primes[i];
    c.h_moddown.pinv[i] = invm(c.h_pc[i].pmod, qi);
    c.h_moddown.pinv_sh[i] = shoup(c.h_moddown.pinv[i], qi);
  }
  // Final inverse-NTT scalings that leave the (D_j/d_i)^-1 or (P/p_k)^-1 factors of the conversions applied
  auto scaled = [&](int prime, u64 f) {
    const u64 q = c.primes[prime];
    NttScale s;
    s.s0 = mulm(c.h_pc[prime].ninv, f, q);
    s.s0_sh = shoup(s.s0, q);
    s.s1 = mulm(c.h_pc[prime].w1ninv, f, q);
    s.s1_sh = shoup(s.s1, q);
    return s;
  };
  std::vector<NttScale> up_scale((size_t)c.num_q * MAX_PRIMES, NttScale{0, 0, 0, 0});
  for (int lv = 0; lv < c.num_q; ++lv)
    for (int i = 0; i <= lv; ++i) {
      const ModUpTab& tb = c.h_modup[(size_t)lv * c.dnum + i / c.alpha];
      up_scale[(size_t)lv * MAX_PRIMES + i] = scaled(i, tb.dinv[i % c.alpha]);
    }
  std::vector<NttScale> down_scale(2 * (size_t)c.num_p);
  for (int pp = 0; pp < 2; ++pp)
    for (int k = 0; k < c.num_p; ++k) down_scale[(size_t)pp * c.num_p + k] = scaled(c.num_q + k, c.h_moddown.pkinv[k]);
  // Rescale tables
  std::vector<RescaleTab> resc(c.num_q);
  for (int lv = 0; lv < c.num_q; ++lv) {
    std::memset(&resc[lv], 0, sizeof(RescaleTab));
    for (int i = 0; i < lv; ++i) {
      const u64 qi = c.primes[i];
      resc[lv].inv[i] = invm(c.primes[lv] % qi, qi);
      resc[lv].inv_sh[i] = shoup(resc[lv].inv[i], qi);
    }
  }
  // 5^k mod 2N
  std::vector<u32> pow5(c.slots);
  u64 e = 1;
  for (int k = 0; k < c.slots; ++k) {
    pow5[k] = (u32)e;
    e = e * 5 % m;
  }
  // Row tables, per level
  std::vector<int2> rows;
  for (int t = 0; t < NUM_ROW_TABLES; ++t) {
    c.row_off[t].assign(c.num_q, 0);
    c.row_cnt[t].assign(c.num_q, 0);
  }
  auto begin = [&](RowTable t, int lv) { c.row_off[t][lv] = (int)rows.size(); };
  auto end = [&](RowTable t, int lv) { c.row_cnt[t][lv] = (int)rows.size() - c.row_off[t][lv]; };
  for (int lv = 0; lv < c.num_q; ++lv) {
    const int l = lv + 1, ext = l + c.num_p;
    begin(ROWS_CT, lv);
    for (int pp = 0; pp < 2; ++pp)
      for (int i = 0; i < l; ++i) rows.push_back(make_int2(pp * l + i, i));
    end(ROWS_CT, lv);
    begin(ROWS_MODUP, lv);
    for (int j = 0; j < c.beta(lv); ++j) {
      const int first = j * c.alpha, last = std::min(first + c.alpha, l);
      for (int r = 0; r < ext; ++r) {
        if (r >= first && r < last) continue;
        rows.push_back(make_int2(j * ext + r, c.ext_prime(lv, r)));
      }
    }
    end(ROWS_MODUP, lv);
    begin(ROWS_SPECIAL, lv);
    for (int pp = 0; pp < 2; ++pp)
      for (int k = 0; k < c.num_p; ++k) rows.push_back(make_int2(pp * ext + l + k, c.num_q + k));
    end(ROWS_SPECIAL, lv);
    begin(ROWS_TOP, lv);
    for (int pp = 0; pp < 2; ++pp) rows.push_back(make_int2(pp, lv));
    end(ROWS_TOP, lv);
    begin(ROWS_ALL, lv);
    for (int i = 0; i < np; ++i) rows.push_back(make_int2(i, i));
    end(ROWS_ALL, lv);
    begin(ROWS_ALL2, lv);
    for (int pp = 0; pp < 2; ++pp)
      for (int i = 0; i < np; ++i) rows.push_back(make_int2(pp * np + i, i));
    end(ROWS_ALL2, lv);
    begin(ROWS_EXT, lv);
    for (int r = 0; r < ext; ++r) rows.push_back(make_int2(r, c.ext_prime(lv, r)));
    end(ROWS_EXT, lv);
  }

  c.d_mod = upload(mods.data(), mods.size(), stream);
  c.d_twd_fwd = upload(twdf.data(), twdf.size(), stream);
  c.d_twd_inv = upload(twdi.data(), twdi.size(), stream);
  std::vector<FpMod> fpm(np);
  for (int i = 0; i < np; ++i) fpm[i] = FpMod{(double)c.primes[i], 1.0 / (double)c.primes[i]};
  c.d_fpm = upload(fpm.data(), fpm.size(), stream);
  c.d_pc = upload(c.h_pc.data(), c.h_pc.size(), stream);
  c.d_modup = upload(c.h_modup.data(), c.h_modup.size(), stream);
  c.d_moddown = upload(&c.h_moddown, 1, stream);
  c.d_rescale = upload(resc.data(), resc.size(), stream);
  c.d_modup_scale = upload(up_scale.data(), up_scale.size(), stream);
  c.d_moddown_scale = upload(down_scale.data(), down_scale.size(), stream);
  c.d_pow5 = upload(pow5.data(), pow5.size(), stream);
  c.d_rows = upload(rows.data(), rows.size(), stream);
  if (hipMalloc(&c.d_roots, (size_t)m * 4 * sizeof(double)) != hipSuccess) fail(HETAL_E_OOM, "roots table");
  make_roots(c);
  HCHECK(hipStreamSynchronize(stream));
}

void context_share(Context& d, const Context& s, hipStream_t stream) {
  d.log_n = s.log_n;
  d.n = s.n;
  d.slots = s.slots;
  d.num_q = s.num_q;
  d.num_p = s.num_p;
  d.dnum = s.dnum;
  d.alpha = s.alpha;
  d.nprimes = s.nprimes;
  d.primes = s.primes;
  d.stream = stream;
  d.d_mod = s.d_mod;
  d.d_twd_fwd = s.d_twd_fwd;
  d.d_twd_inv = s.d_twd_inv;
  d.d_fpm = s.d_fpm;
  d.d_pc = s.d_pc;
  d.d_modup = s.d_modup;
  d.d_moddown = s.d_moddown;
  d.d_modup_scale = s.d_modup_scale;
  d.d_moddown_scale = s.d_moddown_scale;
  d.d_rescale = s.d_rescale;
  d.d_roots = s.d_roots;
  d.d_pow5 = s.d_pow5;
  d.d_rows = s.d_rows;
  for (int t = 0; t < NUM_ROW_TABLES; ++t) {
    d.row_off[t] = s.row_off[t];
    d.row_cnt[t] = s.row_cnt[t];
  }
  d.h_modup = s.h_modup;
  d.h_moddown = s.h_moddown;
  d.h_pc = s.h_pc;
  d.owns_tables = false;
}

void context_free(Context& c) {
  if (c.stream) (void)hipStreamSynchronize(c.stream);
  else (void)hipDeviceSynchronize();
  if (c.d_gauss) (void)hipFree(c.d_gauss);  // each context's own (made on first use)
  c.d_gauss = nullptr;
  if (!c.owns_tables) return;
  void* ptrs[] = {c.d_mod,     c.d_pc,     c.d_modup,  c.d_moddown,
                  c.d_rescale, c.d_roots,  c.d_pow5,   c.d_rows, c.d_modup_scale, c.d_moddown_scale,
                  c.d_twd_fwd, c.d_twd_inv, c.d_fpm};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

}  // namespace hetal
