// extern "C" entry points: argument validation, error translation, and the
// host <-> device transfers of the client-side calls.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "handles.hpp"
#include "sampler.hpp"
#include "softmax.hpp"

using namespace hetal;

namespace {

// Host -> device upload into a pool buffer.  The stream is drained first, so a
// pool buffer that queued kernels still read is never overwritten by a copy
// from pageable memory, whatever ordering the runtime gives such copies.
Tmp upload_words(Context& c, const void* host, size_t bytes) {
  Tmp t(c.pool, (bytes + 7) / 8);
  HCHECK(hipStreamSynchronize(c.stream));
  HCHECK(hipMemcpyAsync(t.p, host, bytes, hipMemcpyHostToDevice, c.stream));
  return t;
}

// The transforms take residues in [0, q): caller-supplied uniform randomness is checked on the host
// ([count][rows][N], row i modulo primes[i]).
static void check_uniform(const Context& c, const uint64_t* host, int count, int rows) {
  for (int b = 0; b < count; ++b)
    for (int i = 0; i < rows; ++i) {
      const uint64_t* r = host + ((size_t)b * rows + i) * c.n;
      const uint64_t q = c.primes[i];
      bool ok = true;
      for (int k = 0; k < c.n; ++k) ok &= r[k] < q;
      need(ok, HETAL_E_INVALID_ARG, "uniform randomness not reduced modulo its prime");
    }
}

// NTT form of coefficient-form randomness already on the device: a ([count][l][N], residues, transformed in
// place) and e ([count][N], signed, reduced into en [count][l][N]).
void randomness_to_ntt(Context& c, u64* a, const i64* ecoef, int level, int count, u64* en) {
  const size_t poly = c.poly_words(level);
  RowsRef rows = c.rows(ROWS_CT, level);
  RowsRef first{rows.d, level + 1};
  ntt_forward(c, a, poly, count, first);
  k_reduce_signed(c, ecoef, en, first, count, c.n, poly);
  ntt_forward(c, en, poly, count, first);
}

// NTT form of caller-supplied coefficient-form randomness a ([count][l][N]) and e ([count][N]).
void load_randomness(Context& c, const uint64_t* a_host, const int64_t* e_host, int level, int count, Tmp& a, Tmp& e) {
  check_uniform(c, a_host, count, level + 1);
  const size_t poly = c.poly_words(level);
  HCHECK(hipStreamSynchronize(c.stream));
  HCHECK(hipMemcpyAsync(a.p, a_host, (size_t)count * poly * 8, hipMemcpyHostToDevice, c.stream));
  Tmp ecoef = upload_words(c, e_host, (size_t)count * c.n * 8);
  randomness_to_ntt(c, a, reinterpret_cast<const i64*>(ecoef.p), level, count, e);
  HCHECK(hipStreamSynchronize(c.stream));
}

// The library's own randomness for encryptions index .. index + count - 1 at `level` (sampler.hip), in NTT form.
void sample_randomness(Context& c, u64 seed, u32 index, int level, int count, Tmp& a, Tmp& e) {
  const size_t poly = c.poly_words(level);
  Tmp ecoef(c.pool, (size_t)count * c.n);
  for (int b = 0; b < count; ++b) {
    sample_uniform(c, seed, PURPOSE_ENC_A, index + (u32)b, level + 1, level + 1, a.p + b * poly);
    sample_gaussian(c, seed, PURPOSE_ENC_E, index + (u32)b, 1, reinterpret_cast<i64*>(ecoef.p) + b * c.n);
  }
  randomness_to_ntt(c, a, reinterpret_cast<const i64*>(ecoef.p), level, count, e);
}

}  // namespace

extern "C" {

const char* hetal_last_error(void) { return g_last_error.c_str(); }

int hetal_ctx_create(const hetal_params* params, void* stream, hetal_ctx** out) {
  return guarded([&] {
    need(params && out, HETAL_E_INVALID_ARG, "null argument");
    hetal_ctx* h = new hetal_ctx();
    try {
      HCHECK(hipGetDevice(&h->device));
      scratch_setup();
      context_init(h->c, *params, (hipStream_t)stream);
    } catch (...) {
      context_free(h->c);
      delete h;
      throw;
    }
    h->masks.c = &h->c;
    *out = h;
  });
}

int hetal_ctx_create_shared(hetal_ctx* base, void* stream, hetal_ctx** out) {
  return guarded([&] {
    need(base && out, HETAL_E_INVALID_ARG, "null argument");
    hetal_ctx* h = new hetal_ctx();
    h->device = base->device;
    context_share(h->c, base->c, (hipStream_t)stream);
    h->masks.c = &h->c;
    h->tuned = base->tuned;  // the schedules chosen so far (later tuning of either context stays its own)
    h->two_streams = base->two_streams;
    *out = h;
  });
}

int hetal_ctx_set_two_streams(hetal_ctx* ctx, int enable) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    ctx->two_streams = enable != 0;
  });
}

void hetal_ctx_destroy(hetal_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->c.stream);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side_stream);
    for (auto& kv : ctx->side_masks.pts) ctx->side->pool.put(kv.second);
    ctx->side_masks.pts.clear();
    context_free(*ctx->side);
    ctx->side.reset();
    (void)hipStreamDestroy(ctx->side_stream);
    for (hipEvent_t e : ctx->join) (void)hipEventDestroy(e);
  }
  for (auto& kv : ctx->masks.pts) ctx->c.pool.put(kv.second);
  ctx->masks.pts.clear();
  for (auto& t : ctx->c.timed) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (auto e : ctx->c.ev_free) (void)hipEventDestroy(e);
  context_free(ctx->c);
  delete ctx;
}

int hetal_ctx_set_stream(hetal_ctx* ctx, void* stream) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    HCHECK(hipStreamSynchronize(ctx->c.stream));
    ctx->c.stream = (hipStream_t)stream;
  });
}

int hetal_ctx_info(const hetal_ctx* ctx, int* n, int* slots, int* max_level, int* num_primes) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    if (n) *n = ctx->c.n;
    if (slots) *slots = ctx->c.slots;
    if (max_level) *max_level = ctx->c.num_q - 1;
    if (num_primes) *num_primes = ctx->c.nprimes;
  });
}

int hetal_ctx_primes(const hetal_ctx* ctx, uint64_t* out) {
  return guarded([&] {
    need(ctx && out, HETAL_E_INVALID_ARG, "null argument");
    std::memcpy(out, ctx->c.primes.data(), ctx->c.primes.size() * 8);
  });
}

int hetal_synchronize(hetal_ctx* ctx) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    HCHECK(hipStreamSynchronize(ctx->c.stream));
  });
}

uint64_t hetal_galois_rot(const hetal_ctx* ctx, int r) { return ctx ? galois_rot(ctx->c, r) : 0; }
uint64_t hetal_galois_conj(const hetal_ctx* ctx) { return ctx ? galois_conj(ctx->c) : 0; }

static hetal_sk* sk_from_coeffs(hetal_ctx* ctx, const int64_t* s_coeffs) {
  Context& c = ctx->c;
  for (int k = 0; k < c.n; ++k) need(s_coeffs[k] >= -1 && s_coeffs[k] <= 1, HETAL_E_INVALID_ARG, "secret must be ternary");
  u64* s = nullptr;
  if (hipMalloc(&s, (size_t)c.nprimes * c.n * 8) != hipSuccess) fail(HETAL_E_OOM, "secret key allocation");
  Tmp coef = upload_words(c, s_coeffs, (size_t)c.n * 8);
  RowsRef all = c.rows(ROWS_ALL, 0);
  k_reduce_signed(c, reinterpret_cast<const i64*>(coef.p), s, all, 1, 0, 0);
  ntt_forward(c, s, 0, 1, all);
  HCHECK(hipStreamSynchronize(c.stream));
  return new hetal_sk{ctx, SecretKeyDev{s}};
}

int hetal_sk_create(hetal_ctx* ctx, const int64_t* s_coeffs, hetal_sk** out) {
  return guarded([&] {
    need(ctx && s_coeffs && out, HETAL_E_INVALID_ARG, "null argument");
    *out = sk_from_coeffs(ctx, s_coeffs);
  });
}

int hetal_keygen(hetal_ctx* ctx, uint64_t seed, hetal_sk** out) {
  return guarded([&] {
    need(ctx && out, HETAL_E_INVALID_ARG, "null argument");
    std::vector<int64_t> s(ctx->c.n);
    sample_ternary(seed, ctx->c.log_n, std::min(SECRET_HAMMING, ctx->c.n), s.data());
    *out = sk_from_coeffs(ctx, s.data());
  });
}

void hetal_sk_destroy(hetal_sk* sk) {
  if (!sk) return;
  (void)hipStreamSynchronize(sk->ctx->c.stream);
  (void)hipFree(sk->key.s);
  delete sk;
}

int hetal_keys_create(hetal_ctx* ctx, hetal_keys** out) {
  return guarded([&] {
    need(ctx && out, HETAL_E_INVALID_ARG, "null argument");
    *out = new hetal_keys{ctx, KeySet{}};
  });
}

void hetal_keys_destroy(hetal_keys* keys) {
  if (!keys) return;
  (void)hipStreamSynchronize(keys->ctx->c.stream);
  if (keys->set.relin) (void)hipFree(keys->set.relin);
  for (auto& kv : keys->set.galois) (void)hipFree(kv.second);
  delete keys;
}

// A switching key for s' (NTT form) from coefficient-form randomness on the device: a [dnum][nprimes][N]
// (transformed in place), e [dnum][N] signed.
static u64* switch_key_from(Context& c, const u64* s, const u64* sp, u64* a, const i64* ecoef, u32 g) {
  const size_t rows_words = (size_t)c.nprimes * c.n;
  Tmp e(c.pool, (size_t)c.dnum * rows_words);
  RowsRef all = c.rows(ROWS_ALL, 0);
  ntt_forward(c, a, rows_words, c.dnum, all);
  k_reduce_signed(c, ecoef, e, all, c.dnum, c.n, rows_words);
  ntt_forward(c, e, rows_words, c.dnum, all);
  u64* key = nullptr;
  if (hipMalloc(&key, c.key_words() * 8) != hipSuccess) fail(HETAL_E_OOM, "key allocation");
  k_keygen(c, a, e, s, sp, key, g);
  HCHECK(hipStreamSynchronize(c.stream));
  return key;
}

static u64* make_switch_key(Context& c, const u64* s, const u64* sp, const uint64_t* a_host, const int64_t* e_host,
                            u32 g) {
  check_uniform(c, a_host, c.dnum, c.nprimes);
  const size_t rows_words = (size_t)c.nprimes * c.n;
  Tmp a(c.pool, (size_t)c.dnum * rows_words);
  HCHECK(hipStreamSynchronize(c.stream));
  HCHECK(hipMemcpyAsync(a.p, a_host, (size_t)c.dnum * rows_words * 8, hipMemcpyHostToDevice, c.stream));
  Tmp ecoef = upload_words(c, e_host, (size_t)c.dnum * c.n * 8);
  return switch_key_from(c, s, sp, a, reinterpret_cast<const i64*>(ecoef.p), g);
}

// s' of the key for Galois element g (1: s^2, the relinearisation key), NTT form over every prime.
static void key_target(Context& c, const hetal_sk* sk, u32 g, u64* out) {
  if (g == 1)
    k_mul_rows(c, sk->key.s, sk->key.s, out, c.nprimes, c.nprimes, c.nprimes);
  else
    k_galois(c, sk->key.s, out, c.nprimes, c.nprimes, g);
}

static void store_key(KeySet& set, u32 g, u64* key) {
  if (g == 1) {
    if (set.relin) (void)hipFree(set.relin);
    set.relin = key;
    return;
  }
  auto it = set.galois.find(g);
  if (it != set.galois.end()) (void)hipFree(it->second);
  set.galois[g] = key;
}

int hetal_keys_gen_relin(hetal_ctx* ctx, hetal_keys* keys, const hetal_sk* sk, const uint64_t* a, const int64_t* e) {
  return guarded([&] {
    need(ctx && keys && sk && a && e, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    Tmp sp(c.pool, (size_t)c.nprimes * c.n);
    key_target(c, sk, 1, sp);
    store_key(keys->set, 1, make_switch_key(c, sk->key.s, sp, a, e, 1));
  });
}

int hetal_keys_gen_galois(hetal_ctx* ctx, hetal_keys* keys, const hetal_sk* sk, uint64_t galois, const uint64_t* a,
                          const int64_t* e) {
  return guarded([&] {
    need(ctx && keys && sk && a && e, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    need(galois % 2 == 1 && galois < 2ull * c.n, HETAL_E_INVALID_ARG, "Galois element must be odd and below 2N");
    if (galois == 1) return;  // the identity needs no key
    Tmp sp(c.pool, (size_t)c.nprimes * c.n);
    key_target(c, sk, (u32)galois, sp);
    store_key(keys->set, (u32)galois, make_switch_key(c, sk->key.s, sp, a, e, (u32)galois));
  });
}

int hetal_gen_evk(hetal_ctx* ctx, hetal_keys* keys, const hetal_sk* sk, uint64_t seed, const int32_t* rot_steps,
                  int n, int conj, int relin) {
  return guarded([&] {
    need(ctx && keys && sk && n >= 0 && (n == 0 || rot_steps), HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    std::vector<u32> gal;
    if (relin) gal.push_back(1);
    for (int i = 0; i < n; ++i) {
      const u32 g = galois_rot(c, rot_steps[i]);
      if (g != 1 && std::find(gal.begin(), gal.end(), g) == gal.end()) gal.push_back(g);
    }
    if (conj) {
      const u32 g = galois_conj(c);
      if (std::find(gal.begin(), gal.end(), g) == gal.end()) gal.push_back(g);
    }
    const size_t rows_words = (size_t)c.nprimes * c.n;
    Tmp sp(c.pool, rows_words);
    Tmp a(c.pool, (size_t)c.dnum * rows_words);
    Tmp ecoef(c.pool, (size_t)c.dnum * c.n);
    for (u32 g : gal) {
      key_target(c, sk, g, sp);
      const u32 kid = g == 1 ? 0u : g;
      sample_uniform(c, seed, PURPOSE_KSK_A, kid, c.dnum * c.nprimes, c.nprimes, a);
      sample_gaussian(c, seed, PURPOSE_KSK_E, kid, c.dnum, reinterpret_cast<i64*>(ecoef.p));
      store_key(keys->set, g, switch_key_from(c, sk->key.s, sp, a, reinterpret_cast<const i64*>(ecoef.p), g));
    }
  });
}

int hetal_encode(hetal_ctx* ctx, const double* re, const double* im, int level, double scale, hetal_pt* out) {
  return guarded([&] {
    need(ctx && re && out && out->data, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    need(level >= 0 && level < c.num_q, HETAL_E_LEVEL, "level out of range");
    need(out->capacity >= c.poly_words(level), HETAL_E_INVALID_ARG, "plaintext capacity too small");
    need(scale > 0, HETAL_E_SCALE, "scale must be positive");
    Tmp dre = upload_words(c, re, (size_t)c.slots * 8);
    Tmp dim(c.pool, c.slots);
    HCHECK(hipStreamSynchronize(c.stream));
    if (im) HCHECK(hipMemcpyAsync(dim.p, im, (size_t)c.slots * 8, hipMemcpyHostToDevice, c.stream));
    encode_slots(c, reinterpret_cast<double*>(dre.p), im ? reinterpret_cast<double*>(dim.p) : nullptr, 1, 0, level,
                 scale, out->data, 0);
    out->level = level;
    out->scale = scale;
  });
}

int hetal_decode(hetal_ctx* ctx, const hetal_pt* pt, double* re, double* im) {
  return guarded([&] {
    need(ctx && re, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_pt(c, pt);
    const size_t poly = c.poly_words(pt->level);
    Tmp coef(c.pool, poly);
    HCHECK(hipMemcpyAsync(coef.p, pt->data, poly * 8, hipMemcpyDeviceToDevice, c.stream));
    RowsRef rows = c.rows(ROWS_CT, pt->level);
    ntt_inverse(c, coef, 0, 1, RowsRef{rows.d, pt->level + 1});
    Tmp out(c.pool, (size_t)c.slots * 2);
    double* dre = reinterpret_cast<double*>(out.p);
    k_decode(c, coef, pt->level, pt->scale, dre, dre + c.slots);
    HCHECK(hipMemcpyAsync(re, dre, (size_t)c.slots * 8, hipMemcpyDeviceToHost, c.stream));
    if (im) HCHECK(hipMemcpyAsync(im, dre + c.slots, (size_t)c.slots * 8, hipMemcpyDeviceToHost, c.stream));
    HCHECK(hipStreamSynchronize(c.stream));
  });
}

int hetal_encrypt(hetal_ctx* ctx, const hetal_sk* sk, const hetal_pt* pt, const uint64_t* a, const int64_t* e,
                  hetal_ct* out) {
  return guarded([&] {
    need(ctx && sk && a && e, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_pt(c, pt);
    check_out(c, out, pt->level);
    const size_t poly = c.poly_words(pt->level);
    Tmp an(c.pool, poly), en(c.pool, poly);
    load_randomness(c, a, e, pt->level, 1, an, en);
    k_encrypt(c, an, en, pt->data, sk->key.s, out->data, pt->level);
    out->level = pt->level;
    out->scale = pt->scale;
  });
}

int hetal_encrypt_seeded(hetal_ctx* ctx, const hetal_sk* sk, const hetal_pt* pt, uint64_t seed, uint32_t index,
                         hetal_ct* out) {
  return guarded([&] {
    need(ctx && sk, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_pt(c, pt);
    check_out(c, out, pt->level);
    const size_t poly = c.poly_words(pt->level);
    Tmp an(c.pool, poly), en(c.pool, poly);
    sample_randomness(c, seed, index, pt->level, 1, an, en);
    k_encrypt(c, an, en, pt->data, sk->key.s, out->data, pt->level);
    HCHECK(hipStreamSynchronize(c.stream));
    out->level = pt->level;
    out->scale = pt->scale;
  });
}

int hetal_gaussian_table(uint64_t* out, int* n) {
  return guarded([&] {
    need(out && n, HETAL_E_INVALID_ARG, "null argument");
    need(*n >= GAUSS_ENTRIES, HETAL_E_INVALID_ARG, "table needs 19 entries");
    u64 t[GAUSS_ENTRIES];
    gaussian_table(t);
    for (int j = 0; j < GAUSS_ENTRIES; ++j) out[j] = t[j];
    *n = GAUSS_ENTRIES;
  });
}

int hetal_sample_ternary(int log_n, uint64_t seed, int h, int64_t* out) {
  return guarded([&] {
    need(out && log_n >= 1 && log_n <= 30 && h >= 0, HETAL_E_INVALID_ARG, "bad argument");
    sample_ternary(seed, log_n, h, out);
  });
}

int hetal_sample_uniform(hetal_ctx* ctx, uint64_t seed, uint32_t purpose, uint32_t index, int rows, int group,
                         uint64_t* host) {
  return guarded([&] {
    need(ctx && host && rows > 0 && group > 0 && group <= ctx->c.nprimes, HETAL_E_INVALID_ARG, "bad argument");
    Context& c = ctx->c;
    Tmp d(c.pool, (size_t)rows * c.n);
    sample_uniform(c, seed, purpose, index, rows, group, d);
    HCHECK(hipMemcpyAsync(host, d.p, (size_t)rows * c.n * 8, hipMemcpyDeviceToHost, c.stream));
    HCHECK(hipStreamSynchronize(c.stream));
  });
}

int hetal_sample_gaussian(hetal_ctx* ctx, uint64_t seed, uint32_t purpose, uint32_t index, int count,
                          int64_t* host) {
  return guarded([&] {
    need(ctx && host && count > 0, HETAL_E_INVALID_ARG, "bad argument");
    Context& c = ctx->c;
    Tmp d(c.pool, (size_t)count * c.n);
    sample_gaussian(c, seed, purpose, index, count, reinterpret_cast<i64*>(d.p));
    HCHECK(hipMemcpyAsync(host, d.p, (size_t)count * c.n * 8, hipMemcpyDeviceToHost, c.stream));
    HCHECK(hipStreamSynchronize(c.stream));
  });
}

int hetal_decrypt(hetal_ctx* ctx, const hetal_sk* sk, const hetal_ct* ct, hetal_pt* out) {
  return guarded([&] {
    need(ctx && sk && out && out->data, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_ct(c, ct, "ciphertext");
    need(out->capacity >= c.poly_words(ct->level), HETAL_E_INVALID_ARG, "plaintext capacity too small");
    k_decrypt(c, ct->data, sk->key.s, out->data, ct->level);
    out->level = ct->level;
    out->scale = ct->scale;
  });
}

int hetal_add(hetal_ctx* ctx, const hetal_ct* a, const hetal_ct* b, hetal_ct* out) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    check_ct(ctx->c, a, "a");
    check_ct(ctx->c, b, "b");
    check_out(ctx->c, out, a->level);
    double s;
    op_add(ctx->c, view_of(a), view_of(b), out->data, &s, false);
    out->level = a->level;
    out->scale = s;
  });
}

int hetal_sub(hetal_ctx* ctx, const hetal_ct* a, const hetal_ct* b, hetal_ct* out) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    check_ct(ctx->c, a, "a");
    check_ct(ctx->c, b, "b");
    check_out(ctx->c, out, a->level);
    double s;
    op_add(ctx->c, view_of(a), view_of(b), out->data, &s, true);
    out->level = a->level;
    out->scale = s;
  });
}

int hetal_mul_i(hetal_ctx* ctx, const hetal_ct* a, hetal_ct* out) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    check_ct(ctx->c, a, "a");
    check_out(ctx->c, out, a->level);
    op_mul_i(ctx->c, view_of(a), out->data);
    out->level = a->level;
    out->scale = a->scale;
  });
}

int hetal_cmult(hetal_ctx* ctx, const hetal_ct* ct, const hetal_pt* pt, hetal_ct* out) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    check_ct(ctx->c, ct, "ciphertext");
    check_pt(ctx->c, pt);
    need(pt->level == ct->level, HETAL_E_LEVEL, "plaintext and ciphertext levels differ");
    check_out(ctx->c, out, ct->level);
    need(out->data != pt->data, HETAL_E_INVALID_ARG, "output must not alias the plaintext");
    op_cmult(ctx->c, view_of(ct), pt->data, out->data);
    out->level = ct->level;
    out->scale = ct->scale * pt->scale;
  });
}

int hetal_hmult(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* a, const hetal_ct* b, hetal_ct* out) {
  return guarded([&] {
    need(ctx && keys, HETAL_E_INVALID_ARG, "null argument");
    check_ct(ctx->c, a, "a");
    check_ct(ctx->c, b, "b");
    check_out(ctx->c, out, a->level);
    const double s = a->scale * b->scale;
    op_hmult(ctx->c, keys->set, view_of(a), view_of(b), out->data);
    out->level = a->level;
    out->scale = s;
  });
}

int hetal_hrot(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* ct, int r, hetal_ct* out) {
  return guarded([&] {
    need(ctx && keys, HETAL_E_INVALID_ARG, "null argument");
    check_ct(ctx->c, ct, "ciphertext");
    check_out(ctx->c, out, ct->level);
    const double s = ct->scale;
    const int lv = ct->level;
    op_galois(ctx->c, keys->set, view_of(ct), galois_rot(ctx->c, r), out->data);
    ctx->c.counters[0] += 1;
    out->level = lv;
    out->scale = s;
  });
}

int hetal_hrot_batch(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* in, const int* steps, int count,
                     hetal_ct* out) {
  return guarded([&] {
    need(ctx && keys && in && steps && out && count >= 0, HETAL_E_INVALID_ARG, "null argument");
    if (count == 0) return;
    Context& c = ctx->c;
    const int lv = in[0].level;
    const size_t w = c.ct_words(lv);
    std::vector<std::pair<uintptr_t, int>> spans;  // (start, +1 input / -1 output), for the overlap check
    for (int i = 0; i < count; ++i) {
      check_ct(c, &in[i], "ciphertext");
      need(in[i].level == lv, HETAL_E_LEVEL, "batch items at different levels");
      check_out(c, &out[i], lv);
      spans.push_back({(uintptr_t)in[i].data, 1});
      spans.push_back({(uintptr_t)out[i].data, -1});
    }
    // outputs overlap no input and no other output (each span is w words)
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i) {
      const bool overlap = spans[i].first < spans[i - 1].first + w * 8;
      need(!overlap || (spans[i].second > 0 && spans[i - 1].second > 0), HETAL_E_INVALID_ARG,
           "outputs overlap the inputs or each other");
    }
    std::vector<int> rot, idn;
    std::vector<u32> gal;
    for (int i = 0; i < count; ++i) {
      const u32 g = galois_rot(c, steps[i]);
      if (g == 1) {
        idn.push_back(i);
      } else {
        rot.push_back(i);
        gal.push_back(g);
      }
    }
    for (int i : idn) HCHECK(hipMemcpyAsync(out[i].data, in[i].data, w * 8, hipMemcpyDeviceToDevice, c.stream));
    if (!rot.empty()) {
      const int m = (int)rot.size();
      // evenly spaced handles are used in place; anything else goes through a packed copy
      auto even = [&](auto ptr) {
        if (m == 1) return (size_t)w;
        const intptr_t d = (intptr_t)ptr(1) - (intptr_t)ptr(0);
        if (d < (intptr_t)(w * 8) || d % 8) return (size_t)0;
        for (int t = 2; t < m; ++t)
          if ((intptr_t)ptr(t) - (intptr_t)ptr(t - 1) != d) return (size_t)0;
        return (size_t)(d / 8);
      };
      const size_t sin = even([&](int t) { return in[rot[t]].data; });
      const size_t sout = even([&](int t) { return out[rot[t]].data; });
      if (sin && sout) {
        b_rotate_into(c, keys->set, BView{in[rot[0]].data, lv, m, in[rot[0]].scale, sin}, gal, out[rot[0]].data,
                      sout);
      } else {
        std::vector<CtView> items;
        for (int i : rot) items.push_back(view_of(&in[i]));
        Batch packed = b_pack(c, items);
        Batch res(c, lv, m);
        b_rotate_into(c, keys->set, packed.v(), gal, res.d, w);
        for (int t = 0; t < m; ++t)
          HCHECK(hipMemcpyAsync(out[rot[t]].data, res.d + (size_t)t * w, w * 8, hipMemcpyDeviceToDevice, c.stream));
      }
    }
    for (int i = 0; i < count; ++i) {
      out[i].level = lv;
      out[i].scale = in[i].scale;
    }
  });
}

int hetal_conj(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* ct, hetal_ct* out) {
  return guarded([&] {
    need(ctx && keys, HETAL_E_INVALID_ARG, "null argument");
    check_ct(ctx->c, ct, "ciphertext");
    check_out(ctx->c, out, ct->level);
    const double s = ct->scale;
    const int lv = ct->level;
    op_galois(ctx->c, keys->set, view_of(ct), galois_conj(ctx->c), out->data);
    ctx->c.counters[1] += 1;
    out->level = lv;
    out->scale = s;
  });
}

int hetal_rescale(hetal_ctx* ctx, const hetal_ct* ct, hetal_ct* out) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    check_ct(ctx->c, ct, "ciphertext");
    need(ct->level >= 1, HETAL_E_LEVEL, "no level left to rescale");
    check_out(ctx->c, out, ct->level - 1);
    const int lv = ct->level;
    const double s = ct->scale / (double)ctx->c.primes[lv];
    op_rescale(ctx->c, view_of(ct), out->data);
    out->level = lv - 1;
    out->scale = s;
  });
}

int hetal_mod_drop(hetal_ctx* ctx, const hetal_ct* ct, int level, hetal_ct* out) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    check_ct(ctx->c, ct, "ciphertext");
    need(level >= 0 && level <= ct->level, HETAL_E_LEVEL, "target level out of range");
    check_out(ctx->c, out, level);
    const double s = ct->scale;
    op_mod_drop(ctx->c, view_of(ct), level, out->data);
    out->level = level;
    out->scale = s;
  });
}

int hetal_cmult_const(hetal_ctx* ctx, const hetal_ct* ct, double value, double sigma, hetal_ct* out) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    check_ct(ctx->c, ct, "ciphertext");
    check_out(ctx->c, out, ct->level);
    need(sigma > 0 && std::isfinite(value), HETAL_E_INVALID_ARG, "sigma must be positive and value finite");
    Context& c = ctx->c;
    const int lv = ct->level;
    Batch r = b_mul_const(c, BView{ct->data, lv, 1, ct->scale, c.ct_words(lv)}, value, sigma);
    HCHECK(hipMemcpyAsync(out->data, r.d, c.ct_words(lv) * 8, hipMemcpyDeviceToDevice, c.stream));
    out->level = lv;
    out->scale = r.scale;
  });
}

int hetal_add_const(hetal_ctx* ctx, const hetal_ct* ct, double value, hetal_ct* out) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    check_ct(ctx->c, ct, "ciphertext");
    check_out(ctx->c, out, ct->level);
    need(std::isfinite(value), HETAL_E_INVALID_ARG, "value must be finite");
    Context& c = ctx->c;
    const int lv = ct->level;
    Batch r = b_add_const(c, BView{ct->data, lv, 1, ct->scale, c.ct_words(lv)}, value);
    HCHECK(hipMemcpyAsync(out->data, r.d, c.ct_words(lv) * 8, hipMemcpyDeviceToDevice, c.stream));
    out->level = lv;
    out->scale = r.scale;
  });
}

int hetal_add_plain(hetal_ctx* ctx, const hetal_ct* ct, const hetal_pt* pt, hetal_ct* out) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    Context& c = ctx->c;
    check_ct(c, ct, "ciphertext");
    check_pt(c, pt);
    need(pt->level == ct->level, HETAL_E_LEVEL, "plaintext and ciphertext levels differ");
    need(std::abs(pt->scale - ct->scale) <= 1e-9 * std::max(std::abs(pt->scale), std::abs(ct->scale)), HETAL_E_SCALE,
         "plaintext and ciphertext scales differ");
    check_out(c, out, ct->level);
    const int lv = ct->level;
    Batch r = b_add_plain(c, BView{ct->data, lv, 1, ct->scale, c.ct_words(lv)}, pt->data);
    HCHECK(hipMemcpyAsync(out->data, r.d, c.ct_words(lv) * 8, hipMemcpyDeviceToDevice, c.stream));
    out->level = lv;
    out->scale = ct->scale;
  });
}

int hetal_refresh(hetal_ctx* ctx, const hetal_sk* sk, const hetal_ct* ct, double scale, const uint64_t* a,
                  const int64_t* e, hetal_ct* out) {
  return guarded([&] {
    need(ctx && sk && a && e, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_ct(c, ct, "ciphertext");
    const int top = c.num_q - 1;
    check_out(c, out, top);
    const size_t poly = c.poly_words(top);
    Tmp an(c.pool, poly), en(c.pool, poly);
    load_randomness(c, a, e, top, 1, an, en);
    need(std::isfinite(scale) && scale >= 0.0, HETAL_E_SCALE, "scale must be 0 (keep) or positive");
    const double s = scale > 0.0 ? scale : ct->scale;
    Tmp res(c.pool, c.ct_words(top));
    refresh_encrypt(c, sk->key.s, view_of(ct), scale, an, en, res);
    HCHECK(hipMemcpyAsync(out->data, res.p, c.ct_words(top) * 8, hipMemcpyDeviceToDevice, c.stream));
    HCHECK(hipStreamSynchronize(c.stream));
    out->level = top;
    out->scale = s;
  });
}

int hetal_poly_eval(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* ct, const double* coeffs, int degree,
                    hetal_refresh_fn refresh, void* user, hetal_ct* out) {
  return guarded([&] {
    need(ctx && keys && coeffs, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_ct(c, ct, "ciphertext");
    check_out(c, out, c.num_q - 1);
    need(degree >= 1 && degree <= 64, HETAL_E_INVALID_ARG, "degree must be in [1, 64]");
    std::vector<double> co(coeffs, coeffs + degree + 1);
    for (double v : co) need(std::isfinite(v), HETAL_E_INVALID_ARG, "coefficients must be finite");
    Refresher rf{refresh, user, 0};
    const int lv = ct->level;
    Batch r = poly_eval(c, keys->set, BView{ct->data, lv, 1, ct->scale, c.ct_words(lv)}, co, rf);
    HCHECK(hipMemcpyAsync(out->data, r.d, c.ct_words(r.level) * 8, hipMemcpyDeviceToDevice, c.stream));
    out->level = r.level;
    out->scale = r.scale;
  });
}

int hetal_softmax_default_params(hetal_softmax_params* out) {
  return guarded([&] {
    need(out != nullptr, HETAL_E_INVALID_ARG, "null argument");
    std::memset(out, 0, sizeof(*out));
    out->R = 8.0;
    out->L = 2.0;
    out->n = 5;
    out->precise = 1;
    out->extend = 1;
    out->comp_g = 3;
    out->exp_B = 8;
    out->exp_degree = 12;
    const std::vector<double> p = default_exp_coeffs(12, 8);
    for (int i = 0; i <= 12; ++i) out->exp_coeffs[i] = p[i];
    out->inv_R = 100.0;
    out->inv_iters = 16;
  });
}

int hetal_softmax_rot_steps(const hetal_ctx* ctx, int cc, int s0, int32_t* out, int* n) {
  return guarded([&] {
    need(ctx && n, HETAL_E_INVALID_ARG, "null argument");
    const Context& c = ctx->c;
    need(s0 > 0 && c.slots % s0 == 0, HETAL_E_SHAPE, "s0 must divide N/2");
    need(cc >= 1, HETAL_E_SHAPE, "c must be positive");
    const std::vector<int> st = softmax_rot_steps(cc, c.slots / s0);
    if (out) {
      need(*n >= (int)st.size(), HETAL_E_INVALID_ARG, "output array too small");
      for (size_t i = 0; i < st.size(); ++i) out[i] = st[i];
    }
    *n = (int)st.size();
  });
}

int hetal_ct_to_coeff(hetal_ctx* ctx, const hetal_ct* ct, uint64_t* host) {
  return guarded([&] {
    need(ctx && host, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_ct(c, ct, "ciphertext");
    const size_t words = c.ct_words(ct->level);
    Tmp t(c.pool, words);
    HCHECK(hipMemcpyAsync(t.p, ct->data, words * 8, hipMemcpyDeviceToDevice, c.stream));
    ntt_inverse(c, t, 0, 1, c.rows(ROWS_CT, ct->level));
    HCHECK(hipMemcpyAsync(host, t.p, words * 8, hipMemcpyDeviceToHost, c.stream));
    HCHECK(hipStreamSynchronize(c.stream));
  });
}

int hetal_pt_to_coeff(hetal_ctx* ctx, const hetal_pt* pt, uint64_t* host) {
  return guarded([&] {
    need(ctx && host, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_pt(c, pt);
    const size_t words = c.poly_words(pt->level);
    Tmp t(c.pool, words);
    HCHECK(hipMemcpyAsync(t.p, pt->data, words * 8, hipMemcpyDeviceToDevice, c.stream));
    RowsRef rows = c.rows(ROWS_CT, pt->level);
    ntt_inverse(c, t, 0, 1, RowsRef{rows.d, pt->level + 1});
    HCHECK(hipMemcpyAsync(host, t.p, words * 8, hipMemcpyDeviceToHost, c.stream));
    HCHECK(hipStreamSynchronize(c.stream));
  });
}

int hetal_ct_from_coeff(hetal_ctx* ctx, const uint64_t* host, int level, double scale, hetal_ct* out) {
  return guarded([&] {
    need(ctx && host, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    need(level >= 0 && level < c.num_q, HETAL_E_LEVEL, "level out of range");
    check_out(c, out, level);
    const size_t words = c.ct_words(level);
    HCHECK(hipStreamSynchronize(c.stream));
    for (int p = 0; p < 2; ++p)
      for (int i = 0; i <= level; ++i)
        for (int k = 0; k < c.n; ++k)
          need(host[((size_t)p * (level + 1) + i) * c.n + k] < c.primes[i], HETAL_E_INVALID_ARG, "residue not reduced");
    HCHECK(hipMemcpyAsync(out->data, host, words * 8, hipMemcpyHostToDevice, c.stream));
    ntt_forward(c, out->data, 0, 1, c.rows(ROWS_CT, level));
    HCHECK(hipStreamSynchronize(c.stream));
    out->level = level;
    out->scale = scale;
  });
}

}  // extern "C"

// Block-encodes and encrypts a host matrix; `randomness(nb, level, an, en)` fills the NTT-form randomness of the
// nb blocks.
template <class R>
static void mat_encrypt(hetal_ctx* ctx, const hetal_sk* sk, const double* host, int rows, int cols, int tiling, int cc,
                        hetal_mat* out, R&& randomness) {
  need(rows > 0 && cols > 0, HETAL_E_SHAPE, "empty matrix");
  need(ctx && sk && host && out && out->data, HETAL_E_INVALID_ARG, "null argument");
  Context& c = ctx->c;
  need(out->s0 > 0 && c.slots % out->s0 == 0, HETAL_E_SHAPE, "s0 must divide N/2");
  const int s0 = out->s0, s1 = c.slots / s0;
  need(out->level >= 0 && out->level < c.num_q, HETAL_E_LEVEL, "level out of range");
  need(out->scale > 0, HETAL_E_SCALE, "scale must be positive");
  int n_rb, n_cb;
  if (tiling == 0) {
    n_rb = (rows + s0 - 1) / s0;
    n_cb = (cols + s1 - 1) / s1;
  } else if (tiling == 1) {
    need(cc >= rows && cc > 0 && s0 % cc == 0, HETAL_E_SHAPE, "vertical tiling needs rows <= c and c | s0");
    n_rb = 1;
    n_cb = (cols + s1 - 1) / s1;
  } else if (tiling == 2) {
    need(cc >= cols && cc > 0 && s1 % cc == 0, HETAL_E_SHAPE, "horizontal tiling needs cols <= c and c | s1");
    n_rb = (rows + s0 - 1) / s0;
    n_cb = 1;
  } else {
    fail(HETAL_E_INVALID_ARG, "tiling must be 0, 1 or 2");
  }
  const int nb = n_rb * n_cb;
  const int lv = out->level;
  need(out->capacity >= (size_t)nb * c.ct_words(lv), HETAL_E_INVALID_ARG, "matrix capacity too small");
  Tmp dmat = upload_words(c, host, (size_t)rows * cols * 8);
  Tmp slots(c.pool, (size_t)nb * c.slots);
  k_block_layout(c, reinterpret_cast<const double*>(dmat.p), rows, cols, tiling, cc, s0, s1, n_rb, n_cb,
                 reinterpret_cast<double*>(slots.p));
  const size_t poly = c.poly_words(lv);
  Tmp pts(c.pool, (size_t)nb * poly);
  encode_slots(c, reinterpret_cast<const double*>(slots.p), nullptr, nb, c.slots, lv, out->scale, pts, poly);
  Tmp an(c.pool, (size_t)nb * poly), en(c.pool, (size_t)nb * poly);
  randomness(nb, lv, an, en);
  for (int b = 0; b < nb; ++b)
    k_encrypt(c, an.p + b * poly, en.p + b * poly, pts.p + b * poly, sk->key.s, out->data + b * c.ct_words(lv), lv);
  out->n_rb = n_rb;
  out->n_cb = n_cb;
  out->s1 = s1;
  HCHECK(hipStreamSynchronize(c.stream));
}

extern "C" {

int hetal_mat_encrypt(hetal_ctx* ctx, const hetal_sk* sk, const double* host, int rows, int cols, int tiling, int cc,
                      const uint64_t* a, const int64_t* e, hetal_mat* out) {
  return guarded([&] {
    need(a && e, HETAL_E_INVALID_ARG, "null argument");
    mat_encrypt(ctx, sk, host, rows, cols, tiling, cc, out,
                [&](int nb, int lv, Tmp& an, Tmp& en) { load_randomness(ctx->c, a, e, lv, nb, an, en); });
  });
}

int hetal_mat_encrypt_seeded(hetal_ctx* ctx, const hetal_sk* sk, const double* host, int rows, int cols, int tiling,
                             int cc, uint64_t seed, uint32_t first_index, hetal_mat* out) {
  return guarded([&] {
    mat_encrypt(ctx, sk, host, rows, cols, tiling, cc, out, [&](int nb, int lv, Tmp& an, Tmp& en) {
      sample_randomness(ctx->c, seed, first_index, lv, nb, an, en);
    });
  });
}

int hetal_mat_decrypt(hetal_ctx* ctx, const hetal_sk* sk, const hetal_mat* m, double* host) {
  return guarded([&] {
    need(ctx && sk && m && m->data && host, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    need(m->s0 > 0 && (long)m->s0 * m->s1 == c.slots, HETAL_E_SHAPE, "bad block shape");
    const int nb = m->n_rb * m->n_cb, lv = m->level;
    need(m->capacity >= (size_t)nb * c.ct_words(lv), HETAL_E_INVALID_ARG, "matrix capacity too small");
    const size_t poly = c.poly_words(lv);
    Tmp pt(c.pool, poly);
    Tmp sl(c.pool, c.slots);
    std::vector<double> slots(c.slots);
    const long width = (long)m->n_cb * m->s1;
    RowsRef rows = c.rows(ROWS_CT, lv);
    for (int b = 0; b < nb; ++b) {
      k_decrypt(c, m->data + b * c.ct_words(lv), sk->key.s, pt, lv);
      ntt_inverse(c, pt, 0, 1, RowsRef{rows.d, lv + 1});
      k_decode(c, pt, lv, m->scale, reinterpret_cast<double*>(sl.p), nullptr);
      HCHECK(hipMemcpyAsync(slots.data(), sl.p, (size_t)c.slots * 8, hipMemcpyDeviceToHost, c.stream));
      HCHECK(hipStreamSynchronize(c.stream));
      const int bi = b / m->n_cb, bj = b % m->n_cb;
      for (int r = 0; r < m->s0; ++r)
        std::memcpy(host + ((long)bi * m->s0 + r) * width + (long)bj * m->s1, slots.data() + (long)r * m->s1,
                    (size_t)m->s1 * 8);
    }
  });
}

static std::vector<CtView> block_views(const Context& c, const hetal_mat* m) {
  std::vector<CtView> v;
  for (int b = 0; b < m->n_rb * m->n_cb; ++b) v.push_back(CtView{m->data + b * c.ct_words(m->level), m->level, m->scale});
  return v;
}

static void check_mat(const Context& c, const hetal_mat* m, const char* what) {
  need(m && m->data, HETAL_E_INVALID_ARG, what);
  need(m->n_rb > 0 && m->n_cb > 0, HETAL_E_SHAPE, "empty block grid");
  need(m->s0 > 0 && (long)m->s0 * m->s1 == c.slots, HETAL_E_SHAPE, "s0 * s1 must equal N/2");
  need(m->level >= 0 && m->level < c.num_q, HETAL_E_LEVEL, "matrix level out of range");
  need(m->capacity >= (size_t)m->n_rb * m->n_cb * c.ct_words(m->level), HETAL_E_INVALID_ARG, "matrix capacity too small");
}

static void store_blocks(Context& c, const Batch& res, hetal_mat* out, int n_rb, int n_cb, int s0, int s1) {
  const int lv = res.level;
  need(out && out->data, HETAL_E_INVALID_ARG, "output matrix");
  need(out->capacity >= (size_t)res.count * c.ct_words(lv), HETAL_E_INVALID_ARG, "output capacity too small");
  HCHECK(hipMemcpyAsync(out->data, res.d, (size_t)res.count * c.ct_words(lv) * 8, hipMemcpyDeviceToDevice, c.stream));
  out->n_rb = n_rb;
  out->n_cb = n_cb;
  out->s0 = s0;
  out->s1 = s1;
  out->level = lv;
  out->scale = res.scale;
}

int hetal_enc_matmul_abt(hetal_ctx* ctx, const hetal_keys* keys, const hetal_mat* a, const hetal_mat* bbar, int cc,
                         double t, hetal_mat* out) {
  return guarded([&] {
    need(ctx && keys, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_mat(c, a, "A");
    check_mat(c, bbar, "Bbar");
    need(a->s0 == bbar->s0, HETAL_E_SHAPE, "A and Bbar block shapes differ");
    need(bbar->n_rb == 1 && bbar->n_cb == a->n_cb, HETAL_E_SHAPE, "Bbar must be one block row matching A's columns");
    std::vector<CtView> av = block_views(c, a), bv = block_views(c, bbar);
    std::vector<std::vector<CtView>> A(a->n_rb);
    for (int i = 0; i < a->n_rb; ++i) A[i].assign(av.begin() + i * a->n_cb, av.begin() + (i + 1) * a->n_cb);
    Batch res = diag_abt_batch(c, keys->set, ctx->masks, A, bv, cc, a->s0, a->s1, t);
    store_blocks(c, res, out, a->n_rb, 1, a->s0, a->s1);
  });
}

int hetal_enc_matmul_atb(hetal_ctx* ctx, const hetal_keys* keys, const hetal_mat* abar, const hetal_mat* b, int cc,
                         double t, hetal_mat* out) {
  return guarded([&] {
    need(ctx && keys, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_mat(c, abar, "Abar");
    check_mat(c, b, "B");
    need(abar->s0 == b->s0, HETAL_E_SHAPE, "Abar and B block shapes differ");
    need(abar->n_cb == 1 && abar->n_rb == b->n_rb, HETAL_E_SHAPE, "Abar must be one block column matching B's rows");
    std::vector<CtView> av = block_views(c, abar), bv = block_views(c, b);
    std::vector<std::vector<CtView>> B(b->n_rb);
    for (int i = 0; i < b->n_rb; ++i) B[i].assign(bv.begin() + i * b->n_cb, bv.begin() + (i + 1) * b->n_cb);
    Batch res = diag_atb_batch(c, keys->set, ctx->masks, av, B, cc, b->s0, b->s1, t);
    store_blocks(c, res, out, 1, b->n_cb, b->s0, b->s1);
  });
}

// The second stream of a context (see hetal_ctx), created on first use.
static Context& side_context(hetal_ctx* ctx) {
  if (!ctx->side) {
    HCHECK(hipStreamCreateWithFlags(&ctx->side_stream, hipStreamNonBlocking));
    HCHECK(hipEventCreateWithFlags(&ctx->join[0], hipEventDisableTiming));
    HCHECK(hipEventCreateWithFlags(&ctx->join[1], hipEventDisableTiming));
    std::unique_ptr<Context> s(new Context());
    context_share(*s, ctx->c, ctx->side_stream);
    ctx->side = std::move(s);
  }
  return *ctx->side;
}

// While alive: the side stream starts after the work queued so far on the main stream, and (at the end, also
// when an error unwinds) the main stream waits for everything queued on the side stream; the side counters are
// folded into the main ones.
struct SideJoin {
  hetal_ctx* ctx;
  SideJoin(hetal_ctx* x) : ctx(x) {
    HCHECK(hipEventRecord(ctx->join[0], ctx->c.stream));
    HCHECK(hipStreamWaitEvent(ctx->side_stream, ctx->join[0], 0));
  }
  ~SideJoin() {
    (void)hipEventRecord(ctx->join[1], ctx->side_stream);
    (void)hipStreamWaitEvent(ctx->c.stream, ctx->join[1], 0);
    for (int i = 0; i < 8; ++i) {
      ctx->c.counters[i] += ctx->side->counters[i];
      ctx->side->counters[i] = 0;
    }
    for (int i = 0; i < MAX_PRIMES; ++i) {
      ctx->c.ks_items[i] += ctx->side->ks_items[i];
      ctx->c.ks_key_reads[i] += ctx->side->ks_key_reads[i];
      ctx->side->ks_items[i] = ctx->side->ks_key_reads[i] = 0;
    }
  }
};

static void matmul_batch(hetal_ctx* ctx, const hetal_keys* keys, const hetal_matmul_req* reqs, int count,
                         hetal_mat* outs) {
  {
    need(ctx && keys && reqs && outs && count >= 0, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    // validate everything first; then group by what makes the algorithm's step sequence identical
    std::map<std::tuple<int, int, int, int, int, double, double>, std::vector<int>> groups;
    for (int i = 0; i < count; ++i) {
      const hetal_matmul_req& r = reqs[i];
      need(r.op == 0 || r.op == 1, HETAL_E_INVALID_ARG, "request op must be 0 (DiagABT) or 1 (DiagATB)");
      check_mat(c, r.a, r.op == 0 ? "A" : "Abar");
      check_mat(c, r.b, r.op == 0 ? "Bbar" : "B");
      need(r.a->s0 == r.b->s0, HETAL_E_SHAPE, "request block shapes differ");
      need(r.c >= 2 && (r.c & (r.c - 1)) == 0 && r.a->s1 % r.c == 0 && r.c <= (r.op == 0 ? r.a->s0 : r.a->s1),
           HETAL_E_SHAPE, "need c a power of two above 1 dividing s1 (and at most s0 for DiagABT)");
      need(outs[i].data != nullptr, HETAL_E_INVALID_ARG, "output matrix");
      int lv_a, lv_b;
      if (r.op == 0) {
        need(r.b->n_rb == 1 && r.b->n_cb == r.a->n_cb, HETAL_E_SHAPE, "Bbar must be one block row matching A's columns");
        need(std::min(r.a->level, r.b->level) >= 3, HETAL_E_LEVEL, "DiagABT needs three levels");
        need(outs[i].capacity >= (size_t)r.a->n_rb * c.ct_words(std::min(r.a->level, r.b->level) - 3),
             HETAL_E_INVALID_ARG, "output capacity too small");
        lv_a = lv_b = std::min(r.a->level, r.b->level);
      } else {
        need(r.a->n_cb == 1 && r.a->n_rb == r.b->n_rb, HETAL_E_SHAPE, "Abar must be one block column matching B's rows");
        const int ls = r.a->level < r.b->level ? std::min(r.a->level - 1, r.b->level - 1)
                                               : std::min(r.a->level - 2, r.b->level);
        need(ls >= 2, HETAL_E_LEVEL, "DiagATB needs more levels");
        need(outs[i].capacity >= (size_t)r.b->n_cb * c.ct_words(ls - 2), HETAL_E_INVALID_ARG,
             "output capacity too small");
        lv_a = r.a->level;
        lv_b = r.b->level;
      }
      groups[std::make_tuple(r.op, r.c, r.a->s0, lv_a, lv_b, r.a->scale, r.b->scale)].push_back(i);
    }
    // Independent groups alternate between the main stream and a second one, so that one group's small
    // launches overlap the other's (unless per-kernel timing is on, which wants kernels one at a time).
    const bool two = groups.size() >= 2 && !c.timing && ctx->two_streams;
    std::unique_ptr<SideJoin> joined;
    if (two) {
      side_context(ctx);
      joined.reset(new SideJoin(ctx));
    }
    int gi = 0;
    for (auto& kv : groups) {
      const bool on_side = two && (gi++ % 2 == 1);
      Context& cx = on_side ? *ctx->side : c;
      MaskCache& mcx = on_side ? ctx->side_masks : ctx->masks;
      const int op = std::get<0>(kv.first), cc = std::get<1>(kv.first), s0 = std::get<2>(kv.first);
      const int s1 = c.slots / s0;
      auto tuned = ctx->tuned.find({op, cc, s0, std::get<3>(kv.first), std::get<4>(kv.first)});
      struct TuneScope {  // the class's schedule for this group only (also when an error unwinds)
        Context& c;
        ~TuneScope() { c.tune = Tune{}; }
      } scope{cx};
      cx.tune = tuned != ctx->tuned.end() ? tuned->second : Tune{};
      const std::vector<int>& idx = kv.second;
      Batch res;
      if (op == 0) {
        std::vector<AbtRequest> rq;
        for (int i : idx) {
          const hetal_matmul_req& r = reqs[i];
          std::vector<CtView> av = block_views(c, r.a);
          AbtRequest q;
          for (int b = 0; b < r.a->n_rb; ++b) q.A.emplace_back(av.begin() + b * r.a->n_cb, av.begin() + (b + 1) * r.a->n_cb);
          q.Bbar = block_views(c, r.b);
          q.t = r.t;
          rq.push_back(std::move(q));
        }
        res = diag_abt_multi(cx, keys->set, mcx, rq, cc, s0, s1);
      } else {
        std::vector<AtbRequest> rq;
        for (int i : idx) {
          const hetal_matmul_req& r = reqs[i];
          std::vector<CtView> bv = block_views(c, r.b);
          AtbRequest q;
          q.Abar = block_views(c, r.a);
          for (int b = 0; b < r.b->n_rb; ++b) q.B.emplace_back(bv.begin() + b * r.b->n_cb, bv.begin() + (b + 1) * r.b->n_cb);
          q.t = r.t;
          rq.push_back(std::move(q));
        }
        res = diag_atb_multi(cx, keys->set, mcx, rq, cc, s0, s1);
      }
      // request i's blocks follow the earlier requests' in the result
      int first = 0;
      const size_t w = cx.ct_words(res.level);
      for (int i : idx) {
        const hetal_matmul_req& r = reqs[i];
        const int nb = op == 0 ? r.a->n_rb : r.b->n_cb;
        hetal_mat* o = &outs[i];
        HCHECK(hipMemcpyAsync(o->data, res.d + (size_t)first * w, (size_t)nb * w * 8, hipMemcpyDeviceToDevice,
                              cx.stream));
        o->n_rb = op == 0 ? nb : 1;
        o->n_cb = op == 0 ? 1 : nb;
        o->s0 = s0;
        o->s1 = s1;
        o->level = res.level;
        o->scale = res.scale;
        first += nb;
      }
    }
  }
}

int hetal_enc_matmul_batch(hetal_ctx* ctx, const hetal_keys* keys, const hetal_matmul_req* reqs, int count,
                           hetal_mat* outs) {
  return guarded([&] { matmul_batch(ctx, keys, reqs, count, outs); });
}

// Median time (ms) of `reps` runs of a batch, between events on the context's stream (the batch joins its second
// stream back into it).
static double time_batch(hetal_ctx* ctx, const hetal_keys* keys, const hetal_matmul_req* reqs, int count,
                         hetal_mat* outs, int reps) {
  hipEvent_t e[2];
  HCHECK(hipEventCreate(&e[0]));
  HCHECK(hipEventCreate(&e[1]));
  std::vector<double> t;
  try {
    for (int r = 0; r < reps; ++r) {
      HCHECK(hipEventRecord(e[0], ctx->c.stream));
      matmul_batch(ctx, keys, reqs, count, outs);
      HCHECK(hipEventRecord(e[1], ctx->c.stream));
      HCHECK(hipEventSynchronize(e[1]));
      float ms = 0.0f;
      HCHECK(hipEventElapsedTime(&ms, e[0], e[1]));
      t.push_back(ms);
    }
  } catch (...) {
    (void)hipEventDestroy(e[0]);
    (void)hipEventDestroy(e[1]);
    throw;
  }
  (void)hipEventDestroy(e[0]);
  (void)hipEventDestroy(e[1]);
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

int hetal_autotune_batch(hetal_ctx* ctx, const hetal_keys* keys, const hetal_matmul_req* reqs, int count,
                         hetal_mat* outs, int reps, hetal_tune_report* report) {
  return guarded([&] {
    need(ctx && keys && reqs && outs && count > 0 && reps >= 1, HETAL_E_INVALID_ARG, "bad argument");
    need(!ctx->c.timing, HETAL_E_INVALID_ARG, "per-kernel timing is on");
    ctx->tuned.clear();
    ctx->two_streams = true;
    matmul_batch(ctx, keys, reqs, count, outs);  // warm-up (masks encoded, pools sized); also validates
    const double untuned = time_batch(ctx, keys, reqs, count, outs, reps);
    // the shape classes of the batch, each tuned alone by coordinate descent over the schedule choices
    std::map<std::array<int, 5>, std::vector<int>> classes;
    for (int i = 0; i < count; ++i) {
      const hetal_matmul_req& r = reqs[i];
      const int lv_a = r.op == 0 ? std::min(r.a->level, r.b->level) : r.a->level;
      const int lv_b = r.op == 0 ? lv_a : r.b->level;
      classes[{r.op, r.c, r.a->s0, lv_a, lv_b}].push_back(i);
    }
    int trials = 0;
    for (auto& kv : classes) {
      std::vector<hetal_matmul_req> sr;
      std::vector<hetal_mat> so;
      for (int i : kv.second) {
        sr.push_back(reqs[i]);
        so.push_back(outs[i]);
      }
      auto run = [&](const Tune& t) {
        ctx->tuned[kv.first] = t;
        ++trials;
        return time_batch(ctx, keys, sr.data(), (int)sr.size(), so.data(), reps);
      };
      Tune best;
      double best_ms = run(best);
      auto consider = [&](Tune cand) {
        const double ms = run(cand);
        if (ms < 0.98 * best_ms) {  // a choice must beat the current one by more than the timing noise
          best = cand;
          best_ms = ms;
        }
      };
      for (int g : {16, 8, 4}) {
        Tune t = best;
        t.ks_group = g;
        consider(t);
      }
      for (int v : {2, 4, 6, 12}) {
        Tune t = best;
        t.tpt_modup = v;
        consider(t);
      }
      for (int v : {2, 3, 6, 12}) {
        Tune t = best;
        t.tpt_moddown = v;
        consider(t);
      }
      ctx->tuned[kv.first] = best;
    }
    // the second stream for independent classes, with the tuned schedules
    double tuned = time_batch(ctx, keys, reqs, count, outs, reps);
    if (classes.size() >= 2) {
      ctx->two_streams = false;
      const double one = time_batch(ctx, keys, reqs, count, outs, reps);
      ++trials;
      if (one < tuned) tuned = one;
      else ctx->two_streams = true;
    }
    if (report) {
      report->untuned_ms = untuned;
      report->tuned_ms = tuned;
      report->classes = (int)classes.size();
      report->trials = trials;
      report->two_streams = ctx->two_streams ? 1 : 0;
    }
  });
}

int hetal_tune_get(const hetal_ctx* ctx, int op, int c, int s0, int level_a, int level_b, hetal_tune* out) {
  return guarded([&] {
    need(ctx && out, HETAL_E_INVALID_ARG, "null argument");
    auto it = ctx->tuned.find({op, c, s0, level_a, level_b});
    const Tune t = it != ctx->tuned.end() ? it->second : Tune{};
    out->ks_group = t.ks_group;
    out->tpt_modup = t.tpt_modup;
    out->tpt_moddown = t.tpt_moddown;
    out->two_streams = ctx->two_streams ? 1 : 0;
    out->work_cts = t.work_cts;
  });
}

int hetal_tune_set(hetal_ctx* ctx, int op, int c, int s0, int level_a, int level_b, const hetal_tune* in) {
  return guarded([&] {
    need(ctx && in, HETAL_E_INVALID_ARG, "null argument");
    need(in->ks_group >= 1 && in->ks_group <= MAX_BATCH && in->tpt_modup >= 0 && in->tpt_moddown >= 0 &&
             in->work_cts >= 0,
         HETAL_E_INVALID_ARG, "schedule out of range");
    Tune t;
    t.ks_group = in->ks_group;
    t.tpt_modup = in->tpt_modup;
    t.tpt_moddown = in->tpt_moddown;
    t.work_cts = in->work_cts;
    ctx->tuned[{op, c, s0, level_a, level_b}] = t;
    ctx->two_streams = in->two_streams != 0;
  });
}

int hetal_tune_reset(hetal_ctx* ctx) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    ctx->tuned.clear();
    ctx->two_streams = true;
  });
}

struct hetal_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hetal_ctx* ctx = nullptr;
};

int hetal_enc_matmul_batch_graph(hetal_ctx* ctx, const hetal_keys* keys, const hetal_matmul_req* reqs, int count,
                                 hetal_mat* outs, hetal_graph** out) {
  return guarded([&] {
    need(ctx && out, HETAL_E_INVALID_ARG, "null argument");
    need(ctx->c.stream != nullptr, HETAL_E_INVALID_ARG, "graph capture needs the context on a created stream");
    need(!ctx->c.timing, HETAL_E_INVALID_ARG, "per-kernel timing is on");
    // two eager runs: the first encodes the masks (each keeps a pool buffer), the second leaves the pools
    // holding the buffers of every size the recorded run asks for (no allocation is allowed while recording);
    // the pools reuse exact size classes until the recording ends, so that the recorded run finds the buffers
    // the second run used
    if (ctx->two_streams) side_context(ctx);
    struct ExactFit {
      hetal_ctx* ctx;
      void set(bool on) {
        ctx->c.pool.exact_fit = on;
        if (ctx->side) ctx->side->pool.exact_fit = on;
      }
      ~ExactFit() { set(false); }
    } exact{ctx};
    exact.set(true);
    matmul_batch(ctx, keys, reqs, count, outs);
    matmul_batch(ctx, keys, reqs, count, outs);
    HCHECK(hipStreamSynchronize(ctx->c.stream));
    if (ctx->side) HCHECK(hipStreamSynchronize(ctx->side_stream));
    std::unique_ptr<hetal_graph> g(new hetal_graph());
    g->ctx = ctx;
    auto recording = [&](bool on) {
      ctx->c.pool.recording = on;
      if (ctx->side) ctx->side->pool.recording = on;
    };
    HCHECK(hipStreamBeginCapture(ctx->c.stream, hipStreamCaptureModeThreadLocal));
    recording(true);
    try {
      matmul_batch(ctx, keys, reqs, count, outs);
    } catch (...) {
      recording(false);
      hipGraph_t partial = nullptr;
      (void)hipStreamEndCapture(ctx->c.stream, &partial);
      if (partial) (void)hipGraphDestroy(partial);
      throw;
    }
    recording(false);
    HCHECK(hipStreamEndCapture(ctx->c.stream, &g->graph));
    HCHECK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    *out = g.release();
  });
}

int hetal_graph_launch(hetal_graph* g) {
  return guarded([&] {
    need(g && g->exec && g->ctx, HETAL_E_INVALID_ARG, "null graph");
    HCHECK(hipGraphLaunch(g->exec, g->ctx->c.stream));
  });
}

void hetal_graph_destroy(hetal_graph* g) {
  if (!g) return;
  if (g->ctx) (void)hipStreamSynchronize(g->ctx->c.stream);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

int hetal_required_rot_steps(const hetal_ctx* ctx, int op, int cc, int s0, int32_t* out, int* n) {
  return guarded([&] {
    need(ctx && n, HETAL_E_INVALID_ARG, "null argument");
    need(s0 > 0 && ctx->c.slots % s0 == 0, HETAL_E_SHAPE, "s0 must divide N/2");
    std::vector<int> steps = required_rot_steps(ctx->c, op, cc, s0);
    need(out == nullptr || *n >= (int)steps.size(), HETAL_E_INVALID_ARG, "output array too small");
    if (out)
      for (size_t i = 0; i < steps.size(); ++i) out[i] = steps[i];
    *n = (int)steps.size();
  });
}

static SoftmaxArgs softmax_args(const hetal_softmax_params& p);

int hetal_softmax_approx(hetal_ctx* ctx, const hetal_keys* keys, const hetal_mat* m, int cc,
                         const hetal_softmax_params* params, hetal_refresh_fn refresh, void* user, hetal_mat* out,
                         int* refreshes) {
  return guarded([&] {
    need(ctx && keys && params && out && out->data, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_mat(c, m, "M");
    need(m->n_cb == 1, HETAL_E_SHAPE, "the input must be one block column (horizontally tiled classes)");
    need(cc >= 1 && cc <= m->s1, HETAL_E_SHAPE, "c out of range");
    need(out->capacity >= (size_t)m->n_rb * c.ct_words(c.num_q - 1), HETAL_E_INVALID_ARG,
         "output capacity: n_rb ciphertexts at the top level");
    const SoftmaxArgs a = softmax_args(*params);
    Refresher rf{refresh, user, 0};
    Batch res = softmax_approx(c, keys->set, ctx->masks,
                               BView{m->data, m->level, m->n_rb, m->scale, c.ct_words(m->level)}, cc, m->s0, m->s1, a,
                               rf);
    store_blocks(c, res, out, m->n_rb, 1, m->s0, m->s1);
    if (refreshes) *refreshes = rf.count;
  });
}

static SoftmaxArgs softmax_args(const hetal_softmax_params& p) {
  need(p.R > 0 && p.L > 1 && p.n >= 0 && p.n <= 30 && p.comp_g >= 0 && p.comp_g <= 16 && p.exp_B >= 1 &&
           p.exp_degree >= 1 && p.exp_degree <= 31 && p.inv_R > 0 && p.inv_iters >= 0 && p.inv_iters <= 64,
       HETAL_E_INVALID_ARG, "softmax parameters out of range");
  for (int i = 0; i <= p.exp_degree; ++i)
    need(std::isfinite(p.exp_coeffs[i]), HETAL_E_INVALID_ARG, "exp coefficients must be finite");
  SoftmaxArgs a;
  a.R = p.R;
  a.L = p.L;
  a.n = p.n;
  a.precise = p.precise;
  a.extend = p.extend;
  a.comp_g = p.comp_g;
  a.exp_B = p.exp_B;
  a.exp_coeffs.assign(p.exp_coeffs, p.exp_coeffs + p.exp_degree + 1);
  a.inv_R = p.inv_R;
  a.inv_iters = p.inv_iters;
  return a;
}

int hetal_nag_step(hetal_ctx* ctx, const hetal_keys* keys, const hetal_mat* x, const hetal_mat* y, const hetal_mat* w,
                   const hetal_mat* v, int cc, double lr, double gamma, const hetal_softmax_params* params,
                   hetal_refresh_fn refresh, void* user, hetal_mat* w_out, hetal_mat* v_out, int* refreshes) {
  return guarded([&] {
    need(ctx && keys && params && w_out && v_out && w_out->data && v_out->data, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    check_mat(c, x, "X");
    check_mat(c, y, "Y");
    check_mat(c, w, "W");
    check_mat(c, v, "V");
    const int s0 = x->s0, s1 = x->s1;
    need(y->s0 == s0 && w->s0 == s0 && v->s0 == s0, HETAL_E_SHAPE, "all matrices need one block shape");
    need(y->n_rb == x->n_rb && y->n_cb == 1, HETAL_E_SHAPE, "Y: one block per block row of X (tiled classes)");
    need(w->n_rb == 1 && v->n_rb == 1 && w->n_cb == x->n_cb && v->n_cb == x->n_cb, HETAL_E_SHAPE,
         "W and V: one block row, one block per block column of X");
    int cp = 1;
    while (cp < cc) cp *= 2;
    need(cc >= 2 && cp <= s0 && s1 % cp == 0, HETAL_E_SHAPE, "need 2 <= c, c' <= s0 and c' | s1");
    need(std::isfinite(lr) && std::isfinite(gamma), HETAL_E_INVALID_ARG, "lr and gamma must be finite");
    const size_t top_words = c.ct_words(c.num_q - 1);
    need(w_out->capacity >= (size_t)x->n_cb * top_words && v_out->capacity >= (size_t)x->n_cb * top_words,
         HETAL_E_INVALID_ARG, "output capacity: n_cb ciphertexts at the top level");
    need(w_out->data != v_out->data, HETAL_E_INVALID_ARG, "W and V outputs must differ");
    const SoftmaxArgs a = softmax_args(*params);
    Refresher rf{refresh, user, 0};
    auto bv = [&](const hetal_mat* m) {
      return BView{m->data, m->level, m->n_rb * m->n_cb, m->scale, c.ct_words(m->level)};
    };
    NagResult r = nag_step(c, keys->set, ctx->masks, bv(x), x->n_rb, x->n_cb, bv(y), bv(w), bv(v), cc, s0, s1, lr,
                           gamma, a, rf);
    store_blocks(c, r.W, w_out, 1, x->n_cb, s0, s1);
    store_blocks(c, r.V, v_out, 1, x->n_cb, s0, s1);
    if (refreshes) *refreshes = rf.count;
  });
}

int hetal_counters_get(const hetal_ctx* ctx, int64_t* out8) {
  return guarded([&] {
    need(ctx && out8, HETAL_E_INVALID_ARG, "null argument");
    std::memcpy(out8, ctx->c.counters, sizeof(ctx->c.counters));
  });
}

int hetal_counters_reset(hetal_ctx* ctx) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    std::memset(ctx->c.counters, 0, sizeof(ctx->c.counters));
    std::memset(ctx->c.ks_items, 0, sizeof(ctx->c.ks_items));
    std::memset(ctx->c.ks_key_reads, 0, sizeof(ctx->c.ks_key_reads));
  });
}

int hetal_ks_counts(const hetal_ctx* ctx, int64_t* items, int64_t* key_reads, int levels) {
  return guarded([&] {
    need(ctx && items && key_reads && levels >= 0, HETAL_E_INVALID_ARG, "null argument");
    for (int i = 0; i < levels; ++i) {
      items[i] = i < MAX_PRIMES ? ctx->c.ks_items[i] : 0;
      key_reads[i] = i < MAX_PRIMES ? ctx->c.ks_key_reads[i] : 0;
    }
  });
}

static void recycle_timed(Context& c) {
  for (auto& t : c.timed) {
    c.ev_free.push_back(t.start);
    c.ev_free.push_back(t.stop);
  }
  c.timed.clear();
}

int hetal_timing_enable(hetal_ctx* ctx, int on) {
  return guarded([&] {
    need(ctx, HETAL_E_INVALID_ARG, "null context");
    HCHECK(hipStreamSynchronize(ctx->c.stream));
    recycle_timed(ctx->c);
    ctx->c.timing = on != 0;
  });
}

int hetal_timing_classes(void) { return NUM_KC; }

int hetal_timing_get(hetal_ctx* ctx, double* ms, int64_t* launches, double* bytes) {
  return guarded([&] {
    need(ctx && ms && launches && bytes, HETAL_E_INVALID_ARG, "null argument");
    Context& c = ctx->c;
    HCHECK(hipStreamSynchronize(c.stream));
    for (int k = 0; k < NUM_KC; ++k) {
      ms[k] = 0.0;
      launches[k] = 0;
      bytes[k] = 0.0;
    }
    for (auto& t : c.timed) {
      float e = 0.f;
      HCHECK(hipEventElapsedTime(&e, t.start, t.stop));
      ms[t.cls] += e;
      launches[t.cls] += 1;
      bytes[t.cls] += t.bytes;
    }
  });
}

}  // extern "C"
