// Internal declarations of the HETAL gfx950 library: the context with its
// precomputed tables, the device memory pool, and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <stdexcept>
#include <string>
#include <vector>

#include "hetal.h"
#include "modarith.hpp"

namespace hetal {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

#define HCHECK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) ::hetal::fail(HETAL_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int MAX_PRIMES = 32;
constexpr int MAX_ALPHA = 8;
constexpr int MAX_K = 8;
constexpr int MAX_BATCH = 32;

// Fast basis conversion constants of one digit at one level (ModUp).
struct ModUpTab {
  int nsrc;
  int first;                      // index of the digit's first prime (digit = [first, first + nsrc))
  u64 dinv[MAX_ALPHA];            // (D / d_i)^-1 mod d_i
  u64 dinv_sh[MAX_ALPHA];         // its Shoup companion
  u64 dhat[MAX_ALPHA][MAX_PRIMES];  // (D / d_i) mod t, t = global prime index
  u64 dhat_sh[MAX_ALPHA][MAX_PRIMES];  // Shoup companions w.r.t. t
};

// Centred conversion from the special primes to q_i, and P^-1 mod q_i (ModDown).
struct ModDownTab {
  int k;
  int pad;
  u64 pkinv[MAX_K];               // (P / p_k)^-1 mod p_k
  u64 pkinv_sh[MAX_K];
  u64 phat[MAX_K][MAX_PRIMES];    // (P / p_k) mod q_i
  u64 phat_sh[MAX_K][MAX_PRIMES];  // Shoup companions w.r.t. q_i
  u64 pinv[MAX_PRIMES];           // P^-1 mod q_i
  u64 pinv_sh[MAX_PRIMES];
};

// Per-row replacement of the inverse transform's final N^-1 scaling: row r of the row list gets
// s0 on the sums and s1 = psi^-(N/2) s0 on the differences of the last butterfly (each with its Shoup
// companion), i.e. the inverse transform times s0 / N^-1.
struct NttScale {
  u64 s0, s0_sh, s1, s1_sh;
};

// A prime as the NTT kernels' FP64 arithmetic takes it: q and its reciprocal rounded to nearest.
struct FpMod {
  double q, qinv;
};

// q_l^-1 mod q_i (i < l) for the rescale at level l.
struct RescaleTab {
  u64 inv[MAX_PRIMES];  // q_level^-1 mod q_i
  u64 inv_sh[MAX_PRIMES];
};

// Per prime: N^-1, and psi^-brev(1) N^-1 (the last inverse butterfly with N^-1 merged);
// i_q = psi^(N/2), a square root of -1 (multiplication by X^(N/2) in the NTT domain).
// Position of twiddle x (the one of forward stage s, x in [2^s, 2^(s+1))) in the twiddle tables.
// The last 8 stages run on 256-point chunks, and in their stages 4..7 the 16 threads of a chunk
// each take a different twiddle of the stage's 2^l for chunk c: thread j takes entries
// j 2^(l-4) + i, i < 2^(l-4).  Those 2^l entries are stored i-major (slot 16 i + j) so that one
// load instruction of the 16 threads reads 256 contiguous bytes.  All other twiddles are in place.
inline int ntt_twiddle_slot(int x, int log_n) {
  const int s0 = log_n - 8;
  if (x < (1 << (s0 + 4))) return x;
  const int s = 31 - __builtin_clz((unsigned)x);
  const int l = s - s0;
  const int base = 1 << s;
  const int c = (x - base) >> l;
  const int k = (x - base) & ((1 << l) - 1);
  const int m = l - 4;
  return base + (c << l) + (((k & ((1 << m) - 1)) << 4) | (k >> m));
}

// g^-1 modulo 2N (a power of two; g odd): g^(N - 1), since the odd residues mod 2N form a group of order N.
inline u32 galois_inverse(u32 g, u32 two_n) {
  u64 r = 1, b = g % two_n;
  for (u32 e = two_n / 2 - 1; e; e >>= 1, b = b * b % two_n)
    if (e & 1) r = r * b % two_n;
  return (u32)r;
}

// Device address of a field of a device-resident table (address arithmetic only, nothing is read).
template <class T, class S>
const T* device_field(const S* table, size_t offset) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(table) + offset);
}

struct PrimeConsts {
  u64 ninv, ninv_sh;
  u64 w1ninv, w1ninv_sh;
  u64 iq, iq_sh;
  u64 pmod;      // P mod q (0 for special primes)
  u64 pmod_sh;
};

// Size-bucketed cache of device allocations; all work is ordered on one stream,
// so a buffer returned to the pool may be handed out again immediately.
//
// Arena mode (between arena_begin and arena_end): get() carves 256-byte aligned buffers out of one
// caller-provided device region in order and never allocates (E_INVALID_ARG once the region is used
// up); put() of the most recent buffer gives its space back, other buffers are held until arena_end.
// The regular free list is neither used nor changed meanwhile.
class Pool {
 public:
  u64* get(size_t words);
  void put(u64* p);
  void release_all();
  ~Pool();
  size_t bytes_held() const { return held_; }
  bool recording = false;  // while work is recorded into a graph: no allocation (an error instead)
  // Reuse only buffers of the request's exact size class: the same sequence of requests then finds the same
  // buffers again, so a run that allocated nothing is followed by runs that allocate nothing (graph recording).
  bool exact_fit = false;
  void arena_begin(u64* base, size_t words);
  void arena_end();
  static size_t arena_round(size_t words) { return (words + 31) / 32 * 32; }  // 256-byte granules

 private:
  std::multimap<size_t, u64*> free_;
  std::map<u64*, size_t> size_of_;
  size_t held_ = 0;
  u64* arena_ = nullptr;
  size_t arena_words_ = 0;
  std::vector<size_t> arena_marks_;  // start offset of every buffer handed out, in order
  size_t arena_top_ = 0;
};

// RAII lease of a pool buffer.
struct Tmp {
  Pool* pool;
  u64* p;
  Tmp(Pool& pl, size_t words) : pool(&pl), p(pl.get(words)) {}
  ~Tmp() {
    if (p) pool->put(p);
  }
  Tmp(Tmp&& o) noexcept : pool(o.pool), p(o.p) { o.p = nullptr; }
  Tmp(const Tmp&) = delete;
  Tmp& operator=(const Tmp&) = delete;
  operator u64*() const { return p; }
};

// Kernel classes for the optional per-launch HIP-event timing: the NTT passes (forward strided = first, forward
// contiguous = final, plain or with the combine epilogue; inverse contiguous = first, inverse strided = final) and
// the key switch's own kernels (keyswitch.hip).
enum KernelClass {
  KC_NTT_FWD_STRIDED = 0,
  KC_KS_MODUP,          // inverse strided pass, ModUp conversion, forward strided pass
  KC_KS_MODDOWN,        // inverse strided pass of the special rows, ModDown conversion, forward strided pass
  KC_NTT_FWD_CONTIG,
  KC_NTT_FWD_EPILOGUE,
  KC_NTT_INV_CONTIG,
  KC_NTT_INV_STRIDED,
  KC_KS_INNER,          // forward contiguous pass of the extended digits, key product, special rows' inverse pass
  KC_RESCALE,
  KC_ELEMWISE,
  KC_ENCODE,
  NUM_KC
};

struct TimedLaunch {
  hipEvent_t start, stop;
  int cls;
  double bytes;  // algorithmic HBM bytes of the launch
};

enum RowTable { ROWS_CT = 0, ROWS_MODUP, ROWS_SPECIAL, ROWS_TOP, ROWS_ALL, ROWS_ALL2, ROWS_EXT, NUM_ROW_TABLES };

struct RowsRef {
  const int2* d;
  int count;
};

// Schedule choices that leave every result unchanged, word for word (an autotuner picks them per shape class):
// ks_group, the most key switches one launch sequence takes (up to MAX_BATCH); tpt_modup / tpt_moddown, the
// target primes per workgroup task of the key switch's conversion kernels (0: the library's rule).
struct Tune {
  int ks_group = MAX_BATCH;
  int tpt_modup = 0;
  int tpt_moddown = 0;
  int work_cts = 0;  // working-set limit of the matrix products, in ciphertexts (0 = the library's rule)
};

struct Context {
  int log_n = 0, n = 0, slots = 0;
  int num_q = 0, num_p = 0, dnum = 0, alpha = 0, nprimes = 0;
  std::vector<u64> primes;  // q_0..q_{num_q-1}, p_0..p_{num_p-1}
  hipStream_t stream = nullptr;

  ModInfo* d_mod = nullptr;          // [nprimes]
  double* d_twd_fwd = nullptr;       // [nprimes][N]: psi^brev(x) at ntt_twiddle_slot(x), as doubles (exact: < 2^50)
  double* d_twd_inv = nullptr;       // [nprimes][N]: psi^-brev(x) likewise
  FpMod* d_fpm = nullptr;            // [nprimes]: (q, 1/q) as doubles
  PrimeConsts* d_pc = nullptr;       // [nprimes]
  ModUpTab* d_modup = nullptr;       // [num_q levels][dnum]
  ModDownTab* d_moddown = nullptr;   // one table (rows q_0..q_{num_q-1})
  NttScale* d_modup_scale = nullptr;    // [num_q levels][MAX_PRIMES]: N^-1 (D_j/d_i)^-1 for limb i of the level
  NttScale* d_moddown_scale = nullptr;  // [2 num_p] (rows of ROWS_SPECIAL): N^-1 (P/p_k)^-1
  RescaleTab* d_rescale = nullptr;   // [num_q]
  double* d_roots = nullptr;         // [2N][4]: exp(2 pi i j / 2N) in double-double (re hi, re lo, im hi, im lo)
  u32* d_pow5 = nullptr;             // [N/2]: 5^k mod 2N
  u64* d_gauss = nullptr;            // the error sampler's cumulative thresholds (sampler.hip), made on first use
  int2* d_rows = nullptr;            // all row tables, packed
  std::vector<int> row_off[NUM_ROW_TABLES], row_cnt[NUM_ROW_TABLES];

  std::vector<ModUpTab> h_modup;
  ModDownTab h_moddown;
  std::vector<PrimeConsts> h_pc;
  bool owns_tables = true;  // false for a context sharing another's device tables (context_share)

  Pool pool;
  Tune tune;
  int64_t counters[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // key switches per input level, and the key-switching keys read for them (one per lockstep batch that shares
  // a key, one per item otherwise): the inputs of the method's minimum HBM traffic
  int64_t ks_items[MAX_PRIMES] = {};
  int64_t ks_key_reads[MAX_PRIMES] = {};

  // Optional timing: events recorded on `stream` around every kernel launch.
  bool timing = false;
  std::vector<hipEvent_t> ev_free;
  std::vector<TimedLaunch> timed;
  hipEvent_t pending_start = nullptr;
  hipEvent_t take_event() {
    if (ev_free.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) throw std::runtime_error("hipEventCreate failed");
      return e;
    }
    hipEvent_t e = ev_free.back();
    ev_free.pop_back();
    return e;
  }
  void begin_launch() {
    if (!timing) return;
    pending_start = take_event();
    (void)hipEventRecord(pending_start, stream);
  }
  void end_launch(int cls, double bytes) {
    counters[7] += 1;
    if (!timing) return;
    hipEvent_t e = take_event();
    (void)hipEventRecord(e, stream);
    timed.push_back(TimedLaunch{pending_start, e, cls, bytes});
  }

  RowsRef rows(RowTable t, int level) const {
    return RowsRef{d_rows + row_off[t][level], row_cnt[t][level]};
  }
  int beta(int level) const { return (level + 1 + alpha - 1) / alpha; }
  int ext_prime(int level, int r) const { return r <= level ? r : num_q + (r - level - 1); }
  size_t poly_words(int level) const { return (size_t)(level + 1) * n; }
  size_t ct_words(int level) const { return 2 * poly_words(level); }
  size_t key_words() const { return (size_t)dnum * 2 * nprimes * n; }
};

void context_init(Context& c, const hetal_params& p, hipStream_t stream);
void context_free(Context& c);
// A second context on `stream` using src's parameters and device tables (not copied, not freed by it), with a pool,
// counters and timing of its own: work on two streams at once.
void context_share(Context& dst, const Context& src, hipStream_t stream);

// ---------------------------------------------------------------- kernels
// Optional separate input of a transform: row r of item b is read from
// p + b * batch_stride + (r * row_mul + row_add) * N (the output stays at base).
struct NttSrc {
  const u64* p = nullptr;
  size_t batch_stride = 0;
  int row_mul = 1, row_add = 0;
};

// NTT over `rows` (row index inside a batch item, prime index) of `batch`
// items spaced batch_stride words apart.  Input and output reduced to [0, q).
// Optional epilogue of a forward NTT over ciphertext rows (row table ROWS_CT, row r = p l + i): the
// transform x of row (p, i) is not stored; the last pass stores instead
//   out[p][i] = (a[p][i] - x) cst[i] + add0[i](gathered through tau_g, p = 0) + add1[i](p = 1) + addx[p][i]
// mod q_i, every addend optional.  ModDown ends this way (a = the Q part of the key inner product,
// cst = P^-1 mod q_i) and so does the rescale (a = the input, cst = q_l^-1 mod q_i).
//
// A key switch by tau_g (g != 1 for the item) hands over a and x in the frame before the automorphism (the keys
// are stored permuted by tau_g^-1): the epilogue then computes (a - x) cst, adds add0 there if `gather` (the
// input's c0, which the result takes as tau_g(c0)), moves the sum to its place under tau_g, and adds the other
// addends after that.  Without a permutation `gather` is ignored.
struct NttEpilogue {
  const u64* a = nullptr;
  size_t a_stride = 0;       // words between items
  int a_poly_rows = 0;       // rows between a[0][i] and a[1][i]
  int a_dbl = 0;             // a holds doubles (the key inner product's rows), not residues
  int l = 0;                 // limbs per output polynomial
  const u64* cst = nullptr;  // device array indexed by prime
  u64* out = nullptr;
  size_t out_stride = 0;
  const u64* add0 = nullptr;  // [l][N] per item
  size_t add0_stride = 0;
  int gather = 0;            // add0 is tau_g's input (added before the permutation)
  const u64* add1 = nullptr;  // [l][N] per item
  size_t add1_stride = 0;
  const u64* addx = nullptr;  // [2][l][N] per item
  size_t addx_stride = 0;
  int a_mul = 0;              // a is first multiplied by a_k[prime] (a residue of a constant, per prime)
  u64 a_k[MAX_PRIMES];
  // When set (a key switch followed by a rescale, no permutation): the rows of prime top_prime also go through
  // the inverse NTT's contiguous pass after the combine, stored as doubles at top_out + item top_out_stride +
  // p N -- the rescale's first launch, done while the rows are in registers.
  u64* top_out = nullptr;
  size_t top_out_stride = 0;
  int top_prime = -1;
  const double* tw_inv = nullptr;
  // When set (a Mult's key switch): the tensor product of the ciphertext pairs (ta[item], tb[item]), both at the
  // output's level, is computed where it is read instead of being stored -- the epilogue adds a0 b0 (rows of c0)
  // or a0 b1 + a1 b0 (rows of c1) as its addend, and the key switch's first launch (ntt_inverse_first_pass_tensor)
  // transforms a1 b1, storing it in NTT form at t_out + item t_out_stride for the inner product's own rows.
  int tensor = 0;
  const u64* ta[MAX_BATCH];
  const u64* tb[MAX_BATCH];
  // When set (a plaintext product followed by a rescale): a is first multiplied by the plaintext ta[item]
  // ([l][N], NTT form) word by word, and the rescale's first launch (ntt_inverse_first_pass_pt) multiplies its
  // rows likewise before transforming them.
  int pt_mul = 0;
  u64* t_out = nullptr;
  size_t t_out_stride = 0;
  u32 g[MAX_BATCH];           // per item: the Galois element (1: no permutation)
  u32 ginv[MAX_BATCH];        // and its inverse modulo 2N
};

// Terms of a basis conversion the key switch fuses into its NTT passes: alpha and K are at most this.
constexpr int MAX_FUSED_CONV = 4;

// Between the two passes of a transform (and between the kernels of a key switch) rows hold the bit patterns of
// exact, integer-valued doubles, not 64-bit residues: only the kernel that reads them as doubles (mid_ld in
// ntt_device.hpp) may read such a row.  Every row a launcher hands back to its caller holds residues in [0, q).
void ntt_forward(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src = NttSrc{},
                 const NttEpilogue* epi = nullptr);
void ntt_inverse(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src = NttSrc{});
// The two passes one at a time, for the key switch (keyswitch.hip), which fuses the other pass of each transform
// into its own kernels: the inverse transform's first (contiguous) pass, stored as doubles; and the forward
// transform's last (contiguous) pass over rows the forward strided pass stored as doubles, with the epilogue.
void ntt_inverse_first_pass(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src);
// The same pass on the products a1 b1 of the pairs in t (t.tensor set, rows: the l rows of c1), also storing the
// products themselves (see NttEpilogue).
void ntt_inverse_first_pass_tensor(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows,
                                   const NttEpilogue& t);
// The same pass on src's rows times the plaintexts of t (t.pt_mul set), word by word.
void ntt_inverse_first_pass_pt(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows, NttSrc src,
                               const NttEpilogue& t);
void ntt_forward_last_pass(Context& c, u64* base, size_t batch_stride, int batch, RowsRef rows,
                           const NttEpilogue& epi);

struct KsItem {
  const u64* key;  // [dnum][2][nprimes][N]
  u32 g;           // Galois element (1: none)
};

// The input polynomials must stay untouched until the switch is done (the
// digits' own rows are read from them by the inner product).
// Hybrid key switching of `count` polynomials at `level` (NTT form, [l][N] each,
// in_stride apart; in_stride = 0: one input shared by all items, whose ModUp
// is then computed once -- hoisting, bit-identical because ModUp precedes the
// automorphism).  count <= MAX_BATCH.
// out_i = (add0_i gathered by g_i (if add0) + ModDown(sum_j tau_g(ModUp_j(d)) * b_j),
//          add1_i (if add1) + ModDown(sum_j tau_g(ModUp_j(d)) * a_j)).
struct KsJob {
  int level = 0;
  int count = 0;
  const u64* in = nullptr;
  size_t in_stride = 0;
  KsItem item[MAX_BATCH];
  u64* out = nullptr;
  size_t out_stride = 0;
  const u64* add0 = nullptr;
  size_t add0_stride = 0;
  bool add0_galois = false;
  const u64* add1 = nullptr;
  size_t add1_stride = 0;
  const u64* addx = nullptr;  // optional: a ciphertext added to the result (x + Lrot(x))
  size_t addx_stride = 0;
  u64* top_out = nullptr;  // optional ([count][2][N] doubles): the result's top rows through the inverse
                           // contiguous pass, for the rescale that follows (items without a permutation only)
  // A Mult's relinearisation: the input is the tensor product of the pairs (ta[i], tb[i]) at `level`, computed
  // on the fly (`in`, add0 and add1 unused; the result is (d0, d1) + the switched d2)
  bool tensor = false;
  const u64* ta[MAX_BATCH];
  const u64* tb[MAX_BATCH];
};
void key_switch(Context& c, const KsJob& job);
// Device words of the temporaries key_switch leases from the pool for a job of `count` distinct inputs at
// `level` (each buffer rounded up to the arena's 256-byte granule).
size_t key_switch_scratch_words(const Context& c, int level, int count);

// The library's static scratch region of the device that is current (see noalloc.hip): looked up once per
// device, at context creation; scratch_region returns it for a device already set up.
void scratch_setup();
u64* scratch_region(int device, size_t* words);

// Elementwise kernels on [rows][N] arrays whose row i is modulo prime (i mod period).
void k_add(Context& c, const u64* a, const u64* b, u64* out, int rows, int period);
void k_sub(Context& c, const u64* a, const u64* b, u64* out, int rows, int period);
// out[item] = a[item] ± b[item] at `level` (packed), reading each operand's first level + 1 rows of each of its
// two polynomials (a_rows, b_rows: the operand's rows per polynomial; a_stride, b_stride: words between items).
void k_addsub_rows(Context& c, const u64* a, size_t a_stride, int a_rows, const u64* b, size_t b_stride, int b_rows,
                   u64* out, int level, int count, bool subtract);
void k_mul_rows(Context& c, const u64* a, const u64* b, u64* out, int rows, int period, int b_period);
void k_mul_i(Context& c, const u64* a, u64* out, int rows, int period);
void k_galois(Context& c, const u64* a, u64* out, int rows, int period, u32 g);
void k_tensor(Context& c, const u64* a, const u64* b, u64* d01, u64* d2, int level);
// Rescale of `batch` ciphertexts (keyswitch.hip: ModDown's three-launch pipeline from the single prime q_level).
// kconst (host, level + 1 residues, or null): rescale the ciphertexts times the constant with these residues
// instead, in the same three launches.  in_poly_rows (0: level + 1): rows between the input's two polynomials,
// more for an input at a higher level, whose first level + 1 limbs are used (a mod-drop on the fly).
// addx (or null): a ciphertext at level - 1 per item, addx_stride words apart, added to each result.
// top_ready (or null): the two top rows of every item already through the inverse contiguous pass ([batch][2][N]
// doubles, from a key switch's epilogue): the first launch is skipped.
// pts (host, `batch` pointers to plaintexts at `level`, or null): rescale the ciphertexts times these plaintexts
// instead (a CMult and its rescale in the rescale's three launches).
void k_rescale(Context& c, const u64* in, u64* out, int level, int batch, size_t in_stride, size_t out_stride,
               const u64* kconst = nullptr, int in_poly_rows = 0, const u64* addx = nullptr, size_t addx_stride = 0,
               const u64* top_ready = nullptr, const u64* const* pts = nullptr);
void k_reduce_signed(Context& c, const i64* coeffs, u64* out, RowsRef rows, int batch, size_t coeff_stride,
                     size_t out_stride);
void k_encrypt(Context& c, const u64* a_ntt, const u64* e_ntt, const u64* m, const u64* s, u64* ct, int level);
void k_decrypt(Context& c, const u64* ct, const u64* s, u64* m, int level);
// A switching key for s' (NTT form) in the layout key_switch reads: g is the Galois element the key serves
// (1 for relinearisation); see keygen_kernel.
void k_keygen(Context& c, const u64* a_ntt, const u64* e_ntt, const u64* s, const u64* sp, u64* key, u32 g);

// Encoding (double-double) and decoding.
void k_encode(Context& c, const double* d_re, const double* d_im, int count, size_t slot_stride, int level,
              double scale, u64* out, size_t out_stride, int* d_status);
void k_decode(Context& c, const u64* m_coeff, int level, double scale, double* d_re, double* d_im);
void k_block_layout(Context& c, const double* d_mat, int rows, int cols, int tiling, int c_rep, int s0, int s1,
                    int n_rb, int n_cb, double* d_slots);

}  // namespace hetal
