/*
 * hetal.h -- C ABI of the MI355X (gfx950) library for encrypted matrix
 * products over RNS-CKKS ciphertexts: the DiagABT and DiagATB algorithms of
 * "HETAL: Efficient Privacy-preserving Transfer Learning with Homomorphic
 * Encryption" (ICML 2023), Sec. 4.2 and App. B (Alg. 1-4), and the CKKS
 * operations they are built from (Sec. 2.2).
 *
 * Conventions
 *  - Every call returns an int status: HETAL_OK (0) or a negative HETAL_E_*
 *    code; hetal_last_error() gives the message of the calling thread's last
 *    failure.  On failure no output is valid.
 *  - Ciphertexts and plaintexts live in device memory that the CALLER owns
 *    (for instance a torch tensor); the structs below carry the pointer, its
 *    capacity in 64-bit words, the level and the FP64 scale.  The library
 *    never frees caller memory.  Outputs must have room for the result
 *    (capacity checked; E_INVALID_ARG otherwise) and get level and scale
 *    written.  An output may alias an input.
 *  - Device layout: a polynomial at level l is uint64 [l+1][N], limb-major,
 *    row i holding the residues modulo q_i in [0, q_i), in the NTT domain in
 *    the library's internal (bit-reversed) evaluation order.  A ciphertext is
 *    uint64 [2][l+1][N].  hetal_ct_to_coeff gives the canonical coefficient
 *    form, the only form meant for comparison with other implementations.
 *  - Host arrays are plain C arrays, row-major, as described per call.
 *  - All device work is queued on the context's HIP stream (set at creation
 *    or by hetal_ctx_set_stream).  Calls that return host data synchronise
 *    that stream first.  A context is not thread-safe.
 *  - Randomness: either an input (the secret key's coefficients, every key
 *    switching key's uniform mask and error, every encryption's mask and
 *    error supplied by the caller), or drawn by the library from a 64-bit seed
 *    (the *_seeded calls, hetal_keygen, hetal_gen_evk; see "Seeded sampling"
 *    below).  Either way results are deterministic.
 */
#ifndef HETAL_H
#define HETAL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HETAL_OK = 0,
  HETAL_E_INVALID_ARG = -1, /* null pointer, bad size, capacity too small */
  HETAL_E_SHAPE = -2,       /* matrix shape / tiling precondition violated */
  HETAL_E_LEVEL = -3,       /* not enough levels left (depth exhausted) */
  HETAL_E_NO_KEY = -4,      /* a needed relinearisation or Galois key is missing */
  HETAL_E_SCALE = -5,       /* operands with incompatible scales */
  HETAL_E_OOM = -6,         /* device allocation failed */
  HETAL_E_DEVICE = -7,      /* HIP runtime error */
  HETAL_E_PARAMS = -8,      /* unsupported parameter set */
  HETAL_E_OVERFLOW = -9     /* an encoded coefficient does not fit in 62 bits */
};

typedef struct hetal_ctx hetal_ctx;
typedef struct hetal_sk hetal_sk;
typedef struct hetal_keys hetal_keys;

/* Parameter set.  N = 2^log_n (12 <= log_n <= 16); q_0 is the largest prime
 * below 2^q0_bits, q_1..q_{num_q-1} the largest primes below 2^q_bits in
 * descending order, and the num_p special primes p_0.. the largest primes
 * below q_0; all are 1 mod 2N (q0_bits, q_bits <= 50).  dnum digits of
 * alpha = ceil(num_q / dnum) consecutive primes are used for hybrid key
 * switching.  Limits: num_q + num_p <= 32, alpha <= 4, num_p <= 4, at most 8 digits. */
typedef struct {
  int log_n;
  int num_q;
  int num_p;
  int dnum;
  int q0_bits;
  int q_bits;
} hetal_params;

typedef struct {
  uint64_t* data;  /* device, [2][level+1][N] */
  size_t capacity; /* 64-bit words available at data */
  int level;
  double scale;
} hetal_ct;

typedef struct {
  uint64_t* data;  /* device, [level+1][N] */
  size_t capacity;
  int level;
  double scale;
} hetal_pt;

/* An encrypted block matrix (App. B.1): the matrix is zero padded to
 * multiples of s0 x s1 (s0 * s1 = N/2) and cut into n_rb x n_cb blocks, block
 * (i, j) written row-major into the slots of ciphertext i * n_cb + j.
 * data: device, [n_rb * n_cb][2][level+1][N]. */
typedef struct {
  uint64_t* data;
  size_t capacity;
  int n_rb;
  int n_cb;
  int s0;
  int s1;
  int level;
  double scale;
} hetal_mat;

/* ---- Seeded sampling (the client's randomness, Sec. 3.1: the client generates the secret key and the public
 * operation keys, and encrypts).  The generator is the ChaCha20 block function of RFC 8439 used as a counter-based
 * stream: stream (seed, purpose, index, sub) has key = the seed (low 32 bits, high 32 bits, then six zero words),
 * nonce = (purpose, index, sub) and block counter = the block number; its 64-bit word p is the little-endian word
 * p mod 8 of block p / 8.  Purposes: 1 the secret; 2 a switching key's uniform masks (index = the key id: 0 for the
 * relinearisation key, else its Galois element; sub = digit * 64 + prime index over all primes); 3 its errors
 * (sub = digit); 4 an encryption's masks (index = the encryption's number, sub = prime index); 5 its error
 * (sub = 0).  Distributions, per coefficient k < N:
 *  - uniform modulo q: the first of the stream's words k, N + k, 2N + k, ... below floor(2^64 / q) q, mod q;
 *  - error: word k; its top bit is the sign, its low 63 bits u give the magnitude #{j < 19 : T_j <= u}, T_j =
 *    floor(2^63 P(|x| <= j)) for the rounded Gaussian of standard deviation 3.2 on |x| <= 19
 *    (hetal_gaussian_table); one value per coefficient, reduced modulo every prime;
 *  - secret: exactly min(192, N) coefficients +-1: word p names position (word mod N) and sign (top bit), in
 *    order, positions already set skipped. */

/* The error sampler's 19 thresholds (host, ascending).  *n: in, capacity (>= 19); out, 19.  No context needed. */
int hetal_gaussian_table(uint64_t* out, int* n);
/* Samples for tests and for callers that keep their own randomness: the ternary secret of `seed` with h
 * nonzero coefficients (host int64 [2^log_n]; no context needed); `rows` rows of uniform residues (host uint64
 * [rows][N], coefficient form; row r is the stream of sub (r / group) * 64 + r % group, modulo prime r % group,
 * group <= num_q + num_p); `count` rows of errors (host int64 [count][N], row r the stream of sub r). */
int hetal_sample_ternary(int log_n, uint64_t seed, int h, int64_t* out);

/* The message of the last failed call on the calling thread (a failed call
 * sets it; successful calls leave it).  Owned by the library, valid until
 * the thread's next failing call. */
const char* hetal_last_error(void);

/* Context: parameters, precomputed tables (roots of unity, basis-conversion
 * constants, double-double FFT roots) and a device memory pool for
 * temporaries.  `stream` is a hipStream_t (NULL = default stream).
 * E_PARAMS if the parameter set is outside the limits above. */
int hetal_ctx_create(const hetal_params* params, void* stream, hetal_ctx** out);
/* A context on `stream` that shares base's parameters and precomputed device tables (not copied), with a memory
 * pool, mask cache, counters and timing of its own: for independent work on several streams at once (a request
 * loop's lanes).  Secret keys and evaluation keys made with base serve it too (same parameters, same layout).
 * base must outlive it; destroying it frees only what it owns. */
int hetal_ctx_create_shared(hetal_ctx* base, void* stream, hetal_ctx** out);
/* Whether hetal_enc_matmul_batch may run independent shape classes on the context's second stream (on by
 * default; hetal_autotune_batch and hetal_tune_set choose it again, hetal_tune_reset turns it back on).  Lanes
 * of a request loop turn it off: HIP maps streams onto a few hardware queues, and a second stream that waits on
 * its lane's work can hold up another lane that shares its queue.  E_INVALID_ARG for a null context. */
int hetal_ctx_set_two_streams(hetal_ctx* ctx, int enable);
void hetal_ctx_destroy(hetal_ctx* ctx);
int hetal_ctx_set_stream(hetal_ctx* ctx, void* stream);
/* n: ring degree; slots: N/2; max_level: num_q - 1; num_primes: num_q + num_p. */
int hetal_ctx_info(const hetal_ctx* ctx, int* n, int* slots, int* max_level, int* num_primes);
/* Writes q_0..q_{num_q-1}, p_0..p_{num_p-1} to out (host, num_q + num_p words). */
int hetal_ctx_primes(const hetal_ctx* ctx, uint64_t* out);
int hetal_synchronize(hetal_ctx* ctx);
/* Galois elements: left rotation by r slots is X -> X^(5^r mod 2N) (r < 0:
 * right rotation); conjugation is X -> X^(2N-1) (Sec. 2.2: Lrot, conj). */
uint64_t hetal_galois_rot(const hetal_ctx* ctx, int r);
uint64_t hetal_galois_conj(const hetal_ctx* ctx);

/* Secret key from its N signed coefficients (host int64, each in {-1,0,1}).
 * The key is stored on the device in NTT form over every prime. */
int hetal_sk_create(hetal_ctx* ctx, const int64_t* s_coeffs, hetal_sk** out);
void hetal_sk_destroy(hetal_sk* sk);

/* The client's secret key drawn from `seed`: ternary with min(192, N) nonzero coefficients (seeded sampling). */
int hetal_keygen(hetal_ctx* ctx, uint64_t seed, hetal_sk** out);
int hetal_sample_uniform(hetal_ctx* ctx, uint64_t seed, uint32_t purpose, uint32_t index, int rows, int group,
                         uint64_t* host);
int hetal_sample_gaussian(hetal_ctx* ctx, uint64_t seed, uint32_t purpose, uint32_t index, int count, int64_t* host);

/* Evaluation keys (public operation keys, Sec. 3.1), held in library-owned
 * device memory: 2 * dnum * (num_q + num_p) * N words per key.
 * Key for s' (s^2 for relinearisation, tau_g(s) for Galois element g):
 *   ksk_j = (-a_j s + e_j + g_j s', a_j), j < dnum, over all primes, where
 *   g_j = P mod q_i for q_i in digit j and 0 otherwise (0 modulo each p_k).
 * a: host uint64 [dnum][num_q + num_p][N], uniform modulo each prime,
 *    coefficient form (E_INVALID_ARG if a word is not below its prime);
 *    e: host int64 [dnum][N], small signed errors. */
int hetal_keys_create(hetal_ctx* ctx, hetal_keys** out);
void hetal_keys_destroy(hetal_keys* keys);
int hetal_keys_gen_relin(hetal_ctx* ctx, hetal_keys* keys, const hetal_sk* sk, const uint64_t* a, const int64_t* e);
int hetal_keys_gen_galois(hetal_ctx* ctx, hetal_keys* keys, const hetal_sk* sk, uint64_t galois, const uint64_t* a,
                          const int64_t* e);
/* The evaluation keys an algorithm needs, with the library's own randomness from `seed`: the relinearisation
 * key (if relin), the Galois key of every rotation step in rot_steps[0 .. n-1] (left rotation by r; steps that
 * are 0 mod N/2 need none; duplicates are made once), and the conjugation key (if conj).  Existing keys for the
 * same elements are replaced.  hetal_required_rot_steps lists the steps of DiagABT / DiagATB. */
int hetal_gen_evk(hetal_ctx* ctx, hetal_keys* keys, const hetal_sk* sk, uint64_t seed, const int32_t* rot_steps,
                  int n, int conj, int relin);

/* Encoding (Sec. 2.2, CKKS): slot k of the message is the value of the
 * plaintext polynomial at zeta^(5^k), zeta = exp(i pi / N).  The
 * coefficients round(scale * sigma^-1(z)) are computed in double-double
 * arithmetic and rounded half to even, values within 2^-24 of a half-integer
 * counting as halves.  re, im: host double [N/2] (im may be NULL).
 * E_OVERFLOW if a coefficient reaches 2^62.  out->capacity >= (level+1)*N. */
int hetal_encode(hetal_ctx* ctx, const double* re, const double* im, int level, double scale, hetal_pt* out);
/* Slots of a plaintext (centred CRT of its first two limbs, divided by its
 * scale).  re, im: host double [N/2] (im may be NULL).  Synchronises. */
int hetal_decode(hetal_ctx* ctx, const hetal_pt* pt, double* re, double* im);

/* Secret-key encryption (c0, c1) = (-a s + m + e, a) at the plaintext's
 * level.  a: host uint64 [level+1][N] uniform modulo q_i, coefficient form
 * (E_INVALID_ARG if a word is not below its prime); e: host int64 [N]. */
int hetal_encrypt(hetal_ctx* ctx, const hetal_sk* sk, const hetal_pt* pt, const uint64_t* a, const int64_t* e,
                  hetal_ct* out);
/* hetal_encrypt with the library's own randomness: the masks and error of encryption number `index` under `seed`. */
int hetal_encrypt_seeded(hetal_ctx* ctx, const hetal_sk* sk, const hetal_pt* pt, uint64_t seed, uint32_t index,
                         hetal_ct* out);
/* m = c0 + c1 s. */
int hetal_decrypt(hetal_ctx* ctx, const hetal_sk* sk, const hetal_ct* ct, hetal_pt* out);

/* Homomorphic operations (Sec. 2.2).  Operands of add/sub/hmult must share
 * level (E_LEVEL) and scale up to a relative 1e-9 (E_SCALE). */
int hetal_add(hetal_ctx* ctx, const hetal_ct* a, const hetal_ct* b, hetal_ct* out);
int hetal_sub(hetal_ctx* ctx, const hetal_ct* a, const hetal_ct* b, hetal_ct* out);
/* Multiplication by i in every slot (by X^(N/2)): exact, no level used. */
int hetal_mul_i(hetal_ctx* ctx, const hetal_ct* a, hetal_ct* out);
/* CMult: (c0 m, c1 m); the scale multiplies.  pt->level must equal ct->level. */
int hetal_cmult(hetal_ctx* ctx, const hetal_ct* ct, const hetal_pt* pt, hetal_ct* out);
/* Mult: tensor product, then relinearisation of the s^2 term (no rescale). */
int hetal_hmult(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* a, const hetal_ct* b, hetal_ct* out);
/* Lrot(ct, r): slot j receives slot j + r (r < 0 rotates right).  Hybrid key
 * switching: ModUp of c1 per digit, the automorphism applied to the extended
 * digits, inner product with the key, ModDown with a centred basis
 * conversion; plus tau_g(c0).  E_NO_KEY without the Galois key. */
int hetal_hrot(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* ct, int r, hetal_ct* out);
/* HRot of `count` ciphertexts at one level: out[i] = Lrot(in[i], steps[i]) (Sec. 2.2), as one batched key
 * switch per group of up to 32 rotations; rotations that share a step share the key's loads.  A step that
 * is 0 mod N/2 copies.  Inputs evenly spaced in one allocation, and outputs likewise, are used in place;
 * other layouts go through a packed device copy.  Outputs must not overlap the inputs or each other
 * (E_INVALID_ARG).  All inputs at one level (E_LEVEL); each output keeps its input's scale.  E_NO_KEY
 * without a step's Galois key. */
int hetal_hrot_batch(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* in, const int* steps, int count,
                     hetal_ct* out);
/* hetal_hrot without device allocation, for callers that cannot allocate: code recorded into a HIP graph,
 * tight serving loops, harnesses that forbid hipMalloc.  Same result as hetal_hrot, word for word.  The key
 * switch's temporaries live in a fixed 64 MiB static device region (one per GPU, held until the process
 * ends) instead of the context's pool; a rotation needs (l + beta (l + K) + 2 (l + K) + 2 l) N words for l =
 * level + 1 limbs, K special primes and beta digits, i.e. 63 MiB at N = 2^16, level 11, K = 3, dnum = 4.
 * E_INVALID_ARG if that exceeds the region, if out->data == ct->data (in place would need a copy) or while
 * per-kernel timing is on; other errors as hetal_hrot.  Every call on a GPU shares that GPU's region:
 * calls that overlap on one GPU (contexts on different streams, several threads) race and must be
 * serialised by the caller. */
int hetal_hrot_noalloc(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* ct, int r, hetal_ct* out);
/* Slot-wise complex conjugation (Galois element 2N-1). */
int hetal_conj(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* ct, hetal_ct* out);
/* Rescale: c_i <- (c_i - [c_l]_centred) q_l^-1 mod q_i, level - 1, scale / q_l.
 * E_LEVEL at level 0. */
int hetal_rescale(hetal_ctx* ctx, const hetal_ct* ct, hetal_ct* out);
/* Drop the limbs above `level`; the scale is unchanged. */
int hetal_mod_drop(hetal_ctx* ctx, const hetal_ct* ct, int level, hetal_ct* out);

/* Canonical coefficient form (host uint64 [2][level+1][N] resp. [level+1][N]);
 * synchronises.  from_coeff is the inverse. */
int hetal_ct_to_coeff(hetal_ctx* ctx, const hetal_ct* ct, uint64_t* host);
int hetal_pt_to_coeff(hetal_ctx* ctx, const hetal_pt* pt, uint64_t* host);
int hetal_ct_from_coeff(hetal_ctx* ctx, const uint64_t* host, int level, double scale, hetal_ct* out);

/* Block-encode and encrypt a host matrix (double, row-major rows x cols).
 * tiling: 0 none; 1 vertical (the c x cols matrix repeated s0 / c times
 * down, the B-bar of Alg. 1); 2 horizontal (the rows x c matrix repeated
 * s1 / c times across, the A-underbar of Alg. 4).  The caller sets
 * out->s0 (s1 = N/2 / s0), out->level and out->scale; the library sets n_rb,
 * n_cb.  a: host uint64 [n_rb*n_cb][level+1][N], each word below its prime
 * (else E_INVALID_ARG); e: host int64 [n_rb*n_cb][N].
 * E_SHAPE for an empty matrix (rows or cols 0, checked before anything
 * else), or if c does not divide the tiled dimension. */
int hetal_mat_encrypt(hetal_ctx* ctx, const hetal_sk* sk, const double* host, int rows, int cols, int tiling, int c,
                      const uint64_t* a, const int64_t* e, hetal_mat* out);
/* hetal_mat_encrypt with the library's own randomness: block b is encryption number first_index + b under seed. */
int hetal_mat_encrypt_seeded(hetal_ctx* ctx, const hetal_sk* sk, const double* host, int rows, int cols, int tiling,
                             int c, uint64_t seed, uint32_t first_index, hetal_mat* out);
/* Decrypt and decode every block: host double [n_rb*s0][n_cb*s1] (real
 * parts; padding included).  Synchronises. */
int hetal_mat_decrypt(hetal_ctx* ctx, const hetal_sk* sk, const hetal_mat* m, double* host);

/* DiagABT (Alg. 1, Prop. 1): <t A Bbar^T> from <A> (n_rb x n_cb blocks) and
 * <Bbar> (1 x n_cb blocks, B tiled vertically).  c: rows of B padded to a
 * power of two, 1 < c <= s0, c | s1.  out: n_rb x 1 blocks at level
 * min(level A, level Bbar) - 3; block i slot (r, j) holds
 * t (A B^T)[i s0 + r][j mod c].  Needs the relinearisation key, the
 * conjugation key and Galois keys for the steps hetal_required_rot_steps
 * lists.  CS uses 2 log s1 rotations and one CMult, RS log s0 rotations. */
int hetal_enc_matmul_abt(hetal_ctx* ctx, const hetal_keys* keys, const hetal_mat* a, const hetal_mat* bbar, int c,
                         double t, hetal_mat* out);
/* DiagATB (Alg. 4, Prop. 2): <t Abar^T B> from <Abar> (n_rb x 1 blocks, A
 * tiled horizontally) and <B> (n_rb x n_cb blocks).  out: 1 x n_cb blocks;
 * block j slot (r, col) holds t (A^T B)[r mod c][j s1 + col].  When
 * level(Abar) < level(B) the PRotUp branch runs (output level
 * min(lA - 1, lB - 1) - 2), else the RotLeft branch (min(lA - 2, lB) - 2). */
int hetal_enc_matmul_atb(hetal_ctx* ctx, const hetal_keys* keys, const hetal_mat* abar, const hetal_mat* b, int c,
                         double t, hetal_mat* out);
/* One request of a batched call: op 0 = DiagABT (a = <A>, b = <Bbar>), op 1 =
 * DiagATB (a = <Abar>, b = <B>), with c and t as in the single calls. */
typedef struct {
  int op;
  const hetal_mat* a;
  const hetal_mat* b;
  int c;
  double t;
} hetal_matmul_req;

/* Many products, of any mix of shapes, in one call: outs[i] receives exactly
 * what hetal_enc_matmul_abt / _atb would return for reqs[i] (bit-identical
 * ciphertexts, same levels and scales).  Requests that share (op, c, s0,
 * input levels, input scales) run in lockstep, so every step of their
 * algorithm -- each rotation step, relinearisation, rescale, mask product --
 * is one batched launch sequence over all of their ciphertexts, with the
 * key read once per step; groups run one after the other.  Errors as in the
 * single calls; on an error no output is written (checked before any work). */
int hetal_enc_matmul_batch(hetal_ctx* ctx, const hetal_keys* keys, const hetal_matmul_req* reqs, int count,
                           hetal_mat* outs);

/* ---- Schedule choices and the autotuner.  Every choice below leaves every result unchanged, word for word; they
 * trade launch sizes, parallelism and recomputation.  ks_group: the most key switches one launch sequence takes
 * (1..32); tpt_modup / tpt_moddown: target primes per workgroup task of the key switch's ModUp / ModDown kernels
 * (each task recomputes its sources' inverse transforms; 0 = the library's rule); two_streams: independent shape
 * classes of a batch alternate between the context's stream and a second one; work_cts: the working-set limit of
 * a product, in ciphertexts at its level (0 = 2 GiB worth): the products of the k loop (DiagABT) or of the block
 * columns (DiagATB) are made that many at a time and summed into place, and requests of one class run in lockstep
 * while their run sums fit.  A shape class of
 * hetal_enc_matmul_batch is (op, c, s0, level of A, level of B) (for DiagABT both levels are min(level A, level
 * Bbar)). */
typedef struct {
  int ks_group;
  int tpt_modup;
  int tpt_moddown;
  int two_streams;
  int work_cts;
} hetal_tune;

typedef struct {
  double untuned_ms; /* median time of the batch with the defaults */
  double tuned_ms;   /* ... with the chosen schedules */
  int classes;       /* shape classes in the batch */
  int trials;        /* timed runs of a class or of the batch */
  int two_streams;   /* the choice made for the batch */
} hetal_tune_report;

/* The autotuner: times `reps` runs (median) of each shape class of the batch alone under candidate schedules
 * (coordinate descent over ks_group in {32, 16, 8, 4}, tpt_modup in {default, 2, 4, 6, 12}, tpt_moddown in
 * {default, 2, 3, 6, 12}; a candidate must beat the current choice by 2%), keeps the best per class in the
 * context, then chooses two_streams for the whole batch.  Later hetal_enc_matmul_batch calls (and graphs
 * recorded after) use the choices; outs receive the batch's results.  Errors as hetal_enc_matmul_batch. */
int hetal_autotune_batch(hetal_ctx* ctx, const hetal_keys* keys, const hetal_matmul_req* reqs, int count,
                         hetal_mat* outs, int reps, hetal_tune_report* report);
/* The schedule a shape class runs with (the defaults if none was chosen), and setting it by hand; reset returns
 * every class to the defaults. */
int hetal_tune_get(const hetal_ctx* ctx, int op, int c, int s0, int level_a, int level_b, hetal_tune* out);
int hetal_tune_set(hetal_ctx* ctx, int op, int c, int s0, int level_a, int level_b, const hetal_tune* in);
int hetal_tune_reset(hetal_ctx* ctx);

/* The products of hetal_enc_matmul_batch recorded into a HIP graph, for callers that repeat the same batch (a
 * training loop over fixed buffers, a serving loop): the call runs the batch twice eagerly (encoding the masks
 * and sizing the library's buffer pools), then records the same work, both streams included, into a graph and
 * returns it; hetal_graph_launch replays it on the context's stream, reading the requests' input matrices and
 * writing `outs` again (their contents at launch time are what is used).  The graph keeps pointers to the
 * inputs, outputs and library buffers: keep all of them alive and unmoved, and the keys unchanged, until
 * hetal_graph_destroy.  The context must be on a stream it was given (not the legacy default stream; E_INVALID_ARG)
 * and per-kernel timing off.  Errors as hetal_enc_matmul_batch; E_DEVICE if the capture fails. */
typedef struct hetal_graph hetal_graph;
int hetal_enc_matmul_batch_graph(hetal_ctx* ctx, const hetal_keys* keys, const hetal_matmul_req* reqs, int count,
                                 hetal_mat* outs, hetal_graph** out);
int hetal_graph_launch(hetal_graph* g);
void hetal_graph_destroy(hetal_graph* g);

/* Rotation steps (signed, left positive) the algorithms need, for key
 * generation: op 0 = DiagABT, 1 = DiagATB (RotLeft branch), 2 = DiagATB
 * (PRotUp branch).  *n: in, capacity of out; out, count written. */
int hetal_required_rot_steps(const hetal_ctx* ctx, int op, int c, int s0, int32_t* out, int* n);

/* ---- Constants and the softmax approximation (App. softmax) ----
 *
 * CMult by a real constant: both polynomials times the integer K = round(value * sigma) (ties to even),
 * no level used; the scale becomes ct->scale * sigma (rescale afterwards to consume one level; sigma =
 * q_level keeps the scale).  E_OVERFLOW when |K| >= 2^62. */
int hetal_cmult_const(hetal_ctx* ctx, const hetal_ct* ct, double value, double sigma, hetal_ct* out);
/* value added to every slot: K = round(value * scale) added to c0's constant coefficient.  E_OVERFLOW as above. */
int hetal_add_const(hetal_ctx* ctx, const hetal_ct* ct, double value, hetal_ct* out);
/* ct + pt (c0 + m): pt at ct's level (E_LEVEL) and scale up to 1e-9 (E_SCALE). */
int hetal_add_plain(hetal_ctx* ctx, const hetal_ct* ct, const hetal_pt* pt, hetal_ct* out);
/* Re-encryption by the key holder, standing in for bootstrapping (which this library does not provide):
 * decrypt, lift the plaintext polynomial m from q_0 (its centred residue; every other limb must agree,
 * i.e. |m| < q_0 / 2, else E_OVERFLOW), re-encode it at `scale` as rint(m * scale / ct->scale) (ties to
 * even; scale 0 keeps the scale and m), encrypt at the top level with the caller's randomness (a: host
 * uint64 [num_q][N] uniform modulo each ciphertext prime, each word below it (else E_INVALID_ARG), e: host int64
 * [N]).  out may alias ct and needs
 * room for the top level.  This hands the ciphertext to the client: it is outside the paper's threat model
 * and meant for pipelines deeper than the modulus chain.  Re-encoding at a fixed scale (2^40) keeps chains
 * of squarings from driving the scale away from the primes. */
int hetal_refresh(hetal_ctx* ctx, const hetal_sk* sk, const hetal_ct* ct, double scale, const uint64_t* a,
                  const int64_t* e, hetal_ct* out);

/* Called by the deep pipelines below when a ciphertext has fewer levels than its next step needs: it
 * must overwrite *ct (the library's buffer, with room for the top level; do not change ct->data) with an
 * encryption of the same message at the top level, e.g. by hetal_refresh, and return HETAL_OK; the library
 * reads back the new scale (the items of one batch must get the same one).  Other return values abort the
 * pipeline with that code. */
typedef int (*hetal_refresh_fn)(void* user, hetal_ct* ct);

/* sum_k coeffs[k] x^k (degree >= 1) in the power basis: x^k = x^a x^b with a the largest power of two
 * below k (k/2 twice for a power of two), each product relinearised and rescaled; every term brought to
 * the lowest level by mod-drop and multiplied by coeffs[k] at the scale that lands on ct's scale; the
 * constant term added last.  The result has ct's scale (to rounding) and sits max_k (depth of x^k) + 1
 * levels lower.  If ct has fewer levels, it is first passed to `refresh` (E_LEVEL without one).
 * out needs room for the top level. */
int hetal_poly_eval(hetal_ctx* ctx, const hetal_keys* keys, const hetal_ct* ct, const double* coeffs, int degree,
                    hetal_refresh_fn refresh, void* user, hetal_ct* out);

/* Parameters of the softmax approximation (App. softmax).  Defaults from hetal_softmax_default_params:
 * R = 8, L = 2, n = 5 (inputs in [-128, 128]), precise = 1, extend = 1, comp_g = 3, exp_B = 8,
 * exp_degree = 12 with the L^2 projection of e^t on [-1, 1], inv_R = 100, inv_iters = 16. */
typedef struct {
  double R;              /* AExp's range [-R, R], the base interval of the domain extension */
  double L;              /* domain extension ratio */
  int n;                 /* domain extension steps: inputs up to L^n R / 2 in magnitude */
  int precise;           /* apply the degree-5 inverse correction after the extension */
  int extend;            /* apply the domain extension at all */
  int comp_g;            /* compositions of g in the comparison f(g(..g(x))) */
  int exp_B;             /* AExp(x) = p(x / B)^B; a power of two */
  int exp_degree;        /* degree of p, at most 31 */
  double exp_coeffs[32]; /* monomial coefficients of p(x / B), [0 .. exp_degree] */
  double inv_R;          /* AInv's scaling: Goldschmidt's iteration on x / inv_R, converging for x < 2 inv_R */
  int inv_iters;         /* Goldschmidt steps */
} hetal_softmax_params;

/* Fills the defaults above (no context needed). */
int hetal_softmax_default_params(hetal_softmax_params* out);
/* Rotation steps hetal_softmax_approx needs, for key generation (as hetal_required_rot_steps). */
int hetal_softmax_rot_steps(const hetal_ctx* ctx, int c, int s0, int32_t* out, int* n);
/* Row-wise softmax approximation (Alg. "Row-wise softmax approximation"): m is the encryption of an
 * a x c matrix tiled horizontally (tiling 2 of hetal_mat_encrypt with c' = the power of two >= c;
 * n_cb = 1; E_SHAPE otherwise); out receives ASoftmax(m) in the same layout, zero in the padded
 * classes.  The pipeline needs about 100 levels: whenever an operand has fewer than its next step
 * needs, it is passed to `refresh` (E_LEVEL without one).  *refreshes (may be NULL) receives the
 * number of refresh calls.  out needs room for n_rb ciphertexts at the top level.  Where the paper is
 * silent or garbled the library takes the readings stated at the top of its softmax source. */
int hetal_softmax_approx(hetal_ctx* ctx, const hetal_keys* keys, const hetal_mat* m, int c,
                         const hetal_softmax_params* params, hetal_refresh_fn refresh, void* user, hetal_mat* out,
                         int* refreshes);

/* One step of the encrypted training loop (the protocol's step 3(a), Sec. 3's NAG update):
 *   P = ASoftmax(X V^T),  W_out = V - lr (P - Y)^T X,  V_out = (1 - gamma) W_out + gamma W,
 * with lr = alpha / N (learning rate over batch size) and gamma the schedule's gamma_t, both chosen by the
 * caller.  X: a x b features, untiled (n_rb x n_cb blocks).  Y: a x c one-hot labels tiled horizontally with
 * c' = the power of two >= c (n_rb x 1).  W, V: c x b weights tiled vertically (1 x n_cb; tiling 1 of
 * hetal_mat_encrypt with c').  X V^T is DiagABT (Alg. 1) and the gradient DiagATB (Alg. 4, t = -lr).  X and V
 * are refreshed below 3 levels, P - Y below 4, and the softmax refreshes as in hetal_softmax_approx (E_LEVEL
 * without a refresh callback).  E_SHAPE unless 2 <= c, c' <= s0 and c' | s1.  W_out and V_out (distinct) need
 * room for n_cb ciphertexts at the top level; *refreshes (may be NULL) counts all refresh calls. */
int hetal_nag_step(hetal_ctx* ctx, const hetal_keys* keys, const hetal_mat* x, const hetal_mat* y, const hetal_mat* w,
                   const hetal_mat* v, int c, double lr, double gamma, const hetal_softmax_params* params,
                   hetal_refresh_fn refresh, void* user, hetal_mat* w_out, hetal_mat* v_out, int* refreshes);

/* Operation counters since the last reset: [0] rotations, [1] conjugations,
 * [2] Mult, [3] CMult, [4] rescales, [5] key switches, [6] NTT limb
 * transforms, [7] kernel launches. */
int hetal_counters_get(const hetal_ctx* ctx, int64_t* out8);
int hetal_counters_reset(hetal_ctx* ctx);
/* Key switches since the last hetal_counters_reset, by input level: items[l] key switches of ciphertexts at
 * level l, and key_reads[l] the key-switching keys they read (once per batch of items that share a key, once
 * per item otherwise).  They fix the minimum HBM traffic of the work (Sec. 5.1 prices the operations, the
 * key switch dominating): each item reads its input and writes its output, 2 (l + 1) limbs each, and each key
 * read moves 2 beta (l + 1 + num_p) limbs, beta = the digits at level l.  Host arrays of `levels` entries
 * (levels above the chain read 0). */
int hetal_ks_counts(const hetal_ctx* ctx, int64_t* items, int64_t* key_reads, int levels);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch (adds two event records per launch while enabled).  There are
 * hetal_timing_classes() classes: [0] forward NTT, strided first pass,
 * [1] the key switch's ModUp kernel (inverse strided pass of the input, the
 * ModUp basis conversion, forward strided pass of the extended digits),
 * [2] its ModDown kernel (the same around the ModDown conversion of the
 * special rows), [3] forward NTT, contiguous final pass, [4] the same pass
 * ending a key switch or rescale (it also subtracts, scales and adds: the
 * ModDown / rescale combine), [5] inverse NTT, contiguous first pass,
 * [6] inverse NTT, strided final pass, [7] the key inner product (with the
 * forward contiguous pass of the extended digits before it and the inverse
 * contiguous pass of the special rows after it), [8] the rescale's conversion
 * kernel (inverse strided pass of the top limbs, their centred lift to every
 * q_i, forward strided pass), [9] elementwise, [10] encode / decode.  enable(on) clears
 * what was collected; get synchronises and fills, per class, the summed kernel
 * time in ms, the launch count and the summed algorithmic HBM bytes (each
 * operand read once and each result written once) into caller arrays of
 * hetal_timing_classes() entries. */
int hetal_timing_classes(void);
int hetal_timing_enable(hetal_ctx* ctx, int on);
int hetal_timing_get(hetal_ctx* ctx, double* ms, int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif

#endif /* HETAL_H */
