/*
 * CPU oracle for RNS-CKKS: the integer and double-double core.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant generator with the GPU library.
 *
 * Every routine is written for obviousness, not speed: modular products go
 * through unsigned __int128 and '%', the NTT is the textbook iterative radix-2
 * transform, and the encoder evaluates the inverse canonical embedding with a
 * plain radix-2 FFT in double-double arithmetic.
 *
 * What is computed follows the CKKS operations listed in Sec. 2.2 of the
 * HETAL paper (Add, Mult, CMult, Rotate, Conjugate, leveled rescaling) on the
 * RNS variant of CKKS that the paper's library implements (Sec. 5.1).  The RNS
 * building blocks (NTT, fast basis conversion, hybrid key switching) are the
 * textbook constructions, which the paper does not restate; the exact
 * definition each routine implements is written next to it.
 *
 * Parity status: every exported function is pinned by tests under tests/
 * (schoolbook products, transform round trips, direct-definition encodings,
 * decryption identities).  No function here is "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* Modular arithmetic: the definitions, nothing clever.                */
/* ------------------------------------------------------------------ */

/* Operands of addmod/submod are reduced (< q); mulmod accepts any 64-bit operands. */
static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static u64 submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

static u64 powmod(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

/* Inverse modulo a prime, by Fermat's little theorem. */
static u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); }

u64 orc_powmod(u64 a, u64 e, u64 q) { return powmod(a, e, q); }
u64 orc_mulmod(u64 a, u64 b, u64 q) { return mulmod(a, b, q); }
u64 orc_invmod(u64 a, u64 q) { return invmod(a, q); }

/* Deterministic Miller-Rabin for n < 2^64 (the first 12 primes as bases). */
int orc_is_prime(u64 n) {
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; ++i) {
        if (n == bases[i]) return 1;
        if (n % bases[i] == 0) return 0;
    }
    u64 d = n - 1;
    int r = 0;
    while ((d & 1) == 0) { d >>= 1; ++r; }
    for (int i = 0; i < 12; ++i) {
        u64 x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int composite = 1;
        for (int k = 1; k < r; ++k) {
            x = mulmod(x, x, n);
            if (x == n - 1) { composite = 0; break; }
        }
        if (composite) return 0;
    }
    return 1;
}

/*
 * The `count` largest primes p < bound with p == 1 (mod m), in descending
 * order.  Returns how many were found.
 */
int orc_primes_below(u64 bound, u64 m, int count, u64* out) {
    if (bound <= 1) return 0;
    u64 p = ((bound - 1) / m) * m + 1; /* largest value == 1 mod m that is <= bound */
    if (p >= bound) p -= m;
    int found = 0;
    while (found < count && p > m) {
        if (orc_is_prime(p)) out[found++] = p;
        p -= m;
    }
    return found;
}

/*
 * A primitive 2N-th root of unity modulo q (q prime, q == 1 mod 2N).
 * Take the smallest x >= 2 whose power x^((q-1)/2N) has order exactly 2N,
 * i.e. whose N-th power is -1.
 */
u64 orc_root_of_unity(u64 q, int log_n) {
    u64 m = 2ull << log_n;
    for (u64 x = 2; x < q; ++x) {
        u64 psi = powmod(x, (q - 1) / m, q);
        if (powmod(psi, m / 2, q) == q - 1) return psi;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Negacyclic NTT: a_hat[k] = a(psi^(2k+1)), k in natural order.        */
/* ------------------------------------------------------------------ */

static void bit_reverse_permute(u64* a, int log_n) {
    u64 n = 1ull << log_n;
    for (u64 i = 0; i < n; ++i) {
        u64 j = 0;
        for (int b = 0; b < log_n; ++b) j |= ((i >> b) & 1ull) << (log_n - 1 - b);
        if (i < j) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
}

/* Cyclic DFT over Z_q with primitive N-th root w: A[k] = sum_j a[j] w^(jk). */
static void cyclic_dft(u64* a, int log_n, u64 q, u64 w) {
    u64 n = 1ull << log_n;
    bit_reverse_permute(a, log_n);
    for (u64 len = 2; len <= n; len <<= 1) {
        u64 wlen = powmod(w, n / len, q);
        for (u64 i = 0; i < n; i += len) {
            u64 wj = 1;
            for (u64 j = 0; j < len / 2; ++j) {
                u64 u = a[i + j];
                u64 v = mulmod(a[i + j + len / 2], wj, q);
                a[i + j] = addmod(u, v, q);
                a[i + j + len / 2] = submod(u, v, q);
                wj = mulmod(wj, wlen, q);
            }
        }
    }
}

/* Forward: twist by psi^j, then cyclic DFT with w = psi^2. */
void orc_ntt(u64* a, int log_n, u64 q) {
    u64 n = 1ull << log_n;
    u64 psi = orc_root_of_unity(q, log_n);
    u64 pj = 1;
    for (u64 j = 0; j < n; ++j) { a[j] = mulmod(a[j], pj, q); pj = mulmod(pj, psi, q); }
    cyclic_dft(a, log_n, q, mulmod(psi, psi, q));
}

/* Inverse: cyclic DFT with w^-1, times N^-1, then untwist by psi^-j. */
void orc_intt(u64* a, int log_n, u64 q) {
    u64 n = 1ull << log_n;
    u64 psi = orc_root_of_unity(q, log_n);
    u64 psi_inv = invmod(psi, q);
    cyclic_dft(a, log_n, q, mulmod(psi_inv, psi_inv, q));
    u64 n_inv = invmod(n % q, q);
    u64 pj = n_inv;
    for (u64 j = 0; j < n; ++j) { a[j] = mulmod(a[j], pj, q); pj = mulmod(pj, psi_inv, q); }
}

/* Batched transforms over `count` polynomials, polynomial i modulo qs[i]. */
void orc_ntt_batch(u64* a, int count, int log_n, const u64* qs) {
    u64 n = 1ull << log_n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < count; ++i) orc_ntt(a + (u64)i * n, log_n, qs[i]);
}

void orc_intt_batch(u64* a, int count, int log_n, const u64* qs) {
    u64 n = 1ull << log_n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < count; ++i) orc_intt(a + (u64)i * n, log_n, qs[i]);
}

/*
 * Negacyclic product in Z_q[X]/(X^N+1), through the NTT:
 * out = iNTT(NTT(a) * NTT(b)).  `out` may alias `a` or `b`.
 */
void orc_polymul(const u64* a, const u64* b, u64* out, int log_n, u64 q) {
    u64 n = 1ull << log_n;
    u64* ta = (u64*)malloc(n * sizeof(u64));
    u64* tb = (u64*)malloc(n * sizeof(u64));
    memcpy(ta, a, n * sizeof(u64));
    memcpy(tb, b, n * sizeof(u64));
    orc_ntt(ta, log_n, q);
    orc_ntt(tb, log_n, q);
    for (u64 i = 0; i < n; ++i) ta[i] = mulmod(ta[i], tb[i], q);
    orc_intt(ta, log_n, q);
    memcpy(out, ta, n * sizeof(u64));
    free(ta);
    free(tb);
}

/* Limb-wise negacyclic products: out[i] = a[i] * b[i] mod (X^N+1, qs[i]). */
void orc_polymul_limbs(const u64* a, const u64* b, u64* out, int count, int log_n, const u64* qs) {
    u64 n = 1ull << log_n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < count; ++i) orc_polymul(a + (u64)i * n, b + (u64)i * n, out + (u64)i * n, log_n, qs[i]);
}

/* Schoolbook negacyclic product, O(N^2); used by the tests as a second witness. */
void orc_polymul_schoolbook(const u64* a, const u64* b, u64* out, int log_n, u64 q) {
    u64 n = 1ull << log_n;
    u64* acc = (u64*)calloc(n, sizeof(u64));
    for (u64 i = 0; i < n; ++i)
        for (u64 j = 0; j < n; ++j) {
            u64 p = mulmod(a[i], b[j], q);
            u64 k = i + j;
            if (k < n) acc[k] = addmod(acc[k], p, q);
            else acc[k - n] = submod(acc[k - n], p, q); /* X^N = -1 */
        }
    memcpy(out, acc, n * sizeof(u64));
    free(acc);
}

/* Pointwise products: out[i][k] = a[i][k] * b[i][k] mod qs[i]. */
void orc_mul_limbs(const u64* a, const u64* b, u64* out, int count, int log_n, const u64* qs) {
    u64 n = 1ull << log_n;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < count; ++i)
        for (u64 k = 0; k < n; ++k) out[(u64)i * n + k] = mulmod(a[(u64)i * n + k], b[(u64)i * n + k], qs[i]);
}

/* out[i][k] = a[i][k] * s[i] mod qs[i]. */
void orc_mul_scalar_limbs(const u64* a, const u64* s, u64* out, int count, int log_n, const u64* qs) {
    u64 n = 1ull << log_n;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < count; ++i)
        for (u64 k = 0; k < n; ++k) out[(u64)i * n + k] = mulmod(a[(u64)i * n + k], s[i], qs[i]);
}

/* ------------------------------------------------------------------ */
/* Galois automorphism tau_g: a(X) -> a(X^g), g odd, coefficient form. */
/* X^(g*j) = X^(g*j mod 2N), and X^(N + r) = -X^r.                      */
/* ------------------------------------------------------------------ */

void orc_automorphism(const u64* a, u64* out, int log_n, u64 q, u64 g) {
    u64 n = 1ull << log_n, m = 2 * n;
    for (u64 j = 0; j < n; ++j) {
        u64 e = (u64)(((u128)g * j) % m);
        if (e < n) out[e] = a[j];
        else out[e - n] = submod(0, a[j], q);
    }
}

void orc_automorphism_limbs(const u64* a, u64* out, int count, int log_n, const u64* qs, u64 g) {
    u64 n = 1ull << log_n;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < count; ++i) orc_automorphism(a + (u64)i * n, out + (u64)i * n, log_n, qs[i], g);
}

/* ------------------------------------------------------------------ */
/* Fast basis conversion (the approximate CRT lift used by ModUp and   */
/* ModDown):  for x given by residues x_i modulo the source primes d_i, */
/* D = prod d_i, each target t receives                                 */
/*     sum_i [x_i * (D/d_i)^-1]_{d_i} * (D/d_i)  mod t,                 */
/* with no correction of the overflow multiple of D.                    */
/* ------------------------------------------------------------------ */

void orc_basis_convert(const u64* x, const u64* src, int ns, const u64* dst, int nd, u64* out, int log_n) {
    u64 n = 1ull << log_n;
    u64* dhat_inv = (u64*)malloc(ns * sizeof(u64));   /* (D/d_i)^-1 mod d_i   */
    u64* dhat_t = (u64*)malloc((size_t)ns * nd * sizeof(u64)); /* (D/d_i) mod t */
    for (int i = 0; i < ns; ++i) {
        u64 prod = 1;
        for (int k = 0; k < ns; ++k)
            if (k != i) prod = mulmod(prod, src[k] % src[i], src[i]);
        dhat_inv[i] = invmod(prod, src[i]);
        for (int t = 0; t < nd; ++t) {
            u64 pt = 1;
            for (int k = 0; k < ns; ++k)
                if (k != i) pt = mulmod(pt, src[k] % dst[t], dst[t]);
            dhat_t[(size_t)i * nd + t] = pt;
        }
    }
#pragma omp parallel for schedule(static)
    for (u64 k = 0; k < n; ++k) {
        for (int t = 0; t < nd; ++t) {
            u64 acc = 0;
            for (int i = 0; i < ns; ++i) {
                u64 y = mulmod(x[(u64)i * n + k], dhat_inv[i], src[i]);
                acc = addmod(acc, mulmod(y, dhat_t[(size_t)i * nd + t], dst[t]), dst[t]);
            }
            out[(u64)t * n + k] = acc;
        }
    }
    free(dhat_inv);
    free(dhat_t);
}

/*
 * Centred fast basis conversion, used by ModDown: as above, but each
 * y_i = [x_i * (D/d_i)^-1]_{d_i} is taken in (-d_i/2, d_i/2].  The lift
 * sum_i y_i (D/d_i) then equals the centred residue of x modulo D plus v*D with
 * v symmetric about 0, so dividing by D afterwards rounds instead of flooring
 * and leaves a zero-mean error.
 */
void orc_basis_convert_centered(const u64* x, const u64* src, int ns, const u64* dst, int nd, u64* out, int log_n) {
    u64 n = 1ull << log_n;
    u64* dhat_inv = (u64*)malloc(ns * sizeof(u64));
    u64* dhat_t = (u64*)malloc((size_t)ns * nd * sizeof(u64));
    for (int i = 0; i < ns; ++i) {
        u64 prod = 1;
        for (int k = 0; k < ns; ++k)
            if (k != i) prod = mulmod(prod, src[k] % src[i], src[i]);
        dhat_inv[i] = invmod(prod, src[i]);
        for (int t = 0; t < nd; ++t) {
            u64 pt = 1;
            for (int k = 0; k < ns; ++k)
                if (k != i) pt = mulmod(pt, src[k] % dst[t], dst[t]);
            dhat_t[(size_t)i * nd + t] = pt;
        }
    }
#pragma omp parallel for schedule(static)
    for (u64 k = 0; k < n; ++k) {
        for (int t = 0; t < nd; ++t) {
            u64 acc = 0;
            for (int i = 0; i < ns; ++i) {
                u64 y = mulmod(x[(u64)i * n + k], dhat_inv[i], src[i]);
                u64 w = dhat_t[(size_t)i * nd + t];
                if (y > src[i] / 2) /* y - d_i < 0: subtract (d_i - y) * (D/d_i) */
                    acc = submod(acc, mulmod(src[i] - y, w, dst[t]), dst[t]);
                else
                    acc = addmod(acc, mulmod(y, w, dst[t]), dst[t]);
            }
            out[(u64)t * n + k] = acc;
        }
    }
    free(dhat_inv);
    free(dhat_t);
}

/* ------------------------------------------------------------------ */
/* Double-double arithmetic (Dekker / Knuth error-free transforms).    */
/* ------------------------------------------------------------------ */

typedef struct { double hi, lo; } dd;
typedef struct { dd re, im; } cdd;

static dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    dd r = {s, e};
    return r;
}
static dd quick_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    dd r = {s, e};
    return r;
}
static dd two_prod(double a, double b) {
    double p = a * b;
    double e = fma(a, b, -p);
    dd r = {p, e};
    return r;
}
static dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = quick_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return quick_two_sum(s.hi, s.lo);
}
static dd dd_neg(dd a) { dd r = {-a.hi, -a.lo}; return r; }
static dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
static dd dd_mul(dd a, dd b) {
    dd p = two_prod(a.hi, b.hi);
    p.lo += a.hi * b.lo + a.lo * b.hi;
    return quick_two_sum(p.hi, p.lo);
}
static dd dd_mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    p.lo += a.lo * b;
    return quick_two_sum(p.hi, p.lo);
}
static dd dd_div_d(dd a, double b) {
    double q1 = a.hi / b;
    dd p = two_prod(q1, b);
    dd r = dd_sub(a, p);
    double q2 = (r.hi + r.lo) / b;
    return quick_two_sum(q1, q2);
}
static dd dd_from(double x) { dd r = {x, 0.0}; return r; }

static cdd cdd_add(cdd a, cdd b) { cdd r = {dd_add(a.re, b.re), dd_add(a.im, b.im)}; return r; }
static cdd cdd_sub(cdd a, cdd b) { cdd r = {dd_sub(a.re, b.re), dd_sub(a.im, b.im)}; return r; }
static cdd cdd_mul(cdd a, cdd b) {
    cdd r = {dd_sub(dd_mul(a.re, b.re), dd_mul(a.im, b.im)), dd_add(dd_mul(a.re, b.im), dd_mul(a.im, b.re))};
    return r;
}

/* pi to double-double precision: the double nearest pi, plus the double nearest the remainder. */
static const double PI_HI = 3.141592653589793116e+00;
static const double PI_LO = 1.224646799147353207e-16;

void orc_dd_pi(double* out2) { out2[0] = PI_HI; out2[1] = PI_LO; }

/* cos and sin of x (|x| <= pi/2) by their Taylor series, summed until the terms vanish. */
static void dd_sincos_taylor(dd x, dd* c, dd* s) {
    dd x2 = dd_mul(x, x);
    dd term = x;             /* x^(2k+1)/(2k+1)! */
    dd sum_s = x;
    for (int k = 1; k < 60; ++k) {
        term = dd_mul(term, x2);
        term = dd_div_d(term, (double)(2 * k) * (double)(2 * k + 1));
        term = dd_neg(term);
        sum_s = dd_add(sum_s, term);
        if (fabs(term.hi) < 1e-40) break;
    }
    term = dd_from(1.0);     /* x^(2k)/(2k)! */
    dd sum_c = term;
    for (int k = 1; k < 60; ++k) {
        term = dd_mul(term, x2);
        term = dd_div_d(term, (double)(2 * k - 1) * (double)(2 * k));
        term = dd_neg(term);
        sum_c = dd_add(sum_c, term);
        if (fabs(term.hi) < 1e-40) break;
    }
    *c = sum_c;
    *s = sum_s;
}

/*
 * exp(2 pi i j / m) for 0 <= j < m (m a power of two, m >= 4): reduce to the
 * first quadrant (multiplying by i^quadrant is exact) and use the series there.
 */
static cdd dd_root_of_unity(u64 j, u64 m) {
    u64 quarter = m / 4;
    u64 quad = j / quarter, r = j % quarter;
    dd angle = dd_mul_d(dd_div_d((dd){PI_HI, PI_LO}, (double)m), 2.0 * (double)r); /* 2 pi r / m */
    dd c, s;
    dd_sincos_taylor(angle, &c, &s);
    cdd w = {c, s};
    for (u64 t = 0; t < quad; ++t) { cdd v = {dd_neg(w.im), w.re}; w = v; } /* times i */
    return w;
}

void orc_dd_root_of_unity(u64 j, u64 m, double* out4) {
    cdd w = dd_root_of_unity(j, m);
    out4[0] = w.re.hi; out4[1] = w.re.lo; out4[2] = w.im.hi; out4[3] = w.im.lo;
}

/* In-place radix-2 DFT of size m over double-double complex numbers:
 * A[k] = sum_j a[j] w^(sign * j k), w = exp(2 pi i / m). */
static void dd_dft(cdd* a, u64 m, const cdd* roots /* exp(2 pi i j / m), j < m */, int sign) {
    int log_m = 0;
    while ((1ull << log_m) < m) ++log_m;
    for (u64 i = 0; i < m; ++i) {
        u64 j = 0;
        for (int b = 0; b < log_m; ++b) j |= ((i >> b) & 1ull) << (log_m - 1 - b);
        if (i < j) { cdd t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (u64 len = 2; len <= m; len <<= 1) {
        u64 step = m / len;
        for (u64 i = 0; i < m; i += len) {
            for (u64 j = 0; j < len / 2; ++j) {
                u64 e = (j * step) % m;
                cdd w = roots[sign > 0 ? e : (m - e) % m];
                cdd u = a[i + j];
                cdd v = cdd_mul(a[i + j + len / 2], w);
                a[i + j] = cdd_add(u, v);
                a[i + j + len / 2] = cdd_sub(u, v);
            }
        }
    }
}

/*
 * Round a double-double value to an integer: round half to even, where any
 * value whose distance to the nearest half-integer is at most 2^-24 counts as
 * that half-integer.  Returns 0 on success, -1 if |v| >= 2^62.
 */
#define TIE_WINDOW 0x1p-24
static int round_dd(dd v, i64* out) {
    if (!(fabs(v.hi) < 0x1p62)) return -1;
    double fh = floor(v.hi);
    i64 f;
    double frac;
    if (fh == v.hi) {
        double fl = floor(v.lo);
        f = (i64)v.hi + (i64)fl;
        frac = v.lo - fl;
    } else {
        f = (i64)fh;
        frac = (v.hi - fh) + v.lo;
    }
    double d = frac - 0.5;
    if (fabs(d) <= TIE_WINDOW) *out = f + (f & 1);
    else *out = f + (d > 0.0 ? 1 : 0);
    return 0;
}

/*
 * CKKS encoding (canonical-embedding inverse).  Slot k (0 <= k < N/2) is the
 * value of the plaintext polynomial at zeta^(5^k), zeta = exp(i pi / N); its
 * conjugate sits at zeta^(-5^k).  The coefficients are
 *     m_j = (1/N) sum_{e odd} Z[e] zeta^(-e j),
 * with Z[5^k mod 2N] = z_k and Z[-5^k mod 2N] = conj(z_k), evaluated here as an
 * inverse DFT of size 2N in double-double, then scaled by `scale` and rounded
 * (round_dd).  Output: N signed coefficients.  Returns 0, or -1 if a
 * coefficient does not fit in 62 bits.
 */
int orc_encode(const double* re, const double* im, int log_n, double scale, i64* out) {
    u64 n = 1ull << log_n, m = 2 * n, slots = n / 2;
    cdd* roots = (cdd*)malloc(m * sizeof(cdd));
    cdd* z = (cdd*)calloc(m, sizeof(cdd));
    for (u64 j = 0; j < m; ++j) roots[j] = dd_root_of_unity(j, m);
    u64 e = 1;
    for (u64 k = 0; k < slots; ++k) {
        cdd v = {dd_from(re[k]), dd_from(im[k])};
        cdd vc = {dd_from(re[k]), dd_neg(dd_from(im[k]))};
        z[e] = v;
        z[m - e] = vc;
        e = (e * 5) % m;
    }
    dd_dft(z, m, roots, -1);
    int rc = 0;
    for (u64 j = 0; j < n; ++j) {
        dd v = dd_mul_d(dd_div_d(z[j].re, (double)n), scale);
        if (round_dd(v, &out[j]) != 0) rc = -1;
    }
    free(roots);
    free(z);
    return rc;
}

/* Reduce signed integer coefficients modulo each prime: out[i][k] = c[k] mod qs[i]. */
void orc_reduce_signed(const i64* c, u64* out, int count, int log_n, const u64* qs) {
    u64 n = 1ull << log_n;
    for (int i = 0; i < count; ++i)
        for (u64 k = 0; k < n; ++k) {
            i64 v = c[k];
            u64 mag = v < 0 ? (u64)(-v) : (u64)v;
            u64 r = mag % qs[i];
            out[(u64)i * n + k] = (v < 0 && r) ? qs[i] - r : r;
        }
}

/*
 * Centred value of a residue vector from its first two limbs (CRT modulo
 * q0*q1), returned as a double.  Used by decoding; exact while the true
 * integer lies in (-q0 q1 / 2, q0 q1 / 2).  With one limb, centres modulo q0.
 */
void orc_crt_centered(const u64* limbs, int count, int log_n, const u64* qs, double* out) {
    u64 n = 1ull << log_n;
    if (count == 1) {
        for (u64 k = 0; k < n; ++k) {
            u64 x = limbs[k];
            out[k] = x > qs[0] / 2 ? -(double)(qs[0] - x) : (double)x;
        }
        return;
    }
    u64 q0 = qs[0], q1 = qs[1];
    u64 q0_inv = invmod(q0 % q1, q1);
    u128 big = (u128)q0 * q1;
    for (u64 k = 0; k < n; ++k) {
        u64 x0 = limbs[k], x1 = limbs[n + k];
        u64 t = mulmod(submod(x1, x0 % q1, q1), q0_inv, q1);
        u128 x = (u128)x0 + (u128)q0 * t; /* in [0, q0 q1) */
        if (x > big / 2) out[k] = -(double)(big - x);
        else out[k] = (double)x;
    }
}

/* Thread count of the parallel loops above (timing only; results do not depend on it). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------ */
/* Seeded sampling: ChaCha20 as the counter-based generator.            */
/* ------------------------------------------------------------------ */

/*
 * The ChaCha20 block function of RFC 8439 (Sec. 2.1-2.3), written from its
 * definition: a 4x4 state of 32-bit words (the four constants, the 256-bit
 * key, a 32-bit block counter, a 96-bit nonce), twenty rounds that alternate
 * quarter rounds on the columns and on the diagonals, then the input state
 * added word by word.  out: the 16 words of the block (the keystream is their
 * little-endian bytes).
 */
static uint32_t rotl32(uint32_t v, int c) { return (v << c) | (v >> (32 - c)); }

static void quarter_round(uint32_t* x, int a, int b, int c, int d) {
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 16);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 12);
    x[a] += x[b]; x[d] ^= x[a]; x[d] = rotl32(x[d], 8);
    x[c] += x[d]; x[b] ^= x[c]; x[b] = rotl32(x[b], 7);
}

void orc_chacha20_quarter_round(uint32_t* x4) { quarter_round(x4, 0, 1, 2, 3); }

void orc_chacha20_block(const uint32_t* key8, uint32_t counter, const uint32_t* nonce3, uint32_t* out16) {
    uint32_t s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u};
    for (int i = 0; i < 8; ++i) s[4 + i] = key8[i];
    s[12] = counter;
    for (int i = 0; i < 3; ++i) s[13 + i] = nonce3[i];
    uint32_t x[16];
    memcpy(x, s, sizeof(x));
    for (int r = 0; r < 10; ++r) {
        quarter_round(x, 0, 4, 8, 12);
        quarter_round(x, 1, 5, 9, 13);
        quarter_round(x, 2, 6, 10, 14);
        quarter_round(x, 3, 7, 11, 15);
        quarter_round(x, 0, 5, 10, 15);
        quarter_round(x, 1, 6, 11, 12);
        quarter_round(x, 2, 7, 8, 13);
        quarter_round(x, 3, 4, 9, 14);
    }
    for (int i = 0; i < 16; ++i) out16[i] = x[i] + s[i];
}

/*
 * The stream of (seed, purpose, index, sub): ChaCha20 with the key = the
 * 64-bit seed (low word first) followed by zeros, the nonce = (purpose, index,
 * sub), and the block counter = the block number.  Its 64-bit word p is bytes
 * 8 (p mod 8) .. 8 (p mod 8) + 7 of block floor(p / 8), little-endian.
 */
static u64 stream_word(u64 seed, uint32_t purpose, uint32_t index, uint32_t sub, u64 p) {
    uint32_t key[8] = {(uint32_t)seed, (uint32_t)(seed >> 32), 0, 0, 0, 0, 0, 0};
    uint32_t nonce[3] = {purpose, index, sub};
    uint32_t blk[16];
    orc_chacha20_block(key, (uint32_t)(p / 8), nonce, blk);
    int w = (int)(p % 8);
    return (u64)blk[2 * w] | ((u64)blk[2 * w + 1] << 32);
}

/* Words p0 .. p0 + count - 1 of a stream. */
void orc_stream_words(u64 seed, uint32_t purpose, uint32_t index, uint32_t sub, u64 p0, u64 count, u64* out) {
    for (u64 i = 0; i < count; ++i) out[i] = stream_word(seed, purpose, index, sub, p0 + i);
}

/*
 * Uniform residues modulo q, one per coefficient k < N: the first of the words
 * k, N + k, 2N + k, ... of the stream that lies below floor(2^64 / q) q (a
 * rejected word would bias the result), reduced modulo q.
 */
void orc_sample_uniform(u64 seed, uint32_t purpose, uint32_t index, uint32_t sub, u64 q, int log_n, u64* out) {
    u64 n = 1ull << log_n;
    u64 bound = (UINT64_MAX / q) * q; /* floor(2^64 / q) q, as 2^64 - (2^64 mod q) */
    if (UINT64_MAX % q == q - 1) bound = 0; /* q divides 2^64: no word is rejected */
    for (u64 k = 0; k < n; ++k) {
        for (u64 layer = 0;; ++layer) {
            u64 w = stream_word(seed, purpose, index, sub, layer * n + k);
            if (bound == 0 || w < bound) {
                out[k] = w % q;
                break;
            }
        }
    }
}

/*
 * Rounded Gaussian errors from a cumulative table: word k of the stream gives
 * coefficient k; its top bit is the sign and its low 63 bits u select the
 * magnitude, the number of thresholds table[j] <= u (table ascending, `entries`
 * of them); magnitude 0 ignores the sign.
 */
void orc_sample_gaussian(u64 seed, uint32_t purpose, uint32_t index, uint32_t sub, const u64* table, int entries,
                         int log_n, i64* out) {
    u64 n = 1ull << log_n;
    for (u64 k = 0; k < n; ++k) {
        u64 w = stream_word(seed, purpose, index, sub, k);
        u64 u = w & 0x7fffffffffffffffull;
        i64 mag = 0;
        for (int j = 0; j < entries; ++j) mag += table[j] <= u;
        out[k] = (w >> 63) ? -mag : mag;
    }
}

/*
 * A ternary secret with exactly h nonzero coefficients: the words of the
 * stream are taken in order; word w names position w mod N (N a power of two)
 * and sign (w >> 63 ? -1 : +1); a position already taken is skipped, until h
 * positions are set.  Returns the number of words used, or -1 if h > N.
 */
i64 orc_sample_ternary(u64 seed, uint32_t purpose, uint32_t index, uint32_t sub, int h, int log_n, i64* out) {
    u64 n = 1ull << log_n;
    if ((u64)h > n) return -1;
    memset(out, 0, n * sizeof(i64));
    u64 p = 0;
    for (int set = 0; set < h; ++p) {
        u64 w = stream_word(seed, purpose, index, sub, p);
        u64 pos = w & (n - 1);
        if (out[pos] != 0) continue;
        out[pos] = (w >> 63) ? -1 : 1;
        ++set;
    }
    return (i64)p;
}
