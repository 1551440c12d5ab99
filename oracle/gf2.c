/*
 * GF(2) toolkit that pins the xorgens oracle to the mathematics.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as xorgens_oracle.c: loaded by the
 * tests, the smoke check and the CPU-baseline leg only; shares nothing with
 * the HIP path).
 *
 * The xorgens x-part is GF(2)-linear (Section 1.5 / Section 2 of the paper):
 * its n = r w bit state evolves by a fixed n x n matrix T.  The paper's period
 * claim (2^4096 - 1) for the x-part, times 2^32 for the Weyl part (Section 1.5,
 * Table 1), holds exactly when the characteristic polynomial of T is primitive.
 * This file provides, in plain form:
 *   - Berlekamp-Massey: minimal polynomial of a bit sequence;
 *   - polynomial arithmetic mod P (schoolbook carry-less products with an
 *     exact Barrett reduction, which needs no correction over GF(2));
 *   - the irreducibility / primitivity test from the factorisation of 2^n - 1
 *     supplied by the caller;
 *   - jump-ahead by z^J mod P (polynomial form) and by T^J (matrix form).
 *
 * Polynomials are little-endian bit arrays in 64-bit words: bit i of the
 * array is the coefficient of z^i.
 */
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#if defined(__PCLMUL__) && defined(__SSE4_1__)
#include <wmmintrin.h>
#include <smmintrin.h>
#endif

#define PW 132 /* words of a product of two polynomials of degree <= 4096 */

/* ---- carry-less 64 x 64 -> 128 multiply ---------------------------------- */

/* Definition: XOR of b shifted left by every set bit position of a. */
void gf2_clmul64_portable(uint64_t a, uint64_t b, uint64_t *lo, uint64_t *hi)
{
    uint64_t l = 0, h = 0;
    int i;
    for (i = 0; i < 64; i++) {
        if ((a >> i) & 1u) {
            l ^= b << i;
            if (i) h ^= b >> (64 - i);
        }
    }
    *lo = l;
    *hi = h;
}

/* The same product through the CPU's carry-less multiply instruction when
   the build enables it (checked against the portable form by the tests). */
void gf2_clmul64(uint64_t a, uint64_t b, uint64_t *lo, uint64_t *hi)
{
#if defined(__PCLMUL__) && defined(__SSE4_1__)
    __m128i r = _mm_clmulepi64_si128(_mm_set_epi64x(0, (long long)a),
                                     _mm_set_epi64x(0, (long long)b), 0x00);
    *lo = (uint64_t)_mm_cvtsi128_si64(r);
    *hi = (uint64_t)_mm_extract_epi64(r, 1);
#else
    gf2_clmul64_portable(a, b, lo, hi);
#endif
}

/* ---- small helpers ------------------------------------------------------- */

static int nwords(int deg) { return deg / 64 + 1; }

static int getbit(const uint64_t *a, int i) { return (int)((a[i >> 6] >> (i & 63)) & 1u); }

static void setbit(uint64_t *a, int i) { a[i >> 6] |= 1ull << (i & 63); }

int gf2_degree(const uint64_t *a, int words)
{
    int w;
    for (w = words - 1; w >= 0; w--)
        if (a[w]) return w * 64 + 63 - __builtin_clzll(a[w]);
    return -1;
}

/* out = a * b; a has wa words, b has wb words, out has wa + wb words. */
static void polmul(const uint64_t *a, int wa, const uint64_t *b, int wb, uint64_t *out)
{
    int i, j;
    memset(out, 0, (size_t)(wa + wb) * sizeof(uint64_t));
    for (i = 0; i < wa; i++) {
        if (!a[i]) continue;
        for (j = 0; j < wb; j++) {
            uint64_t lo, hi;
            gf2_clmul64(a[i], b[j], &lo, &hi);
            out[i + j] ^= lo;
            out[i + j + 1] ^= hi;
        }
    }
}

/* out[0 .. ow) = a >> sh (bit shift), a has wa words. */
static void shr_bits(const uint64_t *a, int wa, int sh, uint64_t *out, int ow)
{
    int q = sh / 64, r = sh % 64, i;
    for (i = 0; i < ow; i++) {
        uint64_t lo = (i + q < wa) ? a[i + q] : 0;
        uint64_t hi = (i + q + 1 < wa) ? a[i + q + 1] : 0;
        out[i] = r ? (lo >> r) | (hi << (64 - r)) : lo;
    }
}

/* ---- reduction modulo a monic P of degree n ------------------------------ */

typedef struct {
    int n, w;          /* degree, words of a residue (deg < n) */
    uint64_t P[PW];    /* the modulus */
    uint64_t mu[PW];   /* floor(z^{2n} / P), degree n */
} modctx;

/* Plain long division of z^{2n} by P gives mu. */
static void modctx_init(modctx *m, const uint64_t *P, int n)
{
    uint64_t rem[2 * PW];
    int i, j, pw = nwords(n);
    memset(m, 0, sizeof(*m));
    m->n = n;
    m->w = nwords(n - 1);
    memcpy(m->P, P, (size_t)pw * sizeof(uint64_t));
    memset(rem, 0, sizeof(rem));
    setbit(rem, 2 * n);
    for (i = 2 * n; i >= n; i--) {
        if (!getbit(rem, i)) continue;
        setbit(m->mu, i - n);
        /* rem ^= P << (i - n) */
        for (j = 0; j <= n; j++)
            if (getbit(P, j)) rem[(j + i - n) >> 6] ^= 1ull << ((j + i - n) & 63);
    }
}

/* r = R mod P for deg R < 2n (Barrett: q = floor(floor(R / z^n) mu / z^n)). */
static void reduce(const modctx *m, const uint64_t *R, int wr, uint64_t *r)
{
    uint64_t R1[PW], t[2 * PW], q[PW], qP[2 * PW];
    int w1 = nwords(m->n), i;
    int wp = nwords(m->n);
    shr_bits(R, wr, m->n, R1, w1);
    polmul(R1, w1, m->mu, w1, t);
    shr_bits(t, 2 * w1, m->n, q, w1);
    polmul(q, w1, m->P, wp, qP);
    for (i = 0; i < m->w; i++) r[i] = (i < wr ? R[i] : 0) ^ qP[i];
}

static void mulmod(const modctx *m, const uint64_t *a, const uint64_t *b, uint64_t *out)
{
    uint64_t prod[2 * PW];
    polmul(a, m->w, b, m->w, prod);
    reduce(m, prod, 2 * m->w, out);
}

/* Exposed for the tests: out = a * b mod P. */
int gf2_mulmod(const uint64_t *P, int n, const uint64_t *a, const uint64_t *b, uint64_t *out)
{
    modctx *m;
    if (n < 2 || n > 4096 || gf2_degree(P, nwords(n)) != n) return -1;
    m = (modctx *)malloc(sizeof(modctx));
    if (!m) return -2;
    modctx_init(m, P, n);
    mulmod(m, a, b, out);
    free(m);
    return 0;
}

/* ---- gcd ------------------------------------------------------------------ */

/* a = a mod b in place (plain long division), both with `words` words. */
static void polmod_inplace(uint64_t *a, const uint64_t *b, int words)
{
    int db = gf2_degree(b, words), da, j;
    while ((da = gf2_degree(a, words)) >= db) {
        int sh = da - db;
        for (j = 0; j <= db; j++)
            if (getbit(b, j)) a[(j + sh) >> 6] ^= 1ull << ((j + sh) & 63);
    }
}

/* Degree of gcd(a, b) by Euclid's algorithm; a, b are copied. */
int gf2_gcd_degree(const uint64_t *a_in, const uint64_t *b_in, int words)
{
    uint64_t *a = (uint64_t *)calloc((size_t)words, sizeof(uint64_t));
    uint64_t *b = (uint64_t *)calloc((size_t)words, sizeof(uint64_t));
    uint64_t *t;
    int d;
    memcpy(a, a_in, (size_t)words * sizeof(uint64_t));
    memcpy(b, b_in, (size_t)words * sizeof(uint64_t));
    while (gf2_degree(b, words) >= 0) {
        polmod_inplace(a, b, words);
        t = a; a = b; b = t;
    }
    d = gf2_degree(a, words);
    free(a);
    free(b);
    return d;
}

/* ---- Berlekamp-Massey ------------------------------------------------------ */

/* Shortest LFSR generating bits[0 .. N).  Returns its length L and writes the
   characteristic polynomial P(z) = z^L + c_1 z^{L-1} + ... + c_L (so that
   s_{k} = c_1 s_{k-1} + ... + c_L s_{k-L}) into `poly` (zeroed, `words` words). */
int gf2_berlekamp_massey(const uint8_t *bits, int N, uint64_t *poly, int words)
{
    uint8_t *C = (uint8_t *)calloc((size_t)N + 2, 1);
    uint8_t *B = (uint8_t *)calloc((size_t)N + 2, 1);
    uint8_t *T = (uint8_t *)calloc((size_t)N + 2, 1);
    int L = 0, m = 1, k, i;
    C[0] = 1;
    B[0] = 1;
    for (k = 0; k < N; k++) {
        int d = bits[k] & 1;
        for (i = 1; i <= L; i++) d ^= C[i] & bits[k - i];
        if (!d) { m++; continue; }
        if (2 * L <= k) {
            memcpy(T, C, (size_t)N + 2);
            for (i = 0; i + m <= N + 1; i++) C[i + m] ^= B[i];
            L = k + 1 - L;
            memcpy(B, T, (size_t)N + 2);
            m = 1;
        } else {
            for (i = 0; i + m <= N + 1; i++) C[i + m] ^= B[i];
            m++;
        }
    }
    memset(poly, 0, (size_t)words * sizeof(uint64_t));
    if (L / 64 < words) {
        for (i = 0; i <= L; i++)
            if (C[i]) setbit(poly, L - i);
    }
    free(C); free(B); free(T);
    return L;
}

/* ---- primitivity ---------------------------------------------------------- */

/* Tests a monic P of degree n (2 <= n <= 4096) for primitivity over GF(2).
   The caller supplies
     - sub_exps[0 .. nsub): the values n / p for every prime p dividing n;
     - exps: nq exponents (2^n - 1) / q for every prime q dividing 2^n - 1, each
       as an n-bit little-endian bit array of exp_words words.
   Return: 0 primitive; 1 z^{2^n} != z (not irreducible, or not square-free);
   2 a gcd with z^{2^{n/p}} - z is non-trivial (not irreducible);
   3 + i   z^{(2^n-1)/q_i} == 1 (irreducible, order not 2^n - 1);
   < 0 bad arguments. */
int gf2_is_primitive(const uint64_t *P, int n, const int *sub_exps, int nsub,
                     const uint64_t *exps, int nq, int exp_words)
{
    modctx *m;
    uint64_t *frob, *acc, *tmp, *g;
    int i, k, w, words, rc = 0;
    if (n < 2 || n > 4096 || gf2_degree(P, nwords(n)) != n) return -1;
    if (!getbit(P, 0)) return 1; /* z divides P */
    m = (modctx *)malloc(sizeof(modctx));
    modctx_init(m, P, n);
    w = m->w;
    words = nwords(n);
    /* frob[i] = z^{2^i} mod P, i = 0 .. n */
    frob = (uint64_t *)calloc((size_t)(n + 1) * (size_t)w, sizeof(uint64_t));
    acc = (uint64_t *)calloc((size_t)w, sizeof(uint64_t));
    tmp = (uint64_t *)calloc((size_t)w, sizeof(uint64_t));
    g = (uint64_t *)calloc((size_t)words + 1, sizeof(uint64_t));
    frob[0] = 2; /* z */
    for (i = 1; i <= n; i++) mulmod(m, frob + (size_t)(i - 1) * w, frob + (size_t)(i - 1) * w, frob + (size_t)i * w);
    /* z^{2^n} == z ? */
    if (memcmp(frob + (size_t)n * w, frob, (size_t)w * sizeof(uint64_t)) != 0) { rc = 1; goto done; }
    /* gcd(z^{2^{n/p}} - z, P) == 1 for each prime p | n */
    for (k = 0; k < nsub; k++) {
        int e = sub_exps[k];
        if (e < 0 || e > n) { rc = -1; goto done; }
        memset(g, 0, ((size_t)words + 1) * sizeof(uint64_t));
        memcpy(g, frob + (size_t)e * w, (size_t)w * sizeof(uint64_t));
        g[0] ^= 2; /* - z */
        if (gf2_degree(g, words) < 0) { rc = 2; goto done; }
        if (gf2_gcd_degree(g, P, words) != 0) { rc = 2; goto done; }
    }
    /* z^{(2^n-1)/q} != 1 for each prime q | 2^n - 1 */
    for (k = 0; k < nq; k++) {
        const uint64_t *e = exps + (size_t)k * exp_words;
        memset(acc, 0, (size_t)w * sizeof(uint64_t));
        acc[0] = 1;
        for (i = 0; i < n && i < exp_words * 64; i++) {
            if (!getbit(e, i)) continue;
            mulmod(m, acc, frob + (size_t)i * w, tmp);
            memcpy(acc, tmp, (size_t)w * sizeof(uint64_t));
        }
        {
            int one = (acc[0] == 1);
            for (i = 1; i < w; i++) one &= (acc[i] == 0);
            if (one) { rc = 3 + k; goto done; }
        }
    }
done:
    free(frob); free(acc); free(tmp); free(g); free(m);
    return rc;
}

/* ---- jump-ahead, polynomial form ------------------------------------------ */

/* g = z^J mod P by square-and-multiply, J given as a little-endian bit array
   of jbits bits.  g has nwords(n - 1) words. */
int gf2_z_pow_mod(const uint64_t *P, int n, const uint8_t *jbits, int nbits, uint64_t *g)
{
    modctx *m;
    uint64_t base[PW], acc[PW], tmp[PW];
    int i, w;
    if (n < 2 || n > 4096 || gf2_degree(P, nwords(n)) != n) return -1;
    m = (modctx *)malloc(sizeof(modctx));
    modctx_init(m, P, n);
    w = m->w;
    memset(base, 0, sizeof(base));
    memset(acc, 0, sizeof(acc));
    base[0] = 2;
    acc[0] = 1;
    for (i = 0; i < nbits; i++) {
        if (jbits[i]) {
            mulmod(m, acc, base, tmp);
            memcpy(acc, tmp, (size_t)w * sizeof(uint64_t));
        }
        mulmod(m, base, base, tmp);
        memcpy(base, tmp, (size_t)w * sizeof(uint64_t));
    }
    memcpy(g, acc, (size_t)w * sizeof(uint64_t));
    free(m);
    return 0;
}

/* ---- jump-ahead, matrix form ---------------------------------------------- */

/* Square bit matrices of order n stored row-major, rw = nwords(n - 1) words per
   row; bit j of row i is entry (i, j).  C = A B: row i of C is the XOR of the
   rows k of B with A(i, k) = 1. */
static void matmul(const uint64_t *A, const uint64_t *B, uint64_t *C, int n, int rw)
{
    int i, k, j;
    memset(C, 0, (size_t)n * (size_t)rw * sizeof(uint64_t));
    for (i = 0; i < n; i++) {
        uint64_t *ci = C + (size_t)i * rw;
        const uint64_t *ai = A + (size_t)i * rw;
        for (k = 0; k < n; k++) {
            if (!((ai[k >> 6] >> (k & 63)) & 1u)) continue;
            {
                const uint64_t *bk = B + (size_t)k * rw;
                for (j = 0; j < rw; j++) ci[j] ^= bk[j];
            }
        }
    }
}

/* v <- M^J v for a column bit vector v of n bits (rw words), by binary
   powering of M.  J is a little-endian bit array of nbits bits. */
int gf2_mat_pow_apply(const uint64_t *M, int n, const uint8_t *jbits, int nbits, uint64_t *v)
{
    int rw = nwords(n - 1), i, k, b;
    size_t msz = (size_t)n * (size_t)rw;
    uint64_t *Mp = (uint64_t *)malloc(msz * sizeof(uint64_t));
    uint64_t *T = (uint64_t *)malloc(msz * sizeof(uint64_t));
    uint64_t *nv = (uint64_t *)calloc((size_t)rw, sizeof(uint64_t));
    if (!Mp || !T || !nv) { free(Mp); free(T); free(nv); return -2; }
    memcpy(Mp, M, msz * sizeof(uint64_t));
    for (b = 0; b < nbits; b++) {
        if (jbits[b]) {
            /* v <- Mp v: bit i of the result is the parity of row i AND v */
            memset(nv, 0, (size_t)rw * sizeof(uint64_t));
            for (i = 0; i < n; i++) {
                uint64_t acc = 0;
                for (k = 0; k < rw; k++) acc ^= Mp[(size_t)i * rw + k] & v[k];
                if (__builtin_parityll(acc)) nv[i >> 6] |= 1ull << (i & 63);
            }
            memcpy(v, nv, (size_t)rw * sizeof(uint64_t));
        }
        if (b + 1 < nbits) {
            matmul(Mp, Mp, T, n, rw);
            memcpy(Mp, T, msz * sizeof(uint64_t));
        }
    }
    free(Mp); free(T); free(nv);
    return 0;
}

/* v_j <- M^(J_j) v_j for k column vectors at once: the binary powers M^(2^b)
   are formed once and applied to every v_j whose exponent has bit b set.
   jbits holds k little-endian bit arrays of nbits bits each (row j for J_j);
   vs holds the k vectors, rw = nwords(n - 1) words each. */
int gf2_mat_pow_apply_many(const uint64_t *M, int n, const uint8_t *jbits, int nbits, int k, uint64_t *vs)
{
    int rw = nwords(n - 1), i, q, b, j;
    size_t msz = (size_t)n * (size_t)rw;
    uint64_t *Mp = (uint64_t *)malloc(msz * sizeof(uint64_t));
    uint64_t *T = (uint64_t *)malloc(msz * sizeof(uint64_t));
    uint64_t *nv = (uint64_t *)calloc((size_t)rw, sizeof(uint64_t));
    if (!Mp || !T || !nv) { free(Mp); free(T); free(nv); return -2; }
    memcpy(Mp, M, msz * sizeof(uint64_t));
    for (b = 0; b < nbits; b++) {
        for (j = 0; j < k; j++) {
            uint64_t *v = vs + (size_t)j * rw;
            if (!jbits[(size_t)j * nbits + b]) continue;
            memset(nv, 0, (size_t)rw * sizeof(uint64_t));
            for (i = 0; i < n; i++) {
                uint64_t acc = 0;
                for (q = 0; q < rw; q++) acc ^= Mp[(size_t)i * rw + q] & v[q];
                if (__builtin_parityll(acc)) nv[i >> 6] |= 1ull << (i & 63);
            }
            memcpy(v, nv, (size_t)rw * sizeof(uint64_t));
        }
        if (b + 1 < nbits) {
            matmul(Mp, Mp, T, n, rw);
            memcpy(Mp, T, msz * sizeof(uint64_t));
        }
    }
    free(Mp); free(T); free(nv);
    return 0;
}
