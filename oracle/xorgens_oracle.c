/*
 * Plain sequential CPU oracle of the xorgens generator that xorgensGP runs on
 * the GPU (Nandapalan, Brent, Murray & Rendell, "High-Performance Pseudo-Random
 * Number Generation on Graphics Processing Units", arXiv:1108.0486).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this file's library.  It shares no code, header or table with the HIP
 * path.  It computes one word at a time, exactly as the recurrence is written,
 * so that a reader can check it against the paper by eye.
 *
 * Definitions followed (section / equation of the paper):
 *   - Section 2, the xorgens recurrence
 *         x_i = x_{i-r} (I + L^a)(I + R^b)  +  x_{i-s} (I + L^c)(I + R^d)
 *     over GF(2): "+" is XOR, L / R are logical left / right shifts of a
 *     w-bit word (row-vector convention: the matrices apply left to right, so
 *     (I + L^a) acts first).
 *   - Section 2, circular buffer of r words: x_i replaces x_{i-r}.
 *   - Section 1.5, Weyl generator W_k = W_{k-1} + omega mod 2^w, and
 *     Eq. (1): output_k = W_k (I + R^gamma) + x_k mod 2^w, where this "+" is
 *     integer addition (non-linear over GF(2)).
 *   - Section 2, parameter set (r,s,a,b,c,d) = (128,65,15,14,12,17), w = 32.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes of the repository):
 *   - omega: the odd integer nearest 2^{w-1}(sqrt 5 - 1) = 0x9E3779B9.
 *   - gamma: w/2 = 16.
 *   - Weyl order: W is incremented, then used with x_k.
 *   - Initialisation (the paper defers to the xorgens sources): SplitMix64
 *     from the 64-bit seed gives r + 1 values; the high w bits of the first r
 *     fill x_{-r} .. x_{-1}, the next one is the Weyl start; an all-zero ring
 *     gets x_{-1} = 1; then 4r generator steps are run and discarded.
 *     Stream i of a family seeded with "seed" uses seed + i (mod 2^64), as the
 *     paper seeds each block with consecutive values (Section 4).
 *   - f32 uniform: (out >> 8) * 2^-24, exact.
 *   - normal (FP64): Box-Muller on consecutive pairs (out_{2m}, out_{2m+1}) of
 *     the call, u1 = ((out_{2m} >> 8) + 1) 2^-24 in (0,1],
 *     u2 = (out_{2m+1} >> 8) 2^-24 in [0,1), rho = sqrt(-2 ln u1),
 *     z_{2m} = rho cos(2 pi u2), z_{2m+1} = rho sin(2 pi u2), with the angle
 *     reduced exactly (2 u2 is dyadic) before calling sin / cos.
 */
#include <stdint.h>
#include <string.h>
#include <stdlib.h>
#include <math.h>
#include <pthread.h>

#define XGO_RMAX 128

typedef struct {
    uint32_t w, r, s, a, b, c, d, gamma;
    uint32_t omega;
} xgo_params;

typedef struct {
    uint32_t x[XGO_RMAX]; /* circular buffer: x[(head + t) % r] = x_{k-r+t} */
    uint32_t head;        /* slot of x_{k-r}, the oldest word */
    uint32_t weyl;        /* W_{k-1}, the last Weyl value used */
    uint64_t pos;         /* k: number of outputs produced since seeding */
} xgo_state;

static uint32_t word_mask(const xgo_params *p)
{
    return p->w == 32 ? 0xFFFFFFFFu : ((1u << p->w) - 1u);
}

int xgo_params_valid(const xgo_params *p)
{
    if (p->w < 2 || p->w > 32) return 0;
    if (p->r < 2 || p->r > XGO_RMAX) return 0;
    if (p->s < 1 || p->s >= p->r) return 0;
    if (p->a < 1 || p->b < 1 || p->c < 1 || p->d < 1) return 0;
    if (p->a >= p->w || p->b >= p->w || p->c >= p->w || p->d >= p->w) return 0;
    if (p->gamma >= p->w) return 0;
    return 1;
}

/* ---- the recurrence (Section 2) ---------------------------------------- */

/* One step of the x-part: returns x_k and stores it in the slot of x_{k-r}. */
static uint32_t step_x(const xgo_params *p, xgo_state *st)
{
    const uint32_t m = word_mask(p);
    const uint32_t x_r = st->x[st->head];                           /* x_{k-r} */
    const uint32_t x_s = st->x[(st->head + p->r - p->s) % p->r];    /* x_{k-s} */
    uint32_t t = x_r ^ ((x_r << p->a) & m);   /* x_{k-r} (I + L^a) */
    t ^= t >> p->b;                           /*         (I + R^b) */
    uint32_t v = x_s ^ ((x_s << p->c) & m);   /* x_{k-s} (I + L^c) */
    v ^= v >> p->d;                           /*         (I + R^d) */
    const uint32_t xk = t ^ v;
    st->x[st->head] = xk;
    st->head = (st->head + 1) % p->r;
    return xk;
}

/* One generator output: Weyl step, then Eq. (1). */
static uint32_t step_out(const xgo_params *p, xgo_state *st)
{
    const uint32_t m = word_mask(p);
    const uint32_t xk = step_x(p, st);
    st->weyl = (st->weyl + p->omega) & m;
    st->pos += 1;
    return (xk + (st->weyl ^ (st->weyl >> p->gamma))) & m;
}

/* ---- initialisation ------------------------------------------------------ */

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): golden-gamma increment, then
   the variant-13 finaliser of MurmurHash3. */
uint64_t xgo_splitmix64(uint64_t *z)
{
    uint64_t m;
    *z += 0x9E3779B97F4A7C15ull;
    m = *z;
    m = (m ^ (m >> 30)) * 0xBF58476D1CE4E5B9ull;
    m = (m ^ (m >> 27)) * 0x94D049BB133111EBull;
    return m ^ (m >> 31);
}

static void seed_state(const xgo_params *p, xgo_state *st, uint64_t seed)
{
    const uint32_t m = word_mask(p);
    uint64_t z = seed;
    uint32_t k, any = 0;
    for (k = 0; k < p->r; k++) {
        st->x[k] = (uint32_t)(xgo_splitmix64(&z) >> (64 - p->w)) & m;
        any |= st->x[k];
    }
    st->weyl = (uint32_t)(xgo_splitmix64(&z) >> (64 - p->w)) & m;
    if (!any) st->x[p->r - 1] = 1;
    st->head = 0;
    st->pos = 0;
    for (k = 0; k < 4 * p->r; k++) (void)step_out(p, st);
    st->pos = 0;
}

/* ---- state import / export (linear ring: ring[t] = x_{pos-r+t}) ---------- */

static void load_state(const xgo_params *p, xgo_state *st, const uint32_t *ring,
                       uint32_t weyl, uint64_t pos)
{
    memcpy(st->x, ring, p->r * sizeof(uint32_t));
    st->head = 0;
    st->weyl = weyl;
    st->pos = pos;
}

static void save_state(const xgo_params *p, const xgo_state *st, uint32_t *ring,
                       uint32_t *weyl, uint64_t *pos)
{
    uint32_t t;
    for (t = 0; t < p->r; t++) ring[t] = st->x[(st->head + t) % p->r];
    *weyl = st->weyl;
    *pos = st->pos;
}

/* ---- output mappings ----------------------------------------------------- */

static float map_f32(uint32_t o)
{
    return (float)ldexp((double)(o >> 8), -24);
}

/* sin(pi v), cos(pi v) for a dyadic v in [0, 2): v is reduced exactly to
   v = q/2 + f with q an integer and |f| <= 1/4, then rotated by q quarter turns. */
static void sincospi_exact(double v, double *s, double *c)
{
    double y = 2.0 * v;            /* exact */
    double q = nearbyint(y);       /* exact integer */
    double f = 0.5 * (y - q);      /* exact, |f| <= 1/4 */
    double sf = sin(M_PI * f), cf = cos(M_PI * f);
    int qi = ((int)q % 4 + 4) % 4;
    if (f == 0.0) { sf = 0.0; cf = 1.0; }
    switch (qi) {
    case 0: *s = sf;  *c = cf;  break;
    case 1: *s = cf;  *c = -sf; break;
    case 2: *s = -sf; *c = -cf; break;
    default: *s = -cf; *c = sf; break;
    }
}

void xgo_box_muller(uint32_t o_even, uint32_t o_odd, double *z0, double *z1)
{
    double u1 = ldexp((double)((o_even >> 8) + 1u), -24);
    double u2 = ldexp((double)(o_odd >> 8), -24);
    double rho = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi_exact(2.0 * u2, &s, &c);
    *z0 = rho * c;
    *z1 = rho * s;
}

/* The map above over many caller-given word pairs: out[2m], out[2m + 1] are
   z_0, z_1 of the pair (words[2m], words[2m + 1]), for m < pairs. */
void xgo_box_muller_many(const uint32_t *words, uint64_t pairs, double *out)
{
    uint64_t m;
    for (m = 0; m < pairs; m++) xgo_box_muller(words[2 * m], words[2 * m + 1], &out[2 * m], &out[2 * m + 1]);
}

/* ---- single-stream drivers ---------------------------------------------- */

enum { XGO_U32 = 0, XGO_F32 = 1, XGO_NORMAL = 2, XGO_MOMENTS = 3, XGO_SKIP = 4 };

/* Runs one request of kind `kind` on one stream.  `out` is uint32_t* (U32),
   float* (F32), double* (NORMAL: n values; MOMENTS: 3 values, the sums of z,
   z^2 and |z|).  A normal or moments request of n variates consumes
   2 * ceil(n / 2) words. */
static void run_one(const xgo_params *p, xgo_state *st, int kind, uint64_t n, void *out)
{
    uint64_t t;
    if (kind == XGO_U32) {
        uint32_t *o = (uint32_t *)out;
        for (t = 0; t < n; t++) o[t] = step_out(p, st);
    } else if (kind == XGO_F32) {
        float *o = (float *)out;
        for (t = 0; t < n; t++) o[t] = map_f32(step_out(p, st));
    } else if (kind == XGO_NORMAL || kind == XGO_MOMENTS) {
        double *o = (double *)out, s1 = 0.0, s2 = 0.0, sa = 0.0;
        for (t = 0; t < n; t += 2) {
            uint32_t e = step_out(p, st);
            uint32_t d = step_out(p, st);
            double z0, z1;
            xgo_box_muller(e, d, &z0, &z1);
            if (kind == XGO_NORMAL) {
                o[t] = z0;
                if (t + 1 < n) o[t + 1] = z1;
            } else {
                s1 += z0; s2 += z0 * z0; sa += fabs(z0);
                if (t + 1 < n) { s1 += z1; s2 += z1 * z1; sa += fabs(z1); }
            }
        }
        if (kind == XGO_MOMENTS) { o[0] = s1; o[1] = s2; o[2] = sa; }
    } else { /* XGO_SKIP */
        for (t = 0; t < n; t++) (void)step_out(p, st);
    }
}

/* ---- many streams, one thread per share of streams ---------------------- */

typedef struct {
    const xgo_params *p;
    uint32_t *ring; uint32_t *weyl; uint64_t *pos;
    uint64_t count, n;
    int kind;
    void *out;
    size_t out_stride_bytes;
    uint64_t lo, hi;
} job_t;

static void *worker(void *arg)
{
    job_t *j = (job_t *)arg;
    xgo_state st;
    uint64_t i;
    for (i = j->lo; i < j->hi; i++) {
        load_state(j->p, &st, j->ring + i * j->p->r, j->weyl[i], j->pos[i]);
        run_one(j->p, &st, j->kind, j->n,
                j->out ? (char *)j->out + i * j->out_stride_bytes : NULL);
        save_state(j->p, &st, j->ring + i * j->p->r, &j->weyl[i], &j->pos[i]);
    }
    return NULL;
}

/* Seeds `count` streams: stream i <- seed + first + i.  State arrays are
   ring[count][r], weyl[count], pos[count]. */
int xgo_seed_streams(const xgo_params *p, uint64_t seed, uint64_t first, uint64_t count,
                     uint32_t *ring, uint32_t *weyl, uint64_t *pos)
{
    xgo_state st;
    uint64_t i;
    if (!xgo_params_valid(p)) return -1;
    for (i = 0; i < count; i++) {
        seed_state(p, &st, seed + first + i);
        save_state(p, &st, ring + i * p->r, &weyl[i], &pos[i]);
    }
    return 0;
}

/* Advances every stream by one request of `kind` and length n, writing
   stream i's result at out + i * out_stride_bytes.  Uses up to `threads`
   POSIX threads over disjoint streams. */
int xgo_run_streams(const xgo_params *p, uint32_t *ring, uint32_t *weyl, uint64_t *pos,
                    uint64_t count, int kind, uint64_t n, void *out,
                    uint64_t out_stride_bytes, int threads)
{
    pthread_t tid[256];
    job_t jobs[256];
    int t, nt;
    if (!xgo_params_valid(p)) return -1;
    if (kind < XGO_U32 || kind > XGO_SKIP) return -1;
    if (kind != XGO_SKIP && out == NULL && count > 0) return -1;
    nt = threads < 1 ? 1 : (threads > 256 ? 256 : threads);
    if ((uint64_t)nt > count) nt = count ? (int)count : 1;
    for (t = 0; t < nt; t++) {
        jobs[t].p = p; jobs[t].ring = ring; jobs[t].weyl = weyl; jobs[t].pos = pos;
        jobs[t].count = count; jobs[t].n = n; jobs[t].kind = kind; jobs[t].out = out;
        jobs[t].out_stride_bytes = out_stride_bytes;
        jobs[t].lo = count * t / nt; jobs[t].hi = count * (t + 1) / nt;
    }
    if (nt == 1) { worker(&jobs[0]); return 0; }
    for (t = 0; t < nt; t++)
        if (pthread_create(&tid[t], NULL, worker, &jobs[t]) != 0) return -2;
    for (t = 0; t < nt; t++) pthread_join(tid[t], NULL);
    return 0;
}

/* ---- the x-part alone (GF(2)-linear), for the algebraic checks ------------ */

/* Steps the x-part of one ring `steps` times (no Weyl), leaving the linear
   ring in place, and writes bit `bit` of each x_k to bits_out (if non-null). */
int xgo_xpart_run(const xgo_params *p, uint32_t *ring, uint64_t steps, uint32_t bit,
                  uint8_t *bits_out)
{
    xgo_state st;
    uint64_t k;
    uint32_t w0 = 0; uint64_t p0 = 0;
    if (!xgo_params_valid(p) || bit >= p->w) return -1;
    load_state(p, &st, ring, 0, 0);
    for (k = 0; k < steps; k++) {
        uint32_t xk = step_x(p, &st);
        if (bits_out) bits_out[k] = (uint8_t)((xk >> bit) & 1u);
    }
    save_state(p, &st, ring, &w0, &p0);
    return 0;
}

/* Brute-force cycle length of the x-part from `ring` (n = r w <= 64 bits of
   state), or 0 if it exceeds max_steps. */
uint64_t xgo_xpart_period(const xgo_params *p, const uint32_t *ring, uint64_t max_steps)
{
    xgo_state st, s0;
    uint64_t k;
    if (!xgo_params_valid(p)) return 0;
    load_state(p, &s0, ring, 0, 0);
    st = s0;
    for (k = 1; k <= max_steps; k++) {
        uint32_t t, same = 1;
        (void)step_x(p, &st);
        for (t = 0; t < p->r; t++)
            if (st.x[(st.head + t) % p->r] != s0.x[t]) { same = 0; break; }
        if (same) return k;
    }
    return 0;
}

/* Brute-force cycle length of the full generator state (x-part and Weyl). */
uint64_t xgo_full_period(const xgo_params *p, const uint32_t *ring, uint32_t weyl,
                         uint64_t max_steps)
{
    xgo_state st, s0;
    uint64_t k;
    if (!xgo_params_valid(p)) return 0;
    load_state(p, &s0, ring, weyl, 0);
    st = s0;
    for (k = 1; k <= max_steps; k++) {
        uint32_t t, same;
        (void)step_out(p, &st);
        same = st.weyl == s0.weyl;
        for (t = 0; same && t < p->r; t++)
            if (st.x[(st.head + t) % p->r] != s0.x[t]) same = 0;
        if (same) return k;
    }
    return 0;
}

/* The x-part as an n x n bit matrix (n = r w), row-major with
   rw = (n - 1) / 64 + 1 words per row.  State bit w t + b is bit b of ring
   word t (ring[t] = x_{pos-r+t}).  Column k is one step applied to the unit
   state e_k, so that next = M state. */
int xgo_xpart_matrix(const xgo_params *p, uint64_t *rows)
{
    uint32_t n, rw, k, t, b;
    uint32_t ring[XGO_RMAX];
    if (!xgo_params_valid(p)) return -1;
    n = p->r * p->w;
    rw = (n - 1) / 64 + 1;
    memset(rows, 0, (size_t)n * rw * sizeof(uint64_t));
    for (k = 0; k < n; k++) {
        memset(ring, 0, sizeof(ring));
        ring[k / p->w] = 1u << (k % p->w);
        xgo_xpart_run(p, ring, 1, 0, NULL);
        for (t = 0; t < p->r; t++)
            for (b = 0; b < p->w; b++)
                if ((ring[t] >> b) & 1u) {
                    uint32_t i = t * p->w + b;
                    rows[(size_t)i * rw + k / 64] |= 1ull << (k % 64);
                }
    }
    return 0;
}

/* Polynomial jump-ahead of the x-part: with g = z^J mod P (P the
   characteristic polynomial of the step matrix T, degree n = r w), T^J = g(T)
   by Cayley-Hamilton, so the state after J steps is the XOR of the states
   after k steps, 0 <= k < n, over the k with g_k = 1.  `g` is a bit array of
   n bits in 64-bit words; `ring` is replaced by the jumped ring. */
int xgo_xpart_jump_poly(const xgo_params *p, uint32_t *ring, const uint64_t *g)
{
    uint32_t n, k, t;
    uint32_t cur[XGO_RMAX], acc[XGO_RMAX];
    if (!xgo_params_valid(p)) return -1;
    n = p->r * p->w;
    memcpy(cur, ring, p->r * sizeof(uint32_t));
    memset(acc, 0, sizeof(acc));
    for (k = 0; k < n; k++) {
        if ((g[k / 64] >> (k % 64)) & 1u)
            for (t = 0; t < p->r; t++) acc[t] ^= cur[t];
        xgo_xpart_run(p, cur, 1, 0, NULL);
    }
    memcpy(ring, acc, p->r * sizeof(uint32_t));
    return 0;
}
