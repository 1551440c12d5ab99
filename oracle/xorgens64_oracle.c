/*
 * Plain sequential CPU oracle of xorgens members with 64-bit words (w = 64).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing here is part of the product: only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load this file's library.  It shares no code, header or table with the HIP
 * path, and none with the 32-bit oracle beside it either: the same
 * definitions, written once more for 64-bit words so that each file reads
 * one word at a time against the paper.
 *
 * Definitions followed (section / equation of arXiv:1108.0486):
 *   - Section 2, the recurrence
 *         x_i = x_{i-r} (I + L^a)(I + R^b)  +  x_{i-s} (I + L^c)(I + R^d)
 *     over GF(2) on w-bit words ("+" is XOR; logical shifts; (I + L^a) acts
 *     first, row-vector convention), with a circular buffer of r words.
 *   - Section 1.5, the Weyl sequence W_k = W_{k-1} + omega mod 2^w and
 *     Eq. (1): output_k = W_k (I + R^gamma) + x_k mod 2^w (integer "+").
 *   - Section 1.5: the family has period 2^n - 1 for n = r w a power of two
 *     up to 4096, so w = 64 allows r <= 64.
 *
 * Readings (as for the 32-bit member): omega is the odd integer nearest
 * 2^{w-1}(sqrt 5 - 1); gamma = w / 2; the Weyl value is incremented, then
 * used; initialisation draws r + 1 SplitMix64 outputs from the stream's seed
 * (all 64 bits of each: r ring words x_{-r} .. x_{-1}, then the Weyl start),
 * sets x_{-1} = 1 if the ring is all zero, and discards 4r steps.
 * f64 uniform: (out >> 11) * 2^-53, exact, in [0, 1 - 2^-53].
 * f64 normal (the paper has none; the 32-bit member's Box-Muller pairing with
 * 53-bit uniforms): for the pair (o_{2m}, o_{2m+1}) of a call's outputs,
 *   u1 = ((o_{2m} >> 11) + 1) 2^-53 in (0, 1],  u2 = (o_{2m+1} >> 11) 2^-53,
 *   rho = sqrt(-2 ln u1),  z_{2m} = rho cos(2 pi u2),  z_{2m+1} = rho sin(2 pi u2),
 * evaluated in long double (64-bit significand) with the dyadic angle reduced
 * exactly, and rounded once to double: a reference for FP64 results.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <string.h>

#define XGO64_RMAX 64

typedef struct {
    uint32_t w, r, s, a, b, c, d, gamma; /* w must be 64 */
    uint64_t omega;
} xgo64_params;

typedef struct {
    uint64_t x[XGO64_RMAX]; /* x[(head + t) % r] = x_{k-r+t} */
    uint32_t head;
    uint64_t weyl;          /* W_{k-1} */
    uint64_t pos;
} xgo64_state;

int xgo64_params_valid(const xgo64_params *p)
{
    if (p->w != 64) return 0;
    if (p->r < 2 || p->r > XGO64_RMAX) return 0;
    if (p->s < 1 || p->s >= p->r) return 0;
    if (p->a < 1 || p->b < 1 || p->c < 1 || p->d < 1) return 0;
    if (p->a >= 64 || p->b >= 64 || p->c >= 64 || p->d >= 64) return 0;
    if (p->gamma >= 64) return 0;
    return 1;
}

/* x_k from x_{k-r} and x_{k-s}; x_k replaces x_{k-r} in the buffer. */
static uint64_t step_x(const xgo64_params *p, xgo64_state *st)
{
    const uint64_t x_r = st->x[st->head];
    const uint64_t x_s = st->x[(st->head + p->r - p->s) % p->r];
    uint64_t t = x_r ^ (x_r << p->a);
    t ^= t >> p->b;
    uint64_t v = x_s ^ (x_s << p->c);
    v ^= v >> p->d;
    const uint64_t xk = t ^ v;
    st->x[st->head] = xk;
    st->head = (st->head + 1) % p->r;
    return xk;
}

/* One output of Eq. (1). */
static uint64_t step_out(const xgo64_params *p, xgo64_state *st)
{
    const uint64_t xk = step_x(p, st);
    st->weyl += p->omega;
    st->pos += 1;
    return xk + (st->weyl ^ (st->weyl >> p->gamma));
}

static uint64_t splitmix64(uint64_t *z)
{
    uint64_t m;
    *z += 0x9E3779B97F4A7C15ull;
    m = *z;
    m = (m ^ (m >> 30)) * 0xBF58476D1CE4E5B9ull;
    m = (m ^ (m >> 27)) * 0x94D049BB133111EBull;
    return m ^ (m >> 31);
}

static void seed_state(const xgo64_params *p, xgo64_state *st, uint64_t seed)
{
    uint64_t z = seed, any = 0;
    uint32_t k;
    for (k = 0; k < p->r; k++) {
        st->x[k] = splitmix64(&z);
        any |= st->x[k];
    }
    st->weyl = splitmix64(&z);
    if (!any) st->x[p->r - 1] = 1;
    st->head = 0;
    st->pos = 0;
    for (k = 0; k < 4 * p->r; k++) (void)step_out(p, st);
    st->pos = 0;
}

static void load_state(const xgo64_params *p, xgo64_state *st, const uint64_t *ring,
                       uint64_t weyl, uint64_t pos)
{
    memcpy(st->x, ring, p->r * sizeof(uint64_t));
    st->head = 0;
    st->weyl = weyl;
    st->pos = pos;
}

static void save_state(const xgo64_params *p, const xgo64_state *st, uint64_t *ring,
                       uint64_t *weyl, uint64_t *pos)
{
    uint32_t t;
    for (t = 0; t < p->r; t++) ring[t] = st->x[(st->head + t) % p->r];
    *weyl = st->weyl;
    *pos = st->pos;
}

static const long double PI_L = 3.14159265358979323846264338327950288L;

/* Box-Muller on one pair of 64-bit outputs (see the header).  4 u2 is a
   multiple of 2^-51 below 4; it splits exactly into q + 2f with q the nearest
   integer and |f| <= 1/4, and the pair (cos, sin) of 2 pi u2 is that of pi f
   turned by q quarter turns. */
void xgo64_box_muller(uint64_t o_even, uint64_t o_odd, double *z0, double *z1)
{
    long double u1 = ldexpl((long double)((o_even >> 11) + 1u), -53);
    long double u2 = ldexpl((long double)(o_odd >> 11), -53);
    long double rho = sqrtl(-2.0L * logl(u1));
    long double y = 4.0L * u2;                 /* exact */
    long double q = nearbyintl(y);             /* exact integer 0 .. 4 */
    long double f = 0.5L * (y - q);            /* exact */
    long double sf = sinl(PI_L * f), cf = cosl(PI_L * f), s, c;
    int qi = (int)q % 4;
    if (f == 0.0L) { sf = 0.0L; cf = 1.0L; }
    switch (qi) {
    case 0: s = sf;  c = cf;  break;
    case 1: s = cf;  c = -sf; break;
    case 2: s = -sf; c = -cf; break;
    default: s = -cf; c = sf; break;
    }
    *z0 = (double)(rho * c);
    *z1 = (double)(rho * s);
}

enum { XGO64_U64 = 0, XGO64_F64 = 1, XGO64_NORMAL = 2, XGO64_MOMENTS = 3, XGO64_SKIP = 4 };

/* A normal (or moments) request of n variates consumes 2 ceil(n / 2) words
   (odd n drops the last sine value).  MOMENTS writes 3 doubles: the sums of
   z, z^2 and |z| over the n normals, accumulated in long double. */
static void run_one(const xgo64_params *p, xgo64_state *st, int kind, uint64_t n, void *out)
{
    uint64_t t;
    if (kind == XGO64_U64) {
        uint64_t *o = (uint64_t *)out;
        for (t = 0; t < n; t++) o[t] = step_out(p, st);
    } else if (kind == XGO64_F64) {
        double *o = (double *)out;
        for (t = 0; t < n; t++) o[t] = (double)(step_out(p, st) >> 11) * 0x1p-53;
    } else if (kind == XGO64_NORMAL || kind == XGO64_MOMENTS) {
        double *o = (double *)out;
        long double s1 = 0.0L, s2 = 0.0L, sa = 0.0L;
        for (t = 0; t < n; t += 2) {
            uint64_t e = step_out(p, st);
            uint64_t d = step_out(p, st);
            double z0, z1;
            xgo64_box_muller(e, d, &z0, &z1);
            if (kind == XGO64_NORMAL) {
                o[t] = z0;
                if (t + 1 < n) o[t + 1] = z1;
            } else {
                s1 += z0; s2 += (long double)z0 * z0; sa += fabsl(z0);
                if (t + 1 < n) { s1 += z1; s2 += (long double)z1 * z1; sa += fabsl(z1); }
            }
        }
        if (kind == XGO64_MOMENTS) { o[0] = (double)s1; o[1] = (double)s2; o[2] = (double)sa; }
    } else {
        for (t = 0; t < n; t++) (void)step_out(p, st);
    }
}

typedef struct {
    const xgo64_params *p;
    uint64_t *ring, *weyl, *pos;
    uint64_t n;
    int kind;
    void *out;
    uint64_t out_stride_bytes;
    uint64_t lo, hi;
} job64_t;

static void *worker(void *arg)
{
    job64_t *j = (job64_t *)arg;
    xgo64_state st;
    uint64_t i;
    for (i = j->lo; i < j->hi; i++) {
        load_state(j->p, &st, j->ring + i * j->p->r, j->weyl[i], j->pos[i]);
        run_one(j->p, &st, j->kind, j->n, j->out ? (char *)j->out + i * j->out_stride_bytes : NULL);
        save_state(j->p, &st, j->ring + i * j->p->r, &j->weyl[i], &j->pos[i]);
    }
    return NULL;
}

/* Seeds `count` streams: stream i <- seed + first + i.  ring[count][r],
   weyl[count], pos[count]. */
int xgo64_seed_streams(const xgo64_params *p, uint64_t seed, uint64_t first, uint64_t count,
                       uint64_t *ring, uint64_t *weyl, uint64_t *pos)
{
    xgo64_state st;
    uint64_t i;
    if (!xgo64_params_valid(p)) return -1;
    for (i = 0; i < count; i++) {
        seed_state(p, &st, seed + first + i);
        save_state(p, &st, ring + i * p->r, &weyl[i], &pos[i]);
    }
    return 0;
}

/* Advances every stream by n values of `kind` (U64: uint64_t out, F64: double
   out, NORMAL: double out, 2 ceil(n / 2) words; MOMENTS: 3 doubles per stream,
   the same words; SKIP: none), stream i's
   values at out + i * out_stride_bytes, on up
   to `threads` POSIX threads over disjoint streams. */
int xgo64_run_streams(const xgo64_params *p, uint64_t *ring, uint64_t *weyl, uint64_t *pos,
                      uint64_t count, int kind, uint64_t n, void *out, uint64_t out_stride_bytes,
                      int threads)
{
    pthread_t tid[256];
    job64_t jobs[256];
    int t, nt;
    if (!xgo64_params_valid(p)) return -1;
    if (kind < XGO64_U64 || kind > XGO64_SKIP) return -1;
    if (kind != XGO64_SKIP && out == NULL && count > 0) return -1;
    nt = threads < 1 ? 1 : (threads > 256 ? 256 : threads);
    if ((uint64_t)nt > count) nt = count ? (int)count : 1;
    for (t = 0; t < nt; t++) {
        jobs[t].p = p; jobs[t].ring = ring; jobs[t].weyl = weyl; jobs[t].pos = pos;
        jobs[t].n = n; jobs[t].kind = kind; jobs[t].out = out;
        jobs[t].out_stride_bytes = out_stride_bytes;
        jobs[t].lo = count * t / nt; jobs[t].hi = count * (t + 1) / nt;
    }
    if (nt == 1) { worker(&jobs[0]); return 0; }
    for (t = 0; t < nt; t++)
        if (pthread_create(&tid[t], NULL, worker, &jobs[t]) != 0) return -2;
    for (t = 0; t < nt; t++) pthread_join(tid[t], NULL);
    return 0;
}

/* Steps the x-part alone (GF(2)-linear) `steps` times in place, writing bit
   `bit` of each x_k to bits_out if non-null. */
int xgo64_xpart_run(const xgo64_params *p, uint64_t *ring, uint64_t steps, uint32_t bit,
                    uint8_t *bits_out)
{
    xgo64_state st;
    uint64_t k, w0 = 0, p0 = 0;
    if (!xgo64_params_valid(p) || bit >= 64) return -1;
    load_state(p, &st, ring, 0, 0);
    for (k = 0; k < steps; k++) {
        const uint64_t xk = step_x(p, &st);
        if (bits_out) bits_out[k] = (uint8_t)((xk >> bit) & 1u);
    }
    save_state(p, &st, ring, &w0, &p0);
    return 0;
}

/* Polynomial jump-ahead of the x-part: the state after J steps is
   sum_k g_k T^k state over GF(2), g = z^J mod P (n = 64 r bits of g). */
int xgo64_xpart_jump_poly(const xgo64_params *p, uint64_t *ring, const uint64_t *g)
{
    uint64_t cur[XGO64_RMAX], acc[XGO64_RMAX];
    uint32_t n, k, t;
    if (!xgo64_params_valid(p)) return -1;
    n = p->r * 64;
    memcpy(cur, ring, p->r * sizeof(uint64_t));
    memset(acc, 0, sizeof(acc));
    for (k = 0; k < n; k++) {
        if ((g[k / 64] >> (k % 64)) & 1u)
            for (t = 0; t < p->r; t++) acc[t] ^= cur[t];
        xgo64_xpart_run(p, cur, 1, 0, NULL);
    }
    memcpy(ring, acc, p->r * sizeof(uint64_t));
    return 0;
}

/* The x-part's one-step matrix M (n = 64 r rows of r words, row-major): state
   bit 64 t + b is bit b of ring word t (ring[t] = x_{pos-r+t}); column k is
   one step applied to the unit state e_k, so that next = M state. */
int xgo64_xpart_matrix(const xgo64_params *p, uint64_t *rows)
{
    uint64_t ring[XGO64_RMAX];
    uint32_t n, rw, k, t, b;
    if (!xgo64_params_valid(p)) return -1;
    n = p->r * 64;
    rw = n / 64;
    memset(rows, 0, (size_t)n * rw * sizeof(uint64_t));
    for (k = 0; k < n; k++) {
        memset(ring, 0, sizeof(ring));
        ring[k / 64] = 1ull << (k % 64);
        xgo64_xpart_run(p, ring, 1, 0, NULL);
        for (t = 0; t < p->r; t++)
            for (b = 0; b < 64; b++)
                if ((ring[t] >> b) & 1u) {
                    uint32_t i = t * 64 + b;
                    rows[(size_t)i * rw + k / 64] |= 1ull << (k % 64);
                }
    }
    return 0;
}
