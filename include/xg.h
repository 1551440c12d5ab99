/*
 * xg.h -- C ABI of libxg: many independent xorgens streams generated on an
 * AMD Instinct MI355X (gfx950).
 *
 * The generator is xorgens as used by xorgensGP (Nandapalan, Brent, Murray &
 * Rendell, arXiv:1108.0486):
 *   - Section 2: x_i = x_{i-r}(I + L^a)(I + R^b) xor x_{i-s}(I + L^c)(I + R^d)
 *     with (r,s,a,b,c,d) = (128,65,15,14,12,17) on 32-bit words; the r = 128
 *     words form a circular buffer and x_i replaces x_{i-r};
 *   - Section 1.5: Weyl sequence W_k = W_{k-1} + omega (mod 2^32) and the output
 *     of Eq. (1), out_k = x_k + (W_k xor (W_k >> gamma)) (mod 2^32), with
 *     omega = 0x9E3779B9 (the odd integer nearest 2^31 (sqrt 5 - 1)) and
 *     gamma = 16;
 *   - Section 2: many independent subsequences, one per group of threads;
 *     up to 64 consecutive words of one stream are computed at once (the
 *     terms x_k .. x_{k+C-1} need only older words while C <= s = 65).
 *
 * Conventions shared by every entry point:
 *   - Pointers named d_* are device pointers owned by the caller.  The
 *     library never allocates or frees device memory (apart from the static
 *     array of xg_generate_batch_static, reserved when the code loads); each
 *     generating call only enqueues kernels on `stream` (a hipStream_t passed
 *     as void*; NULL is the null stream) and returns.
 *   - Invalid arguments are rejected synchronously with a negative status;
 *     then nothing is enqueued and no state changes.  A launch failure
 *     reported by the HIP runtime right after the launch gives XG_EHIP.
 *     Faults inside a kernel surface at the caller's next synchronisation.
 *   - Calls that touch the same streams must be ordered by the caller (same
 *     HIP stream, or events).  Calls on disjoint stream ranges may overlap.
 *   - All sizes count elements (4-byte words), not bytes, unless named *_bytes.
 *   - No C++ exception crosses this interface.
 *   - Host threads: calls on different handles may come from different host
 *     threads.  A handle's launch shape and batch scratch are read at each
 *     launch, so xg_set_plain_tune and xg_set_batch_scratch must not race with
 *     launches on the same handle.  A request server is driven by one host
 *     thread.
 *   - Process-wide state: the jump polynomials' modulus (built once per member
 *     and process, thread-safely) and the 16 most recent jump polynomials
 *     (guarded by a lock), the tuning cache (guarded by a lock), and
 *     xg_generate_batch_static's device array (one per GPU).
 *
 * Stream state (device memory, XG_STATE_WORDS 32-bit words per stream, 528 B):
 *   words [0, 128)   ring[t] = x_{pos-128+t}, the last 128 words of the x-part
 *   word  128        W_{pos-1}, the last Weyl value used
 *   word  129        reserved, 0
 *   words 130, 131   pos, the number of words consumed since seeding
 *                    (uint64, little endian)
 * A stream's state is a plain value: copying those 528 bytes out and back is a
 * checkpoint and a resume.
 */
#ifndef XG_H
#define XG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t xg_status;

#define XG_OK        0
#define XG_EINVAL   (-1)  /* null pointer, zero or out-of-range argument, bad dtype */
#define XG_ERANGE   (-2)  /* stream range outside the context, or a size overflow  */
#define XG_EALIGN   (-3)  /* device pointer not 4-byte (outputs) or 16-byte (state) aligned */
#define XG_EHIP     (-4)  /* the HIP runtime reported an error */
#define XG_ENOTSUP  (-5)  /* the current device is not gfx950, or the stream family
                              has no such operation */
#define XG_ENOMEM   (-6)  /* a host-side allocation failed */
#define XG_EBUSY    (-7)  /* workspace too small for the request table */

#define XG_STATE_WORDS 132u

/* Output types of a request. */
#define XG_U32     0u  /* out_k as uint32 */
#define XG_F32     1u  /* (out_k >> 8) * 2^-24 as float, in [0, 1 - 2^-24]; exact */
#define XG_NORMAL  2u  /* float standard normals by Box-Muller (see xg_generate_normal) */
#define XG_U64     4u  /* out_k as uint64 (64-bit-word family only) */
#define XG_F64     5u  /* (out_k >> 11) * 2^-53 as double, in [0, 1 - 2^-53]; exact */

/* Members of the xorgens family (Section 1.5: period 2^n - 1 with n = r w a
 * power of two up to 4096; Section 2: s = r/2 +- 1 for the GPU).  Every
 * member uses omega = the odd integer nearest 2^{w-1}(sqrt 5 - 1) and
 * gamma = w / 2.
 *   XG_FAMILY_R128_W32  Section 2's member: w = 32, (r,s,a,b,c,d) =
 *                       (128,65,15,14,12,17); n = 4096.  Every call of this
 *                       header supports it.
 *   XG_FAMILY_R64_W32   w = 32, (64,33,19,19,9,18); n = 2048, a 272-byte
 *                       state.  Plain and bulk-fill u32 / f32, normals and
 *                       fused moments (as for Section 2's member), xg_skip,
 *                       batches, and a server without segments.
 *   XG_FAMILY_R64_W64   w = 64, (64,33,24,22,37,45); n = 4096, 64-bit outputs
 *                       (xg_generate_u64 / f64, xg_fill_u64 / f64), FP64
 *                       normals and their fused moments
 *                       (xg_generate_normal_f64, xg_normal_moments_f64),
 *                       xg_skip, batches (u64 / f64 / FP64 normals), and a
 *                       server without segments.
 * The paper gives shifts only for the first; those of the other two were
 * chosen by a search for primitive characteristic polynomials.  Calls a
 * member does not support return XG_ENOTSUP. */
#define XG_FAMILY_R128_W32 0u
#define XG_FAMILY_R64_W32  1u
#define XG_FAMILY_R64_W64  2u

typedef struct xg_ctx xg_ctx;

/* Bytes of device state for num_streams streams (num_streams * 528). */
size_t xg_state_bytes(uint64_t num_streams);

/* Seeds num_streams streams into d_state and creates a host-side handle.
 * Stream i is seeded from seed + i (mod 2^64), as the paper seeds block b with
 * consecutive values (Section 4).  The paper defers the seeding method to the
 * xorgens sources; this library's method: SplitMix64 from the stream's seed
 * yields 129 values whose high 32 bits fill x_{-128} .. x_{-1} and W; a ring
 * that is all zero gets x_{-1} = 1; then 512 generator steps are discarded and
 * pos is set to 0.
 *   out          receives the handle (owned by the caller; free with xg_destroy)
 *   d_state      device buffer of at least xg_state_bytes(num_streams) bytes,
 *                16-byte aligned; the handle keeps the pointer, never the memory
 *   state_bytes  size of d_state in bytes
 *   num_streams  1 .. 2^32 - 1
 * Errors: XG_EINVAL, XG_ERANGE (state_bytes too small), XG_EALIGN,
 * XG_ENOTSUP, XG_ENOMEM, XG_EHIP.  On error *out is NULL. */
xg_status xg_init_streams(xg_ctx **out, void *d_state, size_t state_bytes,
                          uint64_t num_streams, uint64_t seed, void *stream);

/* Wraps an already seeded state buffer (for example one restored from a
 * checkpoint) in a new handle without touching it.  Same arguments and errors
 * as xg_init_streams, minus the seed. */
xg_status xg_attach_streams(xg_ctx **out, void *d_state, size_t state_bytes,
                            uint64_t num_streams);

/* Frees the host handle; never touches d_state.  NULL is accepted. */
void xg_destroy(xg_ctx *ctx);

/* Number of streams and state pointer of a handle (0 / NULL for NULL). */
uint64_t xg_num_streams(const xg_ctx *ctx);
void *xg_state_ptr(const xg_ctx *ctx);

/* Bytes of device state for num_streams streams of a family (0 for an
 * unknown family).  Per stream: R128_W32 528 (see XG_STATE_WORDS); R64_W32
 * 272: ring uint32[64] (ring[t] = x_{pos-64+t}), W_{pos-1}, a zero word, pos
 * (uint64); R64_W64 528: ring uint64[64], W_{pos-1} (uint64), pos (uint64). */
size_t xg_family_state_bytes(uint32_t family, uint64_t num_streams);

/* xg_init_streams / xg_attach_streams for a family.  Seeding of the 32-bit
 * members is that of xg_init_streams with r ring words: SplitMix64(seed + i)
 * outputs 1 .. r give x_{-r} .. x_{-1} (their high w bits), output r + 1 the
 * Weyl start, an all-zero ring gets x_{-1} = 1, and 4 r steps are discarded;
 * the 64-bit member takes all 64 bits of each output.
 * Errors: those of xg_init_streams, and XG_EINVAL for an unknown family. */
xg_status xg_init_family(xg_ctx **out, uint32_t family, void *d_state, size_t state_bytes,
                         uint64_t num_streams, uint64_t seed, void *stream);
xg_status xg_attach_family(xg_ctx **out, uint32_t family, void *d_state, size_t state_bytes,
                           uint64_t num_streams);

/* Family of a handle (XG_FAMILY_*; UINT32_MAX for NULL). */
uint32_t xg_family(const xg_ctx *ctx);

/* Launch shape of a kernel.  Any shape gives the same output bits;
 * xg_autotune_batch picks the fastest for a batch.  A batch launch given no
 * shape takes a default by its number of queue items (groups; for
 * xg_generate_batch and xg_generate_batch_static, requests): {4, 8, 2, 1}
 * with at least 8 per compute unit, where HBM writes bound the launch, else
 * {4, 8, 8, 1}, where each wavefront's own rate does. */
typedef struct {
    uint32_t waves_per_block;  /* streams served at once by one workgroup: 1, 2, 4, 8, 16 */
    uint32_t unroll;           /* 64-word chunks per thread per loop trip: 1, 2, 4, 8
                                  (0: chosen per launch, plain tune only) */
    uint32_t blocks_per_cu;    /* persistent workgroups per compute unit: 1 .. 32 */
    uint32_t store_words;      /* words each lane writes per store instruction: 1, or 4
                                  (groups of four chunks staged through a 1 KB LDS slot
                                  per wavefront; needs unroll >= 4); 0 = library default */
} xg_tune;

/* Launch shape of the plain and fill launches of this handle
 * (waves_per_block, unroll and store_words are used; blocks_per_cu is
 * ignored).  waves_per_block 0 chooses per launch: 4 when count >= 4 x the
 * compute units, else 2 when count >= 2 x, else 1, so one stream's wavefront
 * lands on each SIMD before any SIMD gets a second.  unroll 0 chooses per
 * launch (measured fastest for each): for Section 2's member, when count is
 * at least 4 x the compute units, 4 for the bulk-fill uint32 launch, 8 for
 * the bulk-fill FP32 launch, and 2 with 4-byte stores for the stream-major
 * uint32 and FP32 launches; for XG_FAMILY_R64_W32 (count at least 8 x the
 * compute units: two streams per wavefront) 2 for its stream-major launches;
 * 8 for every other launch.  The default is {0, 0, 1, 4}.  Output bits do not
 * depend on it.
 * Errors: XG_EINVAL (NULL pointer or a shape outside the ranges of xg_tune). */
xg_status xg_set_plain_tune(xg_ctx *ctx, const xg_tune *tune);
xg_status xg_get_plain_tune(const xg_ctx *ctx, xg_tune *tune);

/* The plain launch: streams first .. first + count - 1 each produce n values
 * from their current position, written stream-major:
 *     d_out[(i - first) * n + t] = value t of stream i,   t < n,
 * then each stream's state advances by n words.  One wavefront serves one
 * stream; d_out must hold count * n elements and be 4-byte aligned (16-byte
 * alignment gives the fastest stores).
 * Errors: XG_EINVAL (NULL ctx, NULL d_out with n > 0, count == 0), XG_ERANGE
 * (first + count > num_streams, or count * n overflows), XG_EALIGN, XG_EHIP.
 * n == 0 is valid (d_out may then be NULL): nothing is enqueued or written. */
xg_status xg_generate_u32(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                          uint32_t *d_out, void *stream);
xg_status xg_generate_f32(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                          float *d_out, void *stream);

/* Bulk fill: the same values as xg_generate_u32 / xg_generate_f32 (same
 * streams, same positions, same state advance), placed for HBM write
 * bandwidth rather than per stream.  With k = i - first, full = n / 64 and
 * rem = n mod 64, value t of stream i is at
 *     d_out[(t / 64) * 64 * count + k * 64 + t mod 64]        for t < 64 * full,
 *     d_out[64 * full * count + k * rem + (t - 64 * full)]      otherwise,
 * so the count * n outputs fill d_out contiguously with no gaps, and the
 * wavefronts of a launch advance together through one dense region of HBM
 * (stream-major placement keeps count write fronts n words apart).  A chunk
 * of 64 words of one stream stays contiguous.  For XG_FAMILY_R64_W32 the chunk
 * is 32 words (read 32 for 64 above).  Same arguments and errors as
 * xg_generate_u32; waves_per_block and unroll of the plain tune apply. */
xg_status xg_fill_u32(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                      uint32_t *d_out, void *stream);
xg_status xg_fill_f32(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                      float *d_out, void *stream);

/* 64-bit outputs of the XG_FAMILY_R64_W64 member (Section 1.5: xorgens with
 * w = 64).  Layouts and errors as xg_generate_u32 / xg_fill_u32 with 64-bit
 * elements, except that the bulk-fill chunk is 32 words:
 *   xg_generate_*: stream i's t-th value at d_out[(i - first) n + t];
 *   xg_fill_*:     chunk c (values 32c .. 32c + 31) of the k-th stream of the
 *                  call at d_out[(c count + k) 32 ..], then the ragged last
 *                  chunks (n mod 32 values each) packed at
 *                  d_out[32 (n / 32) count + k (n mod 32) ..].
 * u64: out_k.  f64: (out_k >> 11) * 2^-53, exact.  d_out 8-byte aligned.
 * Other families: XG_ENOTSUP.  (XG_FAMILY_R64_W32 uses xg_generate_u32 /
 * f32 and xg_fill_u32 / f32, whose bulk-fill chunk is then 32 words.) */
xg_status xg_generate_u64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                          uint64_t *d_out, void *stream);
xg_status xg_generate_f64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                          double *d_out, void *stream);
xg_status xg_fill_u64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                      uint64_t *d_out, void *stream);
xg_status xg_fill_f64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                      double *d_out, void *stream);

/* FP64 standard normals of XG_FAMILY_R64_W64 (the paper has no 64-bit
 * member; this is xg_generate_normal's pairing with 53-bit uniforms): for
 * consecutive outputs (o_{2m}, o_{2m+1}) of the call, u1 = ((o_{2m} >> 11)
 * + 1) 2^-53 in (0, 1], u2 = (o_{2m+1} >> 11) 2^-53, rho = sqrt(-2 ln u1),
 * z_{2m} = rho cos(2 pi u2), z_{2m+1} = rho sin(2 pi u2), in FP64 with the
 * angle reduced exactly.  Stream-major d_out[(i - first) n + t] (8-byte
 * aligned; pairs go out as 16-byte stores when it is 16-byte aligned and n
 * even).  Consumes 2 ceil(n / 2) words (odd n drops the last sine value).
 * Other families: XG_ENOTSUP.  Otherwise the errors of xg_generate_u64. */
xg_status xg_generate_normal_f64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                                 double *d_out, void *stream);

/* Fused FP64 generate-and-consume for XG_FAMILY_R64_W64: each stream draws n
 * normals exactly as xg_generate_normal_f64 would (never written to memory)
 * and reduces them in-kernel to d_sums[2 (i - first)] = sum of z and
 * d_sums[2 (i - first) + 1] = sum of z^2, in FP64 with compensated per-lane
 * sums and a pairwise reduction across the stream's lanes.  The streams
 * advance by 2 ceil(n / 2) words.  Other families: XG_ENOTSUP.  Otherwise
 * the errors of xg_generate_u64 (d_sums holds 2 * count doubles). */
xg_status xg_normal_moments_f64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                                double *d_sums, void *stream);

/* Standard normals by the Box-Muller transform on consecutive pairs of
 * outputs (o_{2m}, o_{2m+1}) of the call: u1 = ((o_{2m} >> 8) + 1) 2^-24 in
 * (0, 1], u2 = (o_{2m+1} >> 8) 2^-24 in [0, 1), rho = sqrt(-2 ln u1),
 * z_{2m} = rho cos(2 pi u2), z_{2m+1} = rho sin(2 pi u2), in FP32 (sine and
 * cosine of pi * (2 u2), so the angle is reduced exactly).  Each stream
 * consumes 2 * ceil(n / 2) words; for odd n the last sine value is dropped.
 * Same layout and errors as xg_generate_u32. */
xg_status xg_generate_normal(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                             float *d_out, void *stream);

/* The Box-Muller map of xg_generate_normal on caller-supplied words: for
 * m < pairs, d_out[2m] and d_out[2m + 1] are z_0 and z_1 of the pair
 * (d_words[2m], d_words[2m + 1]), computed by the same device code.  Lets a
 * caller (or a test) apply the map to any words, e.g. every possible u1.
 * Errors: XG_EINVAL (NULL with pairs > 0), XG_ERANGE, XG_EALIGN, XG_EHIP. */
xg_status xg_box_muller(const uint32_t *d_words, uint64_t pairs, float *d_out, void *stream);

/* Fused generate-and-consume: each stream draws n normals exactly as
 * xg_generate_normal would (the same values, never written to memory) and
 * reduces them in-kernel to
 *     d_sums[2 (i - first)]     = sum of z      (FP32)
 *     d_sums[2 (i - first) + 1] = sum of z^2    (FP32)
 * with compensated FP32 per-lane sums, reduced across the wavefront in FP64
 * and rounded once to FP32.  The streams advance by 2 * ceil(n / 2) words.
 * Same errors as xg_generate_u32 (d_sums holds 2 * count floats). */
xg_status xg_normal_moments(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                            float *d_sums, void *stream);

/* Advances streams first .. first + count - 1 by J words each, producing
 * nothing: afterwards they are where J generated words would have left them
 * (positions, rings and Weyl values).  Short skips (J < 2^15) step through the
 * words; longer ones jump: the x-part is GF(2)-linear (Section 1.5), its
 * 4096-bit state moves by a matrix T, and T^J = g(T) with g = z^J mod P, P
 * the characteristic polynomial of T (degree 4096, primitive); the host
 * computes g (keeping the 16 most recent (member, J) results, so a repeated
 * J costs no powering) and the device evaluates g(T) on each stream's state
 * by Horner's rule in steps of 64 words: one wavefront per stream, or, when
 * the streams fit on the GPU at once (at most 3 per compute unit), a
 * workgroup of four per stream.  The Weyl value advances by J omega.
 * Every family member is supported: for the r = 64 members P has degree n
 * (2048 or 4096) and the Horner steps are 32 words.
 * Errors: XG_EINVAL, XG_ERANGE, XG_ENOTSUP (P unavailable), XG_EHIP.  J == 0
 * enqueues nothing. */
xg_status xg_skip(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t J, void *stream);

/* The jump polynomial z^J mod P itself: 4096 coefficients as 64 little-endian
 * 64-bit words in h_g (host memory; bit i of word k is the coefficient of
 * z^(64 k + i)).  Errors: XG_EINVAL (NULL h_g), XG_ENOTSUP. */
xg_status xg_jump_polynomial(uint64_t J, uint64_t *h_g);

/* The same for a family member (XG_FAMILY_*): z^J mod P of that member's
 * x-part, P of degree n = r w, written as n / 64 little-endian words to h_g
 * (host memory of at least n / 64 words).  The library derives each P once
 * per process from its own stepping of the member's recurrence, as the first
 * linear dependency among the states S, T S, ..., T^n S.
 * Errors: XG_EINVAL (NULL h_g, unknown family), XG_ENOTSUP. */
xg_status xg_family_jump_polynomial(uint32_t family, uint64_t J, uint64_t *h_g);

/* ---- batched requests ------------------------------------------------------ */

/* One request: n values of type dtype from stream `stream`'s current
 * position, written at d_out + out_offset (in elements of the handle's word
 * width: 4 bytes, 8 for XG_FAMILY_R64_W64).  flags is 0.  A request reads its
 * stream from where the requests before it on that stream (in table order)
 * leave it, so a batch gives each request the values it would get alone
 * (Section 2: each stream is an independent subsequence; the batch only
 * decides which wavefront serves it and when). */
typedef struct {
    uint64_t stream;
    uint64_t n;
    uint64_t out_offset;
    uint32_t dtype;
    uint32_t flags;
} xg_request;

/* Device scratch of xg_generate_batch on ctx for up to max_reqs requests and
 * up to max_tiles tiles per call (0 if ctx is NULL, max_reqs is 0, or
 * max_reqs + max_tiles > 2^20 or max_tiles > 65536).  It holds the planner's
 * sort keys, prefix sums and queue items, the served table, the start states of
 * tiles and the tile jump table: about 60 B per request plus 530 B per tile
 * (1.1 KB for the 64-bit member) plus 130 KB when tiles are used. */
size_t xg_batch_scratch_bytes(const xg_ctx *ctx, uint32_t max_reqs, uint32_t max_tiles);

/* Gives ctx the device scratch xg_generate_batch works in.
 *   d_scratch   xg_batch_scratch_bytes(ctx, max_reqs, max_tiles) bytes,
 *               256-byte aligned, owned by the caller, used by every later
 *               xg_generate_batch / xg_autotune_batch on ctx (so those calls
 *               must be ordered on one HIP stream); NULL detaches
 *   tile_words  0, or L (a multiple of 64, 2^12 .. 2^30): a stream with a
 *               single request of more than L words (and at most 256 tiles)
 *               is served as tiles of L words run by separate wavefronts,
 *               tile k from the request's start state jumped by k L words
 *               (xg_skip's jump); the values are those of the unsplit request.
 *               Section 2's member only (XG_ENOTSUP otherwise); max_tiles
 *               bounds the tiles of one call (later long requests run whole).
 * With tiles, computes z^(k L) mod P for k = 1 .. 255 on the host and copies
 * them into the scratch on `stream`, then synchronises it.
 * The first 256 bytes of d_scratch are the batch workspace: after a call,
 * ((uint32_t *)d_scratch)[1] is 1 if a request was skipped (stream out of
 * range, bad dtype or flags), else 0.
 * Errors: XG_EINVAL, XG_ERANGE (scratch_bytes too small), XG_EALIGN,
 * XG_ENOTSUP, XG_ENOMEM, XG_EHIP. */
xg_status xg_set_batch_scratch(xg_ctx *ctx, void *d_scratch, size_t scratch_bytes, uint32_t max_reqs,
                               uint32_t max_tiles, uint64_t tile_words, void *stream);

/* Serves num_reqs requests in one call (Section 2: many independent
 * subsequences, one per group of threads).  d_reqs is a table in device memory
 * in the caller's order; same-stream requests are served in that order.  On
 * the device, without a host round trip, the library
 *   - groups the requests by stream (a sort of (stream, index) keys), keeping
 *     table order inside each group;
 *   - splits groups of one long request into tiles (xg_set_batch_scratch);
 *   - orders the queue items (groups and tiles) by cost, largest first;
 *   - serves them in one persistent launch whose wavefronts take items from
 *     an atomic queue.
 * The launch shape is the tuning cache's entry for (this device's
 * architecture, its compute units, the handle's family, tune_key), written
 * by xg_autotune_batch or loaded with xg_tune_cache_load; tune_key NULL or
 * absent from the cache selects the default shape (xg_tune).  Only kernels are
 * enqueued, so the call can be captured in a HIP graph and replayed (each
 * replay serves the table again from the streams' current positions).
 *   d_out   output buffer; every request's [out_offset, out_offset + n) must
 *           lie inside it (the caller's guarantee, as for the plain calls)
 * A request with stream >= num_streams, dtype other than XG_U32 / XG_F32 /
 * XG_NORMAL, or flags != 0 is skipped and sets the scratch's error word.
 * The further members take the same table as for xg_generate_batch_planned.
 * Errors: XG_EINVAL (NULL pointer, no scratch attached), XG_EBUSY (num_reqs
 * above the scratch's max_reqs), XG_EALIGN, XG_EHIP. */
xg_status xg_generate_batch(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs, void *d_out,
                            const char *tune_key, void *stream);

/* Copies the table the last xg_generate_batch on ctx planned into host
 * memory (for inspection and tests), after synchronising `stream`:
 *   h_table    receives *num_entries served entries (at least max_entries):
 *              the requests, grouped by stream in table order; a tile of a
 *              split request appears as a segment entry (flags bit 0 set, bit 1
 *              on its last tile, bits 8..15 the tile number k, bits 16..31 its
 *              start-state slot; n and out_offset cover the tile's values)
 *   h_groups   receives *num_groups + 1 offsets into h_table (at least
 *              max_groups + 1): the queue items in serving order
 * Errors: XG_EINVAL (NULL pointer, no scratch), XG_ERANGE (a buffer too
 * small; the counts are still written), XG_EHIP. */
xg_status xg_batch_read_plan(const xg_ctx *ctx, xg_request *h_table, uint32_t max_entries, uint32_t *h_groups,
                             uint32_t max_groups, uint32_t *num_entries, uint32_t *num_groups, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as xg_generate_batch, with the planner's scratch in a file-scope device
 * array of the library instead of memory attached with xg_set_batch_scratch.
 * It allocates nothing.  The array (XG_STATIC_SCRATCH_BYTES, 5 MiB) is held
 * on each GPU the library runs on until the process ends; its device address
 * is looked up once per GPU, on the first call there.
 *   num_reqs  at most XG_STATIC_MAX_REQS (65536); more gives XG_EBUSY, with
 *             nothing enqueued.  No tiles: long requests run whole.
 *   d_error   NULL, or a device word (caller-owned) that receives 1 if a
 *             request was skipped (as xg_generate_batch's error word), else 0
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * plan: calls that overlap on one GPU (on different HIP streams, or from
 * host threads without ordering) race and must not be made.
 * Errors: XG_EINVAL (NULL pointer, handle of another device, malformed
 * tune_key), XG_EBUSY, XG_EALIGN, XG_ENOTSUP, XG_EHIP. */
#define XG_STATIC_MAX_REQS      65536u
#define XG_STATIC_SCRATCH_BYTES (5u << 20)
xg_status xg_generate_batch_static(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs, void *d_out,
                                   const char *tune_key, uint32_t *d_error, void *stream);

/* Device workspace of xg_generate_batch_planned: a work counter, an error
 * word and the table's counts (256 B). */
size_t xg_batch_workspace_bytes(void);

/* Orders a request table on the host, as xg_generate_batch does on the device
 * (without tiles), for callers that plan on the host.
 *   h_reqs      num_reqs requests (host)
 *   h_sorted    receives the ordered requests (host, num_reqs entries)
 *   h_groups    receives num_groups + 1 offsets into h_sorted (host, at least
 *               num_reqs + 1 entries); group g is h_sorted[h_groups[g] ..
 *               h_groups[g + 1])
 *   num_groups  receives the number of groups
 *   num_streams requests must name streams below this
 *   out_elems   capacity of the output buffer in elements: every request's
 *               [out_offset, out_offset + n) must fit
 * Errors: XG_EINVAL (NULL pointer, dtype or flags invalid), XG_ERANGE (stream
 * or output range out of bounds), XG_ENOMEM. */
xg_status xg_plan_batch(const xg_request *h_reqs, uint32_t num_reqs, uint64_t num_streams,
                        uint64_t out_elems, xg_request *h_sorted, uint32_t *h_groups,
                        uint32_t *num_groups);

/* Serves a table planned by xg_plan_batch in one persistent launch (preceded
 * by a small kernel that fills the workspace, so the pair can be captured in a
 * HIP graph and replayed).  Wavefronts take groups from a device-side atomic
 * queue.
 *   d_reqs, d_groups  device copies of xg_plan_batch's output (num_reqs
 *                     requests, num_groups + 1 offsets)
 *   num_groups        groups in the table
 *   d_out             output buffer of out_elems elements
 *   tune              launch shape (NULL: the default shape for num_groups
 *                     groups, xg_tune)
 *   d_work            xg_batch_workspace_bytes() bytes of device memory
 * A request or group that fails the device-side bounds check (stream, dtype,
 * output range, group offsets) is skipped and sets the error word
 * (((uint32_t *)d_work)[1]) to 1; every wavefront still reaches the exit.
 * The further members (XG_FAMILY_R64_W32, XG_FAMILY_R64_W64) take the same
 * table: dtype XG_U32 gives the member's unsigned words (uint32 / uint64),
 * XG_F32 its uniform reals (FP32 / FP64, as xg_generate_f32 / xg_generate_f64)
 * and XG_NORMAL its normals (FP32 as xg_generate_normal / FP64 as
 * xg_generate_normal_f64), each in elements of the word width.  One wavefront
 * serves two groups, one per half, stepping through both current requests
 * together (a half waits while its request has another dtype); store_words of
 * tune is not used, and d_out must be 8-byte aligned for the 64-bit member.
 * Errors: XG_EINVAL, XG_ERANGE, XG_EALIGN, XG_EHIP. */
xg_status xg_generate_batch_planned(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs,
                                    const uint32_t *d_groups, uint32_t num_groups, void *d_out,
                                    uint64_t out_elems, const xg_tune *tune, void *d_work, void *stream);

/* Times candidate launch shapes of xg_generate_batch on the given table
 * (array order, as for xg_generate_batch) and returns the fastest in *best:
 * first the median of `reps` timed runs per shape after one warm-up, then the
 * 8 fastest of those timed 5 more times each, in turns, the best median of
 * these winning (their records in times_ms carry it).  The table is
 * planned once in ctx's batch scratch; each run times the persistent launch
 * (with the tiles' start states) on a scratch copy of the state:
 *   d_scratch_state  xg_family_state_bytes(family, num_streams of ctx) bytes,
 *                    overwritten
 *   d_scratch_out    as large as the requests' outputs need, overwritten
 * so the streams of ctx do not advance.  With tune_key non-NULL the best shape
 * is stored in the tuning cache under (device architecture, compute units,
 * family, tune_key), where xg_generate_batch looks it up.  Synchronises
 * `stream`.  times_ms, if non-NULL, receives up to max_times (shape, time)
 * records as consecutive groups of 5 floats: waves_per_block, unroll,
 * blocks_per_cu, ms, store_words.  *num_times receives their count.
 * Errors: those of xg_generate_batch, XG_EINVAL (tune_key not a valid key). */
xg_status xg_autotune_batch(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs, void *d_scratch_out,
                            void *d_scratch_state, const char *tune_key, int reps, xg_tune *best,
                            float *times_ms, uint32_t max_times, uint32_t *num_times, void *stream);

/* ---- tuning cache ------------------------------------------------------------ */

/* Batch launch shapes keyed by (arch, cus, family, tune_key): the device
 * architecture name without feature suffixes (e.g. "gfx950"), its compute
 * units, the family member, and the caller's name of the workload signature
 * and its output types (e.g. "ragged65536/u32").  Keys are 1 .. 256
 * printable characters without '"' or '\'.  The cache lives in the process
 * and is thread-safe; the file named by the environment variable
 * XG_TUNE_CACHE, if any, is merged in before the first lookup.
 * File format (JSON): {"xg_tune_cache": 1, "entries": [{"arch": ..., "key":
 * ..., "cus": ..., "family": ..., "waves_per_block": ..., "unroll": ...,
 * "blocks_per_cu": ..., "store_words": ..., "ms": ...}, ...]}. */

/* Merges the entries of a cache file (later entries replace equal keys).
 * Errors: XG_EINVAL (unreadable, or not a valid cache file: then nothing is
 * merged), XG_ENOMEM. */
xg_status xg_tune_cache_load(const char *path);

/* Writes every entry to path (through a temporary file renamed into place).
 * Errors: XG_EINVAL (cannot write), XG_ENOMEM. */
xg_status xg_tune_cache_save(const char *path);

/* Stores a shape (and its measured ms, or NaN) under a key.
 * Errors: XG_EINVAL (bad key, cus 0, unknown family, shape out of range). */
xg_status xg_tune_cache_put(const char *arch, uint32_t cus, uint32_t family, const char *tune_key,
                            const xg_tune *tune, float ms);

/* Looks a key up; *ms (if non-NULL) receives its time, or -1.
 * Errors: XG_EINVAL (bad key or NULL tune), XG_ERANGE (no such entry). */
xg_status xg_tune_cache_get(const char *arch, uint32_t cus, uint32_t family, const char *tune_key,
                            xg_tune *tune, float *ms);

/* Number of entries; and removal of all of them. */
uint32_t xg_tune_cache_size(void);
void xg_tune_cache_clear(void);

/* The (arch, cus) part of the key under which calls on ctx look shapes up:
 * arch receives the architecture name (NUL-terminated, at most arch_len
 * bytes with the NUL).  Errors: XG_EINVAL (NULL or arch_len too small). */
xg_status xg_tune_identity(const xg_ctx *ctx, char *arch, size_t arch_len, uint32_t *cus);

/* ---- serving: continuous batching over device-resident streams ------------- */

/* A request server over the streams of one handle.  Requests (stream, n,
 * dtype) are submitted from the host; xg_server_poll reaps finished batches,
 * admits pending requests in arrival order as output memory and streams free
 * up, and launches each admitted set as one persistent batched launch
 * (xg_generate_batch's kernel) on one of num_lanes HIP streams, so batches that
 * arrive while others run overlap on the device.  A request reads its stream
 * from the position the stream has when it is admitted; requests on one stream
 * are served in submission order and never run in two batches at once, so a
 * request's values equal those of the same request run alone from that
 * position.  Outputs live in a caller-provided device pool until released.
 * Not thread-safe: one host thread drives a server. */
typedef struct xg_server xg_server;

typedef struct {
    uint32_t num_lanes;   /* HIP streams, each with at most one batch in flight: 1 .. 8 */
    uint32_t max_batch;   /* table entries per batch (requests and segments): 1 .. 65536 */
    xg_tune tune;         /* batch launch shape; all zero: the tuning cache's entry for
                             tune_key if there is one, else each batch's default
                             (xg_tune) */
    uint64_t segment_words; /* 0, or L (a multiple of 64, 2^12 .. 2^30): a request of more
                               than L words is served as up to 256 segments of L words run
                               by separate wavefronts, segment k starting from the request's
                               start state jumped by k L words (xg_skip's jump); the values
                               are those of the unsplit request */
    const char *tune_key; /* NULL, or a tuning-cache key (see xg_tune_cache_get) looked up
                             at creation when tune is all zero */
} xg_server_config;

typedef struct {
    uint64_t id;          /* the caller's request id */
    uint64_t stream;
    uint64_t n;
    uint64_t out_offset;  /* element offset of the output in the pool */
    uint64_t start_pos;   /* stream position the request read from */
    uint64_t t_submit_ns; /* host steady-clock times (ns) of submission, launch and */
    uint64_t t_launch_ns; /* of the poll that saw the batch finish */
    uint64_t t_done_ns;
    uint32_t dtype;
    uint32_t lane;
} xg_completion;

typedef struct {
    uint64_t submitted, completed, batches, admitted;
    uint64_t max_lanes_busy;     /* most batches observed in flight at once */
    uint64_t max_batch_seen;     /* most requests in one batch */
    uint64_t pool_high_water;    /* most pool elements in use at once */
    uint64_t admission_waits;    /* polls where the oldest request waited for pool memory */
} xg_server_stats;

/* Device bytes of request tables and workspaces a server needs. */
size_t xg_server_device_bytes(const xg_server_config *cfg);

/* Creates a server.  d_pool (pool_elems >= 64 elements of the handle's word
 * width, 4 or 8 bytes; 256-byte aligned) holds request outputs: the server
 * hands out 64-element-aligned
 * ranges of its first floor(pool_elems / 64) * 64 elements.  d_tables
 * (xg_server_device_bytes(cfg) bytes, 256-byte aligned) holds request tables.
 * Both stay owned by the caller.  Creates num_lanes HIP streams (default
 * priority) and pinned host staging; synchronises the device once and reads
 * the streams' positions.  The server keeps those positions on the host, so
 * while it exists no other call may advance the streams of ctx.  The further
 * members (XG_FAMILY_R64_W32, XG_FAMILY_R64_W64) are served through their
 * batch kernel and only with segment_words 0 (otherwise XG_ENOTSUP).
 * Errors: XG_EINVAL (among others pool_elems < 64), XG_ERANGE (a buffer too
 * small), XG_EALIGN, XG_ENOMEM, XG_ENOTSUP, XG_EHIP. */
xg_status xg_server_create(xg_server **out, xg_ctx *ctx, const xg_server_config *cfg,
                           void *d_pool, uint64_t pool_elems, void *d_tables, size_t tables_bytes);

/* Queues a request of n >= 1 values under the caller's tag id, which must not
 * belong to a request still pending, in flight, or completed and not yet
 * released.  Errors: XG_EINVAL (NULL server, n == 0, bad dtype, id in use),
 * XG_ERANGE (stream out of range, or n rounded up to a multiple of 64 larger
 * than the usable pool: such a request could never be admitted). */
xg_status xg_server_submit(xg_server *srv, uint64_t id, uint64_t stream, uint64_t n, uint32_t dtype);

/* Makes progress without blocking: reaps finished batches, admits and
 * launches, and returns up to max_out completions (more wait for the next
 * poll).  Errors: XG_EINVAL (bad arguments; nothing changes), XG_EHIP,
 * XG_ENOMEM.  A poll that fails with XG_EHIP or XG_ENOMEM (or with any other
 * status once it has started moving requests) leaves the server failed: the
 * streams of ctx may have been partly advanced, and every later submit, poll
 * and release returns that status.  Only xg_server_destroy (and the counters)
 * remain; outputs of requests already handed out stay valid. */
xg_status xg_server_poll(xg_server *srv, xg_completion *out, uint32_t max_out, uint32_t *num_out);

/* Returns a completed request's output to the pool.  Errors: XG_EINVAL
 * (unknown or unfinished id). */
xg_status xg_server_release(xg_server *srv, uint64_t id);

/* Requests submitted but not yet completed. */
uint64_t xg_server_outstanding(const xg_server *srv);

xg_status xg_server_get_stats(const xg_server *srv, xg_server_stats *out);

/* The launch shape the server's batches use (all zero: each batch's default).
 * Errors: XG_EINVAL (NULL). */
xg_status xg_server_get_tune(const xg_server *srv, xg_tune *out);

/* Waits for in-flight batches, then frees the server's host resources and
 * streams (never the caller's buffers).  NULL is accepted. */
void xg_server_destroy(xg_server *srv);

/* Write-only reference for the generators' store path: d_out[0 .. words)
 * receive `value`, written with 16-byte stores, each 256-thread block one
 * contiguous 4 KB piece in dispatch order.  It generates nothing; its
 * bandwidth is the practical HBM write ceiling the benchmark reports the
 * generators against.  d_out must be 16-byte aligned.  words == 0 enqueues
 * nothing.  Errors: XG_EINVAL (NULL), XG_ERANGE, XG_EALIGN, XG_ENOTSUP,
 * XG_EHIP. */
xg_status xg_fill_value(void *d_out, uint64_t words, uint32_t value, void *stream);

/* Human-readable name of a status. */
const char *xg_strerror(xg_status status);

#ifdef __cplusplus
}
#endif

#endif /* XG_H */
