// C-ABI layer of libxg (include/xg.h): argument validation, stream handles,
// the host-side batch planner and the batch autotuner.  Every generating call
// validates synchronously, then only enqueues kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <unordered_map>
#include <vector>

#include "xg.h"
#include "xg_internal.h"
#include "xg_fam_batch.h"

namespace {

constexpr uint64_t kMaxStreams = 0xFFFFFFFFull;

xg_status current_gfx950(int *device, int *num_cus) {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return XG_EHIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, d) != hipSuccess) return XG_EHIP;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return XG_ENOTSUP;
  *device = d;
  *num_cus = prop.multiProcessorCount;
  return XG_OK;
}

xg_status make_ctx(xg_ctx **out, void *d_state, size_t state_bytes, uint64_t num_streams,
                   uint32_t family = XG_FAMILY_R128_W32) {
  if (!out) return XG_EINVAL;
  *out = nullptr;
  const uint32_t per_stream = xg::family_state_bytes(family);
  if (!d_state || num_streams == 0 || num_streams > kMaxStreams || per_stream == 0) return XG_EINVAL;
  if (state_bytes / per_stream < num_streams) return XG_ERANGE;
  if (reinterpret_cast<uintptr_t>(d_state) % 16 != 0) return XG_EALIGN;
  int dev = 0, cus = 0;
  const xg_status st = current_gfx950(&dev, &cus);
  if (st != XG_OK) return st;
  xg_ctx *c = new (std::nothrow) xg_ctx;
  if (!c) return XG_ENOMEM;
  c->d_state = static_cast<uint32_t *>(d_state);
  c->num_streams = num_streams;
  c->device = dev;
  c->num_cus = cus;
  c->plain = xg::kDefaultPlain;
  c->family = family;
  *out = c;
  return XG_OK;
}

xg_status check_ctx_device(const xg_ctx *ctx) {
  int d = -1;
  if (hipGetDevice(&d) != hipSuccess) return XG_EHIP;
  return d == ctx->device ? XG_OK : XG_EINVAL;
}

// Validates a plain launch over streams [first, first + count) with
// per_stream_elems elements of elem_bytes each (out may be NULL when n == 0).
xg_status check_range(const xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n,
                      const void *out, uint64_t per_stream_elems, uint32_t elem_bytes = 4) {
  if (!ctx || count == 0) return XG_EINVAL;
  if (first > ctx->num_streams || count > ctx->num_streams - first) return XG_ERANGE;
  if (n == 0) return XG_OK;
  if (!out) return XG_EINVAL;
  if (count > (UINT64_MAX / elem_bytes) / per_stream_elems) return XG_ERANGE;
  if (reinterpret_cast<uintptr_t>(out) % elem_bytes != 0) return XG_EALIGN;
  return check_ctx_device(ctx);
}

// Calls that only Section 2's member supports.
bool paper_member(const xg_ctx *ctx) { return ctx && ctx->family == XG_FAMILY_R128_W32; }

// The plain shape with an automatic waves_per_block and unroll resolved for
// this launch (the further members run two streams per wavefront).  The
// 64-bit member takes one wavefront per block: measured ~10 % faster than four
// for its bulk fill and equal for stream-major, where the 32-bit kernels want
// four.  The automatic unroll (interleaved A/B runs over several boxes,
// 1024 streams x 2^20 words) is, for Section 2's member:
//  - uint32 bulk fill: 4 (at 8 it ran 700-770 us per 4 GiB on some boxes,
//    at 4 600-640 us everywhere);
//  - FP32 bulk fill: 8 (4-5 % faster than 4);
//  - uint32 / FP32 stream-major: 2 with 4-byte stores (FP32 710-735 us
//    against 780-815 us for unroll 8 with 16-byte stores; uint32 with its
//    stores paced, see the kernels, 717-736 us);
//  - normals and moments: 8.
// For the 32-bit r = 64 member (2048 streams, 1024 wavefronts) stream-major
// uint32 / FP32 take 2 as well (u32 764-779 us against 828 us, f32 740-754
// against 789-812 us, three boxes); its fills keep 8.
// Those were measured with a wavefront on every SIMD; smaller launches (fewer
// than 4 x CUs wavefronts, e.g. one stream per launch) keep unroll 8, as does
// the 64-bit member.
xg::Shape plain_shape(const xg_ctx *ctx, uint64_t count, xg::Kind kind, bool fill_layout) {
  xg::Shape s = ctx->plain;
  const uint64_t waves = ctx->family == XG_FAMILY_R128_W32 ? count : (count + 1) / 2;
  if (s.waves_per_block == 0)
    s.waves_per_block = ctx->family == XG_FAMILY_R64_W64 ? 1u : xg::auto_waves_per_block(waves, ctx->num_cus);
  if (s.unroll == 0) {
    s.unroll = 8;
    const bool every_simd = waves >= 4 * (uint64_t)(ctx->num_cus > 0 ? ctx->num_cus : 1);
    if (ctx->family == XG_FAMILY_R128_W32 && every_simd && (kind == xg::kU32 || kind == xg::kF32)) {
      if (fill_layout) {
        s.unroll = kind == xg::kU32 ? 4u : 8u;
      } else {
        s.unroll = 2;
        s.store_words = 1;
      }
    } else if (ctx->family == XG_FAMILY_R64_W32 && every_simd && !fill_layout &&
               (kind == xg::kU32 || kind == xg::kF32)) {
      s.unroll = 2;
    }
  }
  return s;
}

// u32 / f32 (and u64 / f64) of the further members, both layouts.
xg_status family_words(xg_ctx *ctx, xg::Kind kind, bool fill_layout, uint64_t first, uint64_t count, uint64_t n,
                       void *out, void *stream) {
  const bool w64 = kind == xg::kU64 || kind == xg::kF64;
  if (!ctx) return XG_EINVAL;
  if (ctx->family != (w64 ? XG_FAMILY_R64_W64 : XG_FAMILY_R64_W32)) return XG_ENOTSUP;
  xg_status st = check_range(ctx, first, count, n, out, n, w64 ? 8 : 4);
  if (st != XG_OK || n == 0) return st;
  const hipError_t e = xg::launch_family_generate(ctx->family, kind, fill_layout, plain_shape(ctx, count, kind, fill_layout),
                                                  reinterpret_cast<unsigned char *>(ctx->d_state), first, count,
                                                  n, out, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

xg_status plain(xg_ctx *ctx, xg::Kind kind, uint64_t first, uint64_t count, uint64_t n, void *out,
                void *stream) {
  if (ctx && ctx->family == XG_FAMILY_R64_W32) {
    if (kind == xg::kU32 || kind == xg::kF32) return family_words(ctx, kind, false, first, count, n, out, stream);
    // normals and their fused moments (kNormal, kMoments)
    xg_status st = check_range(ctx, first, count, n, out, kind == xg::kMoments ? 2 : n);
    if (st != XG_OK || n == 0) return st;
    const hipError_t e = xg::launch_family_generate(ctx->family, kind, false, plain_shape(ctx, count, kind, false),
                                                    reinterpret_cast<unsigned char *>(ctx->d_state), first, count,
                                                    n, out, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? XG_OK : XG_EHIP;
  }
  if (ctx && !paper_member(ctx)) return XG_ENOTSUP;
  const uint64_t per_stream = kind == xg::kMoments ? 2 : n;
  xg_status st = check_range(ctx, first, count, n, out, per_stream);
  if (st != XG_OK || n == 0) return st;
  const hipError_t e = xg::launch_generate(kind, plain_shape(ctx, count, kind, false), ctx->d_state, first, count,
                                           n, out, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

xg_status fill(xg_ctx *ctx, xg::Kind kind, uint64_t first, uint64_t count, uint64_t n, void *out,
               void *stream) {
  if (ctx && ctx->family == XG_FAMILY_R64_W32) return family_words(ctx, kind, true, first, count, n, out, stream);
  if (ctx && !paper_member(ctx)) return XG_ENOTSUP;
  xg_status st = check_range(ctx, first, count, n, out, n);
  if (st != XG_OK || n == 0) return st;
  const hipError_t e = xg::launch_fill(kind, plain_shape(ctx, count, kind, true), ctx->d_state, first, count, n,
                                       static_cast<uint32_t *>(out), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

// FP64 normals (kNormal: n doubles per stream) or their fused sums
// (kMoments: 2 doubles per stream) of the 64-bit member.
xg_status normals_f64(xg_ctx *ctx, xg::Kind kind, uint64_t first, uint64_t count, uint64_t n, double *d_out,
                      void *stream) {
  if (!ctx) return XG_EINVAL;
  if (ctx->family != XG_FAMILY_R64_W64) return XG_ENOTSUP;
  const xg_status st = check_range(ctx, first, count, n, d_out, kind == xg::kMoments ? 2 : n, 8);
  if (st != XG_OK || n == 0) return st;
  const hipError_t e = xg::launch_family_generate(ctx->family, kind, false, plain_shape(ctx, count, kind, false),
                                                  reinterpret_cast<unsigned char *>(ctx->d_state), first, count,
                                                  n, d_out, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

bool tune_to_shape(const xg_tune *t, uint32_t blocks_per_cu, xg::Shape *s) {
  if (!t) return false;
  const uint32_t sw = t->store_words ? t->store_words : (t->unroll >= 4 ? 4u : 1u);
  *s = xg::Shape{t->waves_per_block, t->unroll, blocks_per_cu, sw};
  return xg::shape_valid(*s);
}

}  // namespace


extern "C" {

size_t xg_state_bytes(uint64_t num_streams) {
  if (num_streams > kMaxStreams) return 0;
  return (size_t)num_streams * XG_STATE_WORDS * 4;
}

xg_status xg_init_streams(xg_ctx **out, void *d_state, size_t state_bytes, uint64_t num_streams,
                          uint64_t seed, void *stream) {
  xg_status st = make_ctx(out, d_state, state_bytes, num_streams);
  if (st != XG_OK) return st;
  const hipError_t e = xg::launch_init((*out)->d_state, num_streams, seed, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    delete *out;
    *out = nullptr;
    return XG_EHIP;
  }
  return XG_OK;
}

xg_status xg_attach_streams(xg_ctx **out, void *d_state, size_t state_bytes, uint64_t num_streams) {
  return make_ctx(out, d_state, state_bytes, num_streams);
}

size_t xg_family_state_bytes(uint32_t family, uint64_t num_streams) {
  if (num_streams > kMaxStreams) return 0;
  return (size_t)num_streams * xg::family_state_bytes(family);
}

xg_status xg_init_family(xg_ctx **out, uint32_t family, void *d_state, size_t state_bytes, uint64_t num_streams,
                         uint64_t seed, void *stream) {
  if (family == XG_FAMILY_R128_W32) return xg_init_streams(out, d_state, state_bytes, num_streams, seed, stream);
  xg_status st = make_ctx(out, d_state, state_bytes, num_streams, family);
  if (st != XG_OK) return st;
  const hipError_t e = xg::launch_family_init(family, reinterpret_cast<unsigned char *>(d_state), num_streams,
                                              seed, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    delete *out;
    *out = nullptr;
    return XG_EHIP;
  }
  return XG_OK;
}

xg_status xg_attach_family(xg_ctx **out, uint32_t family, void *d_state, size_t state_bytes,
                           uint64_t num_streams) {
  return make_ctx(out, d_state, state_bytes, num_streams, family);
}

uint32_t xg_family(const xg_ctx *ctx) { return ctx ? ctx->family : UINT32_MAX; }

void xg_destroy(xg_ctx *ctx) { delete ctx; }

uint64_t xg_num_streams(const xg_ctx *ctx) { return ctx ? ctx->num_streams : 0; }

void *xg_state_ptr(const xg_ctx *ctx) { return ctx ? ctx->d_state : nullptr; }

xg_status xg_set_plain_tune(xg_ctx *ctx, const xg_tune *tune) {
  if (!ctx || !tune) return XG_EINVAL;
  xg_tune t = *tune;
  const bool auto_wpb = t.waves_per_block == 0, auto_unroll = t.unroll == 0;
  if (auto_wpb) t.waves_per_block = 1;  // validate the other fields
  if (auto_unroll) t.unroll = 8;
  xg::Shape s;
  if (!tune_to_shape(&t, 1, &s)) return XG_EINVAL;
  if (auto_wpb) s.waves_per_block = 0;
  if (auto_unroll) s.unroll = 0;
  ctx->plain = s;
  return XG_OK;
}

xg_status xg_get_plain_tune(const xg_ctx *ctx, xg_tune *tune) {
  if (!ctx || !tune) return XG_EINVAL;
  tune->waves_per_block = ctx->plain.waves_per_block;
  tune->unroll = ctx->plain.unroll;
  tune->blocks_per_cu = 1;
  tune->store_words = ctx->plain.store_words;
  return XG_OK;
}

xg_status xg_generate_u32(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, uint32_t *d_out,
                          void *stream) {
  return plain(ctx, xg::kU32, first, count, n, d_out, stream);
}

xg_status xg_generate_f32(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, float *d_out,
                          void *stream) {
  return plain(ctx, xg::kF32, first, count, n, d_out, stream);
}

xg_status xg_generate_normal(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, float *d_out,
                             void *stream) {
  return plain(ctx, xg::kNormal, first, count, n, d_out, stream);
}

xg_status xg_normal_moments(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, float *d_sums,
                            void *stream) {
  return plain(ctx, xg::kMoments, first, count, n, d_sums, stream);
}

xg_status xg_fill_u32(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, uint32_t *d_out,
                      void *stream) {
  return fill(ctx, xg::kU32, first, count, n, d_out, stream);
}

xg_status xg_fill_f32(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, float *d_out,
                      void *stream) {
  return fill(ctx, xg::kF32, first, count, n, d_out, stream);
}

xg_status xg_generate_u64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, uint64_t *d_out,
                          void *stream) {
  return family_words(ctx, xg::kU64, false, first, count, n, d_out, stream);
}

xg_status xg_generate_f64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, double *d_out,
                          void *stream) {
  return family_words(ctx, xg::kF64, false, first, count, n, d_out, stream);
}

xg_status xg_fill_u64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, uint64_t *d_out, void *stream) {
  return family_words(ctx, xg::kU64, true, first, count, n, d_out, stream);
}

xg_status xg_fill_f64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, double *d_out, void *stream) {
  return family_words(ctx, xg::kF64, true, first, count, n, d_out, stream);
}

xg_status xg_generate_normal_f64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, double *d_out,
                                 void *stream) {
  return normals_f64(ctx, xg::kNormal, first, count, n, d_out, stream);
}

xg_status xg_normal_moments_f64(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t n, double *d_sums,
                                void *stream) {
  return normals_f64(ctx, xg::kMoments, first, count, n, d_sums, stream);
}

xg_status xg_skip(xg_ctx *ctx, uint64_t first, uint64_t count, uint64_t J, void *stream) {
  if (!ctx || count == 0) return XG_EINVAL;
  if (first > ctx->num_streams || count > ctx->num_streams - first) return XG_ERANGE;
  xg_status st = check_ctx_device(ctx);
  if (st != XG_OK || J == 0) return st;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const bool step = J < xg::kJumpThreshold;
  xg::JumpPoly g{};
  if (!step && !xg::jump_polynomial(ctx->family, J, g.w)) return XG_ENOTSUP;
  hipError_t e;
  if (paper_member(ctx))
    e = xg::launch_skip(ctx->d_state, first, count, J, step ? nullptr : &g, s);
  else
    e = xg::launch_family_skip(ctx->family, reinterpret_cast<unsigned char *>(ctx->d_state), first, count, J,
                               step ? nullptr : &g, s);
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

xg_status xg_fill_value(void *d_out, uint64_t words, uint32_t value, void *stream) {
  if (words == 0) return XG_OK;
  if (!d_out) return XG_EINVAL;
  if (words > UINT64_MAX / 4) return XG_ERANGE;
  if (reinterpret_cast<uintptr_t>(d_out) % 16 != 0) return XG_EALIGN;
  int dev = 0, cus = 0;
  const xg_status st = current_gfx950(&dev, &cus);
  if (st != XG_OK) return st;
  const hipError_t e = xg::launch_fill_value(static_cast<uint32_t *>(d_out), words, value, cus,
                                             static_cast<hipStream_t>(stream));
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

xg_status xg_box_muller(const uint32_t *d_words, uint64_t pairs, float *d_out, void *stream) {
  if (pairs == 0) return XG_OK;
  if (!d_words || !d_out) return XG_EINVAL;
  if (pairs > (UINT64_MAX / 16) || pairs / 256 >= 0xFFFFFFFFull) return XG_ERANGE;
  if (reinterpret_cast<uintptr_t>(d_words) % 4 || reinterpret_cast<uintptr_t>(d_out) % 4) return XG_EALIGN;
  return xg::launch_box_muller(d_words, pairs, d_out, static_cast<hipStream_t>(stream)) == hipSuccess ? XG_OK
                                                                                                      : XG_EHIP;
}

xg_status xg_jump_polynomial(uint64_t J, uint64_t *h_g) {
  if (!h_g) return XG_EINVAL;
  return xg::jump_polynomial(J, h_g) ? XG_OK : XG_ENOTSUP;
}

xg_status xg_family_jump_polynomial(uint32_t family, uint64_t J, uint64_t *h_g) {
  if (!h_g || family > XG_FAMILY_R64_W64) return XG_EINVAL;
  return xg::jump_polynomial(family, J, h_g) ? XG_OK : XG_ENOTSUP;
}

size_t xg_batch_workspace_bytes(void) { return 256; }

xg_status xg_generate_batch(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs,
                            const uint32_t *d_groups, uint32_t num_groups, void *d_out,
                            uint64_t out_elems, const xg_tune *tune, void *d_work, void *stream) {
  if (!ctx || !d_reqs || !d_groups || !d_out || !d_work) return XG_EINVAL;
  const bool member = !paper_member(ctx);
  if (member && ctx->family != XG_FAMILY_R64_W32 && ctx->family != XG_FAMILY_R64_W64) return XG_ENOTSUP;
  if (num_groups > num_reqs) return XG_ERANGE;
  const uintptr_t out_align = ctx->family == XG_FAMILY_R64_W64 ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(d_reqs) % 8 || reinterpret_cast<uintptr_t>(d_groups) % 4 ||
      reinterpret_cast<uintptr_t>(d_out) % out_align || reinterpret_cast<uintptr_t>(d_work) % 4)
    return XG_EALIGN;
  xg::Shape shape = xg::kDefaultBatch;
  if (tune && !tune_to_shape(tune, tune->blocks_per_cu, &shape)) return XG_EINVAL;
  xg_status st = check_ctx_device(ctx);
  if (st != XG_OK) return st;
  if (num_groups == 0) return XG_OK;
  if (member) {
    const hipError_t e = xg::launch_family_batch(ctx->family, shape, ctx->num_cus,
                                                 reinterpret_cast<unsigned char *>(ctx->d_state), ctx->num_streams,
                                                 d_reqs, num_reqs, d_groups, num_groups, d_out, out_elems,
                                                 static_cast<uint32_t *>(d_work), static_cast<hipStream_t>(stream));
    return e == hipSuccess ? XG_OK : XG_EHIP;
  }
  const hipError_t e = xg::launch_batch(shape, ctx->num_cus, ctx->d_state, ctx->num_streams, d_reqs,
                                        num_reqs, d_groups, num_groups,
                                        static_cast<uint32_t *>(d_out), out_elems,
                                        static_cast<uint32_t *>(d_work),
                                        static_cast<hipStream_t>(stream));
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

constexpr int kMaxReps = 100;  // timed repetitions per candidate shape

xg_status xg_autotune_batch(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs,
                            const uint32_t *d_groups, uint32_t num_groups, void *d_scratch_out,
                            uint64_t out_elems, void *d_scratch_state, void *d_work, int reps,
                            xg_tune *best, float *times_ms, uint32_t max_times,
                            uint32_t *num_times, void *stream) {
  if (!ctx || !best || !d_scratch_state || reps < 1 || reps > kMaxReps) return XG_EINVAL;
  const bool member = !paper_member(ctx);
  if (member && ctx->family != XG_FAMILY_R64_W32 && ctx->family != XG_FAMILY_R64_W64) return XG_ENOTSUP;
  if (num_times) *num_times = 0;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t state_bytes = xg_family_state_bytes(ctx->family, ctx->num_streams);
  xg_ctx scratch = *ctx;
  scratch.d_state = static_cast<uint32_t *>(d_scratch_state);
  if (reinterpret_cast<uintptr_t>(d_scratch_state) % 16) return XG_EALIGN;

  static const uint32_t kWpb[] = {1, 2, 4, 8, 16};
  static const uint32_t kUnroll[] = {1, 2, 4, 8};
  static const uint32_t kBpc[] = {1, 2, 4, 8, 16, 32};
  static const uint32_t kStoreWords[] = {1, 4};
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return XG_EHIP;
  }
  float best_ms = -1.f;
  xg_status result = XG_OK;
  uint32_t recorded = 0;
  for (uint32_t wpb : kWpb) {
    for (uint32_t un : kUnroll) {
      for (uint32_t bpc : kBpc) {
        for (uint32_t sw : kStoreWords) {
          if (wpb * bpc > 32) continue;  // more waves than a compute unit holds
          if (sw == 4 && (un < 4 || member)) continue;  // the members' batch kernel has no wide stores
          const xg_tune cand{wpb, un, bpc, sw};
          float ms[kMaxReps];
          int nms = 0;
          for (int rep = 0; rep <= reps && result == XG_OK; ++rep) {
            if (hipMemcpyAsync(d_scratch_state, ctx->d_state, state_bytes, hipMemcpyDeviceToDevice, s) !=
                hipSuccess) {
              result = XG_EHIP;
              break;
            }
            if (hipEventRecord(t0, s) != hipSuccess) { result = XG_EHIP; break; }
            result = xg_generate_batch(&scratch, d_reqs, num_reqs, d_groups, num_groups, d_scratch_out,
                                       out_elems, &cand, d_work, stream);
            if (result != XG_OK) break;
            if (hipEventRecord(t1, s) != hipSuccess || hipEventSynchronize(t1) != hipSuccess) {
              result = XG_EHIP;
              break;
            }
            float t = 0.f;
            if (hipEventElapsedTime(&t, t0, t1) != hipSuccess) { result = XG_EHIP; break; }
            if (rep > 0) ms[nms++] = t;  // rep 0 is the warm-up
          }
          if (result != XG_OK) break;
          std::sort(ms, ms + nms);
          const float med = ms[nms / 2];
          if (times_ms && recorded < max_times) {
            float *rec = times_ms + 5 * recorded;
            rec[0] = (float)wpb; rec[1] = (float)un; rec[2] = (float)bpc; rec[3] = med; rec[4] = (float)sw;
            ++recorded;
          }
          if (best_ms < 0.f || med < best_ms) {
            best_ms = med;
            *best = cand;
          }
        }
        if (result != XG_OK) break;
      }
      if (result != XG_OK) break;
    }
    if (result != XG_OK) break;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (num_times) *num_times = recorded;
  return result;
}

const char *xg_strerror(xg_status status) {
  switch (status) {
    case XG_OK: return "ok";
    case XG_EINVAL: return "invalid argument";
    case XG_ERANGE: return "stream or size out of range";
    case XG_EALIGN: return "misaligned device pointer";
    case XG_EHIP: return "HIP runtime error";
    case XG_ENOTSUP: return "current device is not gfx950";
    case XG_ENOMEM: return "host allocation failed";
    case XG_EBUSY: return "workspace too small";
    default: return "unknown status";
  }
}

}  // extern "C"
