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

xg_status current_gfx950(int *device, int *num_cus, char *arch = nullptr, size_t arch_len = 0) {
  int d = 0;
  if (hipGetDevice(&d) != hipSuccess) return XG_EHIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, d) != hipSuccess) return XG_EHIP;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return XG_ENOTSUP;
  *device = d;
  *num_cus = prop.multiProcessorCount;
  if (arch && arch_len) {  // the name up to its first ':' (feature suffixes)
    size_t i = 0;
    for (; i + 1 < arch_len && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i) arch[i] = prop.gcnArchName[i];
    arch[i] = '\0';
  }
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
  char arch[sizeof(xg_ctx::arch)];
  const xg_status st = current_gfx950(&dev, &cus, arch, sizeof arch);
  if (st != XG_OK) return st;
  // The static batch scratch's address on this device, set up before any
  // caller can be capturing a graph (a failure surfaces in that call).
  (void)xg::static_scratch_prepare(dev);
  xg_ctx *c = new (std::nothrow) xg_ctx{};
  if (!c) return XG_ENOMEM;
  c->d_state = static_cast<uint32_t *>(d_state);
  c->num_streams = num_streams;
  c->device = dev;
  c->num_cus = cus;
  std::memcpy(c->arch, arch, sizeof arch);
  c->plain = xg::kDefaultPlain;
  c->family = family;
  c->d_batch = nullptr;
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
                                           n, out, ctx->num_cus, static_cast<hipStream_t>(stream));
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

// Families with a batch kernel.
bool batch_member(const xg_ctx *ctx) {
  return ctx->family == XG_FAMILY_R128_W32 || ctx->family == XG_FAMILY_R64_W32 || ctx->family == XG_FAMILY_R64_W64;
}

// Tile start-state slots are numbered in 16 bits of a table entry's flags.
constexpr uint32_t kMaxTileSlots = 65536;

xg::PlanLayout batch_layout(const xg_ctx *ctx, uint32_t max_reqs, uint32_t max_tiles) {
  const uint32_t jump_bytes = (uint32_t)(xg::member_degree(ctx->family) / 8);
  return xg::plan_layout(max_reqs, max_tiles, xg::family_state_bytes(ctx->family), jump_bytes);
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
    e = xg::launch_skip(ctx->d_state, first, count, J, step ? nullptr : &g, ctx->num_cus, s);
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

xg_status xg_generate_batch_planned(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs,
                                    const uint32_t *d_groups, uint32_t num_groups, void *d_out,
                                    uint64_t out_elems, const xg_tune *tune, void *d_work, void *stream) {
  if (!ctx || !d_reqs || !d_groups || !d_out || !d_work) return XG_EINVAL;
  if (!batch_member(ctx)) return XG_ENOTSUP;
  if (num_groups > num_reqs) return XG_ERANGE;
  const uintptr_t out_align = ctx->family == XG_FAMILY_R64_W64 ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(d_reqs) % 8 || reinterpret_cast<uintptr_t>(d_groups) % 4 ||
      reinterpret_cast<uintptr_t>(d_out) % out_align || reinterpret_cast<uintptr_t>(d_work) % 4)
    return XG_EALIGN;
  xg::Shape shape = xg::default_batch_shape(num_groups, ctx->num_cus);
  if (tune && !tune_to_shape(tune, tune->blocks_per_cu, &shape)) return XG_EINVAL;
  xg_status st = check_ctx_device(ctx);
  if (st != XG_OK) return st;
  if (num_groups == 0) return XG_OK;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t *work = static_cast<uint32_t *>(d_work);
  hipError_t e = xg::launch_work_init(work, num_groups, num_reqs, s);
  if (e == hipSuccess) {
    if (paper_member(ctx))
      e = xg::launch_batch(shape, ctx->num_cus, ctx->d_state, ctx->num_streams, d_reqs, d_groups, num_groups,
                           static_cast<uint32_t *>(d_out), out_elems, work, s);
    else
      e = xg::launch_family_batch(ctx->family, shape, ctx->num_cus, reinterpret_cast<unsigned char *>(ctx->d_state),
                                  ctx->num_streams, d_reqs, d_groups, num_groups, d_out, out_elems, work, s);
  }
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

size_t xg_batch_scratch_bytes(const xg_ctx *ctx, uint32_t max_reqs, uint32_t max_tiles) {
  if (!ctx || max_reqs == 0 || max_tiles > kMaxTileSlots ||
      (uint64_t)max_reqs + max_tiles > xg::kPlanMaxElems)
    return 0;
  return batch_layout(ctx, max_reqs, max_tiles).total;
}

xg_status xg_set_batch_scratch(xg_ctx *ctx, void *d_scratch, size_t scratch_bytes, uint32_t max_reqs,
                               uint32_t max_tiles, uint64_t tile_words, void *stream) {
  if (!ctx) return XG_EINVAL;
  if (!d_scratch) {
    ctx->d_batch = nullptr;
    return XG_OK;
  }
  if (!batch_member(ctx)) return XG_ENOTSUP;
  if (max_reqs == 0 || max_tiles > kMaxTileSlots || (uint64_t)max_reqs + max_tiles > xg::kPlanMaxElems)
    return XG_EINVAL;
  const bool tiles = tile_words != 0 && max_tiles != 0;
  if (tile_words && (tile_words % 64 || tile_words < (1ull << 12) || tile_words > (1ull << 30))) return XG_EINVAL;
  if (tiles && !paper_member(ctx)) return XG_ENOTSUP;
  if (reinterpret_cast<uintptr_t>(d_scratch) % 256) return XG_EALIGN;
  const xg::PlanLayout layout = batch_layout(ctx, max_reqs, tiles ? max_tiles : 0);
  if (scratch_bytes < layout.total) return XG_ERANGE;
  xg_status st = check_ctx_device(ctx);
  if (st != XG_OK) return st;
  if (tiles) {
    std::vector<uint64_t> table;
    try {
      table.resize((size_t)(xg::kMaxSegments - 1) * 64);
    } catch (const std::bad_alloc &) {
      return XG_ENOMEM;
    }
    if (!xg::jump_table(ctx->family, tile_words, xg::kMaxSegments - 1, table.data())) return XG_ENOTSUP;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const xg::PlanPtrs p = xg::plan_ptrs(d_scratch, layout);
    if (hipMemcpyAsync(p.jump, table.data(), table.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return XG_EHIP;
  }
  ctx->d_batch = d_scratch;
  ctx->batch_layout = layout;
  ctx->batch_max_reqs = max_reqs;
  ctx->batch_max_tiles = tiles ? max_tiles : 0;
  ctx->tile_words = tiles ? tile_words : 0;
  return XG_OK;
}

xg_status xg_generate_batch(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs, void *d_out,
                            const char *tune_key, void *stream) {
  if (!ctx || !d_reqs || !d_out || !ctx->d_batch) return XG_EINVAL;
  if (!batch_member(ctx)) return XG_ENOTSUP;
  if (num_reqs > ctx->batch_max_reqs) return XG_EBUSY;
  const uintptr_t out_align = ctx->family == XG_FAMILY_R64_W64 ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(d_reqs) % 8 || reinterpret_cast<uintptr_t>(d_out) % out_align) return XG_EALIGN;
  xg::Shape shape;
  xg_status st = xg::batch_shape(ctx, tune_key, num_reqs, &shape);
  if (st != XG_OK) return st;
  st = check_ctx_device(ctx);
  if (st != XG_OK) return st;
  // An empty table still runs the planner, which clears the workspace's
  // counts and error word.
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = xg::plan_on_device(ctx, ctx->d_batch, ctx->batch_layout, d_reqs, num_reqs, ctx->tile_words,
                                    ctx->batch_max_tiles, s);
  if (e == hipSuccess)
    e = xg::serve_planned(ctx, ctx->d_batch, ctx->batch_layout, num_reqs, ctx->tile_words, ctx->batch_max_tiles,
                          ctx->d_state, d_out, shape, s);
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

xg_status xg_batch_read_plan(const xg_ctx *ctx, xg_request *h_table, uint32_t max_entries, uint32_t *h_groups,
                             uint32_t max_groups, uint32_t *num_entries, uint32_t *num_groups, void *stream) {
  if (!ctx || !ctx->d_batch || !h_table || !h_groups || !num_entries || !num_groups) return XG_EINVAL;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const xg::PlanPtrs p = xg::plan_ptrs(ctx->d_batch, ctx->batch_layout);
  uint32_t counts[4];
  if (hipMemcpyAsync(counts, p.work, sizeof counts, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return XG_EHIP;
  *num_groups = counts[2];
  *num_entries = counts[3];
  if (counts[3] > max_entries || counts[2] > max_groups) return XG_ERANGE;
  if (hipMemcpyAsync(h_table, p.table, (size_t)counts[3] * sizeof(xg_request), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(h_groups, p.offs, ((size_t)counts[2] + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return XG_EHIP;
  return XG_OK;
}

constexpr int kMaxReps = 100;  // timed repetitions per candidate shape

xg_status xg_autotune_batch(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs, void *d_scratch_out,
                            void *d_scratch_state, const char *tune_key, int reps, xg_tune *best,
                            float *times_ms, uint32_t max_times, uint32_t *num_times, void *stream) {
  if (num_times) *num_times = 0;
  if (!ctx || !d_reqs || !d_scratch_out || !best || !d_scratch_state || reps < 1 || reps > kMaxReps ||
      !ctx->d_batch)
    return XG_EINVAL;
  if (!batch_member(ctx)) return XG_ENOTSUP;
  if (num_reqs > ctx->batch_max_reqs) return XG_EBUSY;
  if (tune_key) {  // a valid key (the lookup's own check)
    xg_tune probe;
    if (xg_tune_cache_get(ctx->arch, ctx->num_cus, ctx->family, tune_key, &probe, nullptr) == XG_EINVAL)
      return XG_EINVAL;
  }
  const uintptr_t out_align = ctx->family == XG_FAMILY_R64_W64 ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(d_reqs) % 8 || reinterpret_cast<uintptr_t>(d_scratch_out) % out_align ||
      reinterpret_cast<uintptr_t>(d_scratch_state) % 16)
    return XG_EALIGN;
  xg_status result = check_ctx_device(ctx);
  if (result != XG_OK) return result;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t state_bytes = xg_family_state_bytes(ctx->family, ctx->num_streams);
  if (xg::plan_on_device(ctx, ctx->d_batch, ctx->batch_layout, d_reqs, num_reqs, ctx->tile_words,
                         ctx->batch_max_tiles, s) != hipSuccess)
    return XG_EHIP;

  static const uint32_t kWpb[] = {1, 2, 4, 8, 16};
  static const uint32_t kUnroll[] = {1, 2, 4, 8};
  static const uint32_t kBpc[] = {1, 2, 4, 8, 16, 32};
  static const uint32_t kStoreWords[] = {1, 4};
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return XG_EHIP;
  }
  // One timed run of the planned table in `shape` on a scratch copy of the
  // state; -1 on a HIP error.
  auto time_once = [&](const xg::Shape &shape) -> float {
    float t = 0.f;
    if (hipMemcpyAsync(d_scratch_state, ctx->d_state, state_bytes, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipEventRecord(t0, s) != hipSuccess ||
        xg::serve_planned(ctx, ctx->d_batch, ctx->batch_layout, num_reqs, ctx->tile_words, ctx->batch_max_tiles,
                          static_cast<uint32_t *>(d_scratch_state), d_scratch_out, shape, s, true) != hipSuccess ||
        hipEventRecord(t1, s) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
        hipEventElapsedTime(&t, t0, t1) != hipSuccess)
      return -1.f;
    return t;
  };
  struct Cand {
    xg_tune tune;
    xg::Shape shape;
    float med;
    uint32_t rec;  // its record in times_ms (UINT32_MAX: none)
  };
  std::vector<Cand> cands;
  uint32_t recorded = 0;
  const bool member = !paper_member(ctx);
  // First pass: every shape, median of `reps` runs after a warm-up.
  for (uint32_t wpb : kWpb) {
    for (uint32_t un : kUnroll) {
      for (uint32_t bpc : kBpc) {
        for (uint32_t sw : kStoreWords) {
          if (result != XG_OK) break;
          if (wpb * bpc > 32) continue;                 // more waves than a compute unit holds
          if (sw == 4 && (un < 4 || member)) continue;  // the members' batch kernel has no wide stores
          Cand c{xg_tune{wpb, un, bpc, sw}, xg::Shape{}, 0.f, UINT32_MAX};
          (void)tune_to_shape(&c.tune, bpc, &c.shape);
          float ms[kMaxReps];
          int nms = 0;
          for (int rep = 0; rep <= reps; ++rep) {
            const float t = time_once(c.shape);
            if (t < 0.f) {
              result = XG_EHIP;
              break;
            }
            if (rep > 0) ms[nms++] = t;  // rep 0 is the warm-up
          }
          if (result != XG_OK) break;
          std::sort(ms, ms + nms);
          c.med = ms[nms / 2];
          if (times_ms && recorded < max_times) {
            float *rec = times_ms + 5 * recorded;
            rec[0] = (float)wpb; rec[1] = (float)un; rec[2] = (float)bpc; rec[3] = c.med; rec[4] = (float)sw;
            c.rec = recorded++;
          }
          try {
            cands.push_back(c);
          } catch (const std::bad_alloc &) {
            result = XG_ENOMEM;
          }
        }
      }
    }
  }
  // Second pass: the kFinalists fastest, timed again kRefineReps more times
  // each, in turns (so that a drift of the clock touches all alike); the best
  // median of the refined times wins and replaces their records.
  constexpr size_t kFinalists = 8;
  constexpr int kRefineReps = 5;
  float best_ms = -1.f;
  if (result == XG_OK && !cands.empty()) {
    std::sort(cands.begin(), cands.end(), [](const Cand &a, const Cand &b) { return a.med < b.med; });
    const size_t nf = cands.size() < kFinalists ? cands.size() : kFinalists;
    float refined[kFinalists][kRefineReps];
    for (int rep = 0; rep < kRefineReps && result == XG_OK; ++rep)
      for (size_t f = 0; f < nf && result == XG_OK; ++f) {
        const float t = time_once(cands[f].shape);
        if (t < 0.f) result = XG_EHIP;
        refined[f][rep] = t;
      }
    for (size_t f = 0; f < nf && result == XG_OK; ++f) {
      std::sort(refined[f], refined[f] + kRefineReps);
      const float med = refined[f][kRefineReps / 2];
      if (times_ms && cands[f].rec != UINT32_MAX) times_ms[5 * cands[f].rec + 3] = med;
      if (best_ms < 0.f || med < best_ms) {
        best_ms = med;
        *best = cands[f].tune;
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (num_times) *num_times = recorded;
  if (result == XG_OK && tune_key) result = xg_tune_cache_put(ctx->arch, ctx->num_cus, ctx->family, tune_key,
                                                              best, best_ms);
  return result;
}

xg_status xg_tune_identity(const xg_ctx *ctx, char *arch, size_t arch_len, uint32_t *cus) {
  if (!ctx || !arch || !cus || arch_len <= std::strlen(ctx->arch)) return XG_EINVAL;
  std::memcpy(arch, ctx->arch, std::strlen(ctx->arch) + 1);
  *cus = (uint32_t)ctx->num_cus;
  return XG_OK;
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

namespace xg {

xg_status batch_shape(const xg_ctx *ctx, const char *tune_key, uint64_t items, Shape *shape) {
  *shape = default_batch_shape(items, ctx->num_cus);
  if (!tune_key) return XG_OK;
  xg_tune t;
  const xg_status st = xg_tune_cache_get(ctx->arch, (uint32_t)ctx->num_cus, ctx->family, tune_key, &t, nullptr);
  if (st == XG_EINVAL) return XG_EINVAL;
  if (st == XG_OK) {
    const Shape cached{t.waves_per_block, t.unroll, t.blocks_per_cu,
                       t.store_words ? t.store_words : (t.unroll >= 4 ? 4u : 1u)};
    if (shape_valid(cached)) *shape = cached;
  }
  return XG_OK;
}

hipError_t plan_on_device(const xg_ctx *ctx, void *base, const PlanLayout &layout, const xg_request *d_reqs,
                          uint32_t num_reqs, uint64_t tile_words, uint32_t max_tiles, hipStream_t s) {
  const PlanPtrs p = plan_ptrs(base, layout);
  return launch_plan(p, layout, d_reqs, num_reqs, ctx->num_streams, tile_words, tile_words ? max_tiles : 0, s);
}

hipError_t serve_planned(const xg_ctx *ctx, void *base, const PlanLayout &layout, uint32_t num_reqs,
                         uint64_t tile_words, uint32_t max_tiles, uint32_t *state, void *d_out, const Shape &shape,
                         hipStream_t s, bool requeue) {
  const PlanPtrs p = plan_ptrs(base, layout);
  const uint32_t tiles = tile_words ? max_tiles : 0;
  const uint32_t max_items = num_reqs + tiles;
  hipError_t e = requeue ? launch_work_requeue(p.work, s) : hipSuccess;
  if (e != hipSuccess) return e;
  if (ctx->family != XG_FAMILY_R128_W32)
    return launch_family_batch(ctx->family, shape, ctx->num_cus, reinterpret_cast<unsigned char *>(state),
                               ctx->num_streams, p.table, p.offs, max_items, d_out, UINT64_MAX, p.work, s);
  const SegmentArgs seg{p.jump, tile_words, tiles ? kMaxSegments - 1 : 0u, p.stage, tiles};
  if (tiles) e = launch_seg_starts(state, ctx->num_streams, p.table, max_items, p.work, seg, ctx->num_cus, s);
  if (e == hipSuccess)
    e = launch_batch(shape, ctx->num_cus, state, ctx->num_streams, p.table, p.offs, max_items,
                     static_cast<uint32_t *>(d_out), UINT64_MAX, p.work, s, tiles ? &seg : nullptr);
  return e;
}

}  // namespace xg
