// xg_generate_batch_static: the one-call batch for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  The planner's scratch is a file-scope
// device array of this library instead of memory the caller attaches; each
// GPU the library runs on holds its own copy until the process ends.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>

#include "xg.h"
#include "xg_internal.h"
#include "xg_launch.h"
#include "xg_plan_dev.h"

namespace {

constexpr uint32_t kStaticMaxReqs = XG_STATIC_MAX_REQS;
constexpr size_t kStaticBytes = XG_STATIC_SCRATCH_BYTES;  // holds the planner's layout for kStaticMaxReqs, no tiles

// The scratch.  In host code this name is not a device address: kernels only
// ever get the per-device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[kStaticBytes];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void *g_scratch[kMaxDevices];
hipError_t g_status[kMaxDevices];

// The device address of scratch on device dev (current), looked up once per
// device: when a handle is created there (static_scratch_prepare), or else on
// the first call.
void *scratch_on(int dev, hipError_t *status) {
  std::call_once(g_once[dev], [dev] {
    void *p = nullptr;
    g_status[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_scratch[dev] = g_status[dev] == hipSuccess ? p : nullptr;
  });
  *status = g_status[dev];
  return g_scratch[dev];
}

// Copies the batch's error word to the caller's word.
__global__ void k_copy_error(const uint32_t *__restrict__ work, uint32_t *__restrict__ dst) {
  if (threadIdx.x == 0) *dst = work[1];
}

}  // namespace

namespace xg {

hipError_t static_scratch_prepare(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  hipError_t st = hipSuccess;
  (void)scratch_on(dev, &st);
  return st;
}

}  // namespace xg

extern "C" {

xg_status xg_generate_batch_static(xg_ctx *ctx, const xg_request *d_reqs, uint32_t num_reqs, void *d_out,
                                   const char *tune_key, uint32_t *d_error, void *stream) {
  if (!ctx || !d_reqs || !d_out) return XG_EINVAL;
  if (ctx->family != XG_FAMILY_R128_W32 && ctx->family != XG_FAMILY_R64_W32 && ctx->family != XG_FAMILY_R64_W64)
    return XG_ENOTSUP;
  if (num_reqs > kStaticMaxReqs) return XG_EBUSY;
  const uintptr_t out_align = ctx->family == XG_FAMILY_R64_W64 ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(d_reqs) % 8 || reinterpret_cast<uintptr_t>(d_out) % out_align ||
      reinterpret_cast<uintptr_t>(d_error) % 4)
    return XG_EALIGN;
  xg::Shape shape;
  xg_status st = xg::batch_shape(ctx, tune_key, num_reqs, &shape);
  if (st != XG_OK) return st;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return XG_EHIP;
  if (dev != ctx->device) return XG_EINVAL;
  if (dev < 0 || dev >= kMaxDevices) return XG_ENOTSUP;
  const xg::PlanLayout layout =
      xg::plan_layout(kStaticMaxReqs, 0, xg::family_state_bytes(ctx->family), 0);
  if (layout.total > kStaticBytes) return XG_ENOTSUP;
  hipError_t e = hipSuccess;
  void *base = scratch_on(dev, &e);
  if (!base) return XG_EHIP;
  const hipStream_t s = static_cast<hipStream_t>(stream);
  // The planner's first kernel clears the counters and the error word the
  // previous call left in the array; every other word it reads it writes first.
  e = xg::plan_on_device(ctx, base, layout, d_reqs, num_reqs, 0, 0, s);
  if (e == hipSuccess) e = xg::serve_planned(ctx, base, layout, num_reqs, 0, 0, ctx->d_state, d_out, shape, s);
  if (e == hipSuccess && d_error)
    e = xg::launch(k_copy_error, dim3(1), dim3(64), 0, s, xg::plan_ptrs(base, layout).work, d_error);
  return e == hipSuccess ? XG_OK : XG_EHIP;
}

}  // extern "C"
