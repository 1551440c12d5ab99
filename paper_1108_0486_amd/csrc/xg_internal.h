// Internal interface between the C-ABI layer (xg_api.cpp) and the HIP kernels
// (xg_kernels.hip).  Not installed; the public interface is include/xg.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xg.h"

namespace xg {

constexpr uint32_t kStateWords = XG_STATE_WORDS;
constexpr uint32_t kWave = 64;

// Request kinds of the plain launch (the three output types of xg.h plus the
// fused normal-moments reduction).
enum Kind : uint32_t { kU32 = XG_U32, kF32 = XG_F32, kNormal = XG_NORMAL, kMoments = 3 };

struct Shape {
  uint32_t waves_per_block;  // 1, 2, 4, 8, 16
  uint32_t unroll;           // 1, 2, 4, 8
  uint32_t blocks_per_cu;    // persistent batch only
};

bool shape_valid(const Shape &s);

hipError_t launch_init(uint32_t *state, uint64_t num_streams, uint64_t seed, hipStream_t stream);

hipError_t launch_generate(Kind kind, const Shape &shape, uint32_t *state, uint64_t first,
                           uint64_t count, uint64_t n, void *out, hipStream_t stream);

hipError_t launch_batch(const Shape &shape, int num_cus, uint32_t *state, uint64_t num_streams,
                        const xg_request *reqs, uint32_t num_reqs, const uint32_t *groups,
                        uint32_t num_groups,
                        uint32_t *out, uint64_t out_elems, uint32_t *work, hipStream_t stream);

}  // namespace xg
