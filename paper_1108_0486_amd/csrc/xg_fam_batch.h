// Launcher of the batched kernel for the further family members
// (xg_family.hip), used by xg_generate_batch and the request server, and the
// byte offset of pos in a member's stream state.  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xg.h"
#include "xg_internal.h"

namespace xg {

// Serves the table described by the workspace (work[2] groups of reqs,
// work[3] entries; see launch_work_init) with blocks_per_cu x CUs persistent
// workgroups of waves_per_block wavefronts, two groups per wavefront (fewer
// workgroups when max_groups, an upper bound of work[2], is smaller);
// shape.store_words is not used.  out holds out_elems elements of the
// member's word width.
hipError_t launch_family_batch(uint32_t family, const Shape &shape, int num_cus, unsigned char *state,
                               uint64_t num_streams, const xg_request *reqs, const uint32_t *groups,
                               uint32_t max_groups, void *out, uint64_t out_elems, uint32_t *work,
                               hipStream_t stream);

// Byte offset of the 64-bit position in one stream's state of a family.
uint32_t family_pos_offset(uint32_t family);

}  // namespace xg
