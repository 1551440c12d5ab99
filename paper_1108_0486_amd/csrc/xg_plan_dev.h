// Device-side batch planner of libxg (the one-call xg_generate_batch) and the
// layout of its scratch memory.  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "xg.h"

namespace xg {

// Planner limits: requests plus tiles of one call, and elements one scan
// handles (1024 workgroups of 1024 elements).
constexpr uint32_t kPlanMaxElems = 1u << 20;

// Byte offsets of the planner's arrays inside one scratch buffer (each
// 256-byte aligned), for up to max_reqs requests and max_tiles tiles per call.
struct PlanLayout {
  size_t work;    // 64 words: queue counter, error word, items, table entries
  size_t meta;    // 64 words: planner counters
  size_t keys;    // key_cap 64-bit keys (stream << 32 | request index)
  size_t heads;   // max_reqs + 1 words: group number of each sorted request
  size_t costs;   // max_reqs + 1 64-bit prefix sums of request costs
  size_t hp;      // max_reqs + 1 words: first sorted position of each group
  size_t tiles;   // max_reqs + 1 words: prefix sums of tiles per group
  size_t items;   // item_cap 64-bit queue item keys
  size_t offs;    // max_reqs + max_tiles + 1 words: table offset of each item
  size_t table;   // max_reqs + max_tiles requests: the served table
  size_t sums;    // 1024 64-bit scan block sums
  size_t stage;   // max_tiles stream states: each tile's start state
  size_t jump;    // kMaxSegments - 1 jump polynomials z^(k L) mod P
  size_t total;
  uint32_t key_cap, item_cap;
};

// state_bytes: one stream's state; jump_bytes: one jump polynomial (0 when
// the member has no tiles).
PlanLayout plan_layout(uint32_t max_reqs, uint32_t max_tiles, uint32_t state_bytes, uint32_t jump_bytes);

// Pointers into one scratch buffer laid out by plan_layout.
struct PlanPtrs {
  uint32_t *work, *meta;
  uint64_t *keys;
  uint32_t *heads;
  uint64_t *costs;
  uint32_t *hp, *tiles;
  uint64_t *items;
  uint32_t *offs;
  xg_request *table;
  uint64_t *sums;
  uint32_t *stage;
  uint64_t *jump;
};

PlanPtrs plan_ptrs(void *base, const PlanLayout &l);

// Plans num_reqs requests (array order, device memory) on the device:
//   - a request with stream >= num_streams, dtype > XG_NORMAL or flags != 0 is
//     dropped and sets work[1];
//   - requests of one stream form one group, in array order;
//   - with tile_words = L > 0, a group of one request of more than L words
//     (and at most kMaxSegments tiles) becomes tiles of L words, each a
//     segment entry (kReqSegment, tile k, start-state slot), as long as the
//     tiles of all groups so far fit max_tiles slots;
//   - queue items (groups and tiles) are ordered by cost, largest first;
//   - work[0] = 0, work[2] = items, work[3] = table entries on return.
// Kernels only (graph-capturable); num_reqs <= max_reqs of the layout.
hipError_t launch_plan(const PlanPtrs &p, const PlanLayout &l, const xg_request *reqs, uint32_t num_reqs,
                       uint64_t num_streams, uint64_t tile_words, uint32_t max_tiles, hipStream_t stream);

}  // namespace xg
