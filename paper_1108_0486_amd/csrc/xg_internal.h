// Internal interface between the C-ABI layer (xg_api.cpp) and the HIP kernels
// (xg_kernels.hip).  Not installed; the public interface is include/xg.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xg.h"
#include "xg_host.h"
#include "xg_plan_dev.h"

namespace xg {

constexpr uint32_t kStateWords = XG_STATE_WORDS;
constexpr uint32_t kWave = 64;

// Request kinds of the plain launch (the three output types of xg.h plus the
// fused normal-moments reduction).
enum Kind : uint32_t { kU32 = XG_U32, kF32 = XG_F32, kNormal = XG_NORMAL, kMoments = 3, kU64 = XG_U64, kF64 = XG_F64 };

struct Shape {
  uint32_t waves_per_block;  // 1, 2, 4, 8, 16; 0 (plain launches only): chosen per launch
  uint32_t unroll;           // 1, 2, 4, 8; 0 (plain launches only): chosen per launch
  uint32_t blocks_per_cu;    // persistent batch only
  uint32_t store_words;      // 1 or 4 (4 needs unroll >= 4)
};

constexpr Shape kDefaultPlain{0, 0, 1, 4};  // waves_per_block and unroll chosen per launch

// Waves per block for a plain launch of `count` streams on `num_cus` compute
// units: one stream per wavefront, and at least as many blocks as compute
// units, so that the wavefronts spread one per SIMD before any SIMD gets two.
uint32_t auto_waves_per_block(uint64_t count, int num_cus);
// Default persistent-batch shapes, chosen by the number of queue items.  With
// at least eight items per compute unit the batch is bound by HBM writes, and
// eight wavefronts per compute unit write fastest (every unroll takes the same
// time on unaligned requests; eight chunks per trip are faster on aligned
// ones).  With fewer items each wavefront's own rate decides, and eight
// wavefronts per compute unit at eight chunks per trip serve a group fastest.
// Neither uses the wide stores: staging through LDS gained nothing.
// Queue items a batch wavefront takes per atomic: up to kBatchTakeWords
// words' worth at the size of the items it just served, at most
// kBatchMaxTake (one counter serves every wavefront, and same-address atomics
// complete one at a time).
constexpr uint32_t kBatchMaxTake = 16;
constexpr uint64_t kBatchTakeWords = 65536;

constexpr Shape kBatchThroughput{4, 8, 2, 1};
constexpr Shape kBatchLatency{4, 8, 8, 1};
inline Shape default_batch_shape(uint64_t items, int num_cus) {
  return items >= 8u * (uint64_t)(num_cus > 0 ? num_cus : 1) ? kBatchThroughput : kBatchLatency;
}

bool shape_valid(const Shape &s);

hipError_t launch_init(uint32_t *state, uint64_t num_streams, uint64_t seed, hipStream_t stream);

// num_cus: normals and moments with fewer than two wavefronts per SIMD take
// the pair gather that needs no LDS.
hipError_t launch_generate(Kind kind, const Shape &shape, uint32_t *state, uint64_t first,
                           uint64_t count, uint64_t n, void *out, int num_cus, hipStream_t stream);

// Bulk-fill layout of xg_fill_u32 / xg_fill_f32 (kind kU32 or kF32).
hipError_t launch_fill(Kind kind, const Shape &shape, uint32_t *state, uint64_t first, uint64_t count,
                       uint64_t n, uint32_t *out, hipStream_t stream);

hipError_t launch_box_muller(const uint32_t *words, uint64_t pairs, float *out, hipStream_t stream);

// Skips below this many words step through them; longer skips jump.
constexpr uint64_t kJumpThreshold = 1ull << 15;

struct JumpPoly {
  uint64_t w[64];
};

// Advances streams [first, first + count) by J words: by stepping when
// g == nullptr, else by evaluating g(T) on each state (g = z^J mod P), with a
// workgroup per stream when the streams fit on num_cus compute units at once.
hipError_t launch_skip(uint32_t *state, uint64_t first, uint64_t count, uint64_t J, const JumpPoly *g,
                       int num_cus, hipStream_t stream);

// Segment entries of a batch table (kReqSegment, see xg_host.h): tile k of a
// request starts from its stream's state jumped by k L words, staged in slot
// (flags >> 16) by launch_seg_starts before the batch kernel runs.
struct SegmentArgs {
  const uint64_t *jump_table;  // (max_k) x 64 words: entry k - 1 = z^(k L) mod P
  uint64_t seg_words;          // L
  uint32_t max_k;              // entries in jump_table
  uint32_t *stage;             // max_slots x kStateWords words
  uint32_t max_slots;
};

// The batch kernels' workspace (64 words): work[0] queue counter, work[1]
// error word (set to 1 by a skipped request or group), work[2] groups in the
// table, work[3] table entries.  launch_work_init fills it for a host-built
// table; the device planner fills it itself.
hipError_t launch_work_init(uint32_t *work, uint32_t num_groups, uint32_t num_reqs, hipStream_t stream);
// Clears only the queue counter, to serve the same table again.
hipError_t launch_work_requeue(uint32_t *work, hipStream_t stream);

// Stages the start state of every segment entry among the table's first
// work[3] entries: as many workgroups as the chip holds at once (at most
// max_entries), each taking every gridDim-th entry.
hipError_t launch_seg_starts(const uint32_t *state, uint64_t num_streams, const xg_request *reqs,
                             uint32_t max_entries, const uint32_t *work, const SegmentArgs &seg, int num_cus,
                             hipStream_t stream);

// Serves the table described by work (groups: work[2] + 1 offsets into reqs)
// with blocks_per_cu x CUs persistent workgroups (fewer when max_groups, an
// upper bound of work[2], is smaller).  seg may be null when the table has no
// segment entries.
hipError_t launch_batch(const Shape &shape, int num_cus, uint32_t *state, uint64_t num_streams,
                        const xg_request *reqs, const uint32_t *groups, uint32_t max_groups, uint32_t *out,
                        uint64_t out_elems, uint32_t *work, hipStream_t stream, const SegmentArgs *seg = nullptr);

// Write-only reference: out[0 .. words) = value with 16-byte non-temporal
// stores (out 16-byte aligned).
hipError_t launch_fill_value(uint32_t *out, uint64_t words, uint32_t value, int num_cus, hipStream_t stream);

// Further family members (r = 64, s = 33; two streams per wavefront).
// Bytes of one stream's state (0: unknown family).
uint32_t family_state_bytes(uint32_t family);
hipError_t launch_family_init(uint32_t family, unsigned char *state, uint64_t num_streams, uint64_t seed,
                              hipStream_t stream);
// kind: kU32 / kF32 for XG_FAMILY_R64_W32, kU64 / kF64 for XG_FAMILY_R64_W64;
// fill selects the bulk-fill layout (32-word chunks).  shape.waves_per_block
// counts wavefronts, i.e. pairs of streams.
hipError_t launch_family_generate(uint32_t family, Kind kind, bool fill, const Shape &shape, unsigned char *state,
                                  uint64_t first, uint64_t count, uint64_t n, void *out, hipStream_t stream);
// Advances streams [first, first + count) of a further member by J words: by
// stepping when g == nullptr, else by evaluating g(T) (g = z^J mod P, its
// member_degree / 64 low words used).
hipError_t launch_family_skip(uint32_t family, unsigned char *state, uint64_t first, uint64_t count, uint64_t J,
                              const JumpPoly *g, hipStream_t stream);


}  // namespace xg

struct xg_ctx;

namespace xg {

// The one-call batch, shared by its entry points (xg_api.cpp).
// The launch shape for tune_key: the tuning cache's entry for ctx's device
// and family, else the default for `items` queue items (XG_EINVAL for a
// malformed key).
xg_status batch_shape(const xg_ctx *ctx, const char *tune_key, uint64_t items, Shape *shape);
// Plans num_reqs requests (device memory, table order) into the scratch at
// base, with tiles of tile_words words in up to max_tiles slots (0: none).
hipError_t plan_on_device(const xg_ctx *ctx, void *base, const PlanLayout &layout, const xg_request *d_reqs,
                          uint32_t num_reqs, uint64_t tile_words, uint32_t max_tiles, hipStream_t s);
// Serves the table the planner left in the scratch at base on the streams at
// state (the tiles' start states, then the persistent launch); requeue
// re-arms the queue first, to serve the same plan again.
hipError_t serve_planned(const xg_ctx *ctx, void *base, const PlanLayout &layout, uint32_t num_reqs,
                         uint64_t tile_words, uint32_t max_tiles, uint32_t *state, void *d_out, const Shape &shape,
                         hipStream_t s, bool requeue = false);

// Looks up the device address of xg_generate_batch_static's scratch array on
// device dev (current) once; called when a handle is created there.
hipError_t static_scratch_prepare(int dev);

}  // namespace xg

// The handle behind xg_ctx (include/xg.h).
struct xg_ctx {
  uint32_t *d_state;
  uint64_t num_streams;
  int device;
  int num_cus;
  char arch[32];    // device architecture name without feature suffixes
  xg::Shape plain;
  uint32_t family;  // XG_FAMILY_*
  // Scratch of the one-call batch (xg_set_batch_scratch); d_batch == nullptr: none.
  void *d_batch;
  xg::PlanLayout batch_layout;
  uint32_t batch_max_reqs, batch_max_tiles;
  uint64_t tile_words;  // 0: no tiles
};
