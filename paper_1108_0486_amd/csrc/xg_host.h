// Host-only internals of libxg (no HIP): the batch planner and the jump
// polynomials.  Kept free of HIP headers so that they also build with a plain
// host compiler (the sanitizer tests do that).
#pragma once

#include <stdint.h>

#include "xg.h"

namespace xg {

// Request flags of library-built tables (callers' requests take flags 0).  A
// segment covers values [k L, k L + n') of a longer request on its stream
// (bits 8..15: k; bits 16..31: its staging slot).  Its start state is the
// stream's state jumped by k L words (jump_table entry k - 1 holds
// z^(k L) mod P), staged in its slot before the batch; it generates its n'
// values from there.  Only the last segment (kReqLast) writes the stream's
// state, so a request split into segments must be alone on its stream within
// its table.
constexpr uint32_t kReqSegment = 1u;
constexpr uint32_t kReqLast = 2u;
constexpr uint32_t kReqUndefinedBits = 0x000000FCu;
constexpr uint32_t kMaxSegments = 256;  // k in 0 .. 255

// xg_plan_batch, with segment requests (kReqSegment) allowed when
// allow_segments: each forms its own group.
xg_status plan_batch(const xg_request *h_reqs, uint32_t num_reqs, uint64_t num_streams, uint64_t out_elems,
                     xg_request *h_sorted, uint32_t *h_groups, uint32_t *num_groups, bool allow_segments);

// Jump polynomial z^J mod P of the x-part's characteristic polynomial
// (4096 bits, little-endian words) of Section 2's member.  False if P could
// not be derived.
bool jump_polynomial(uint64_t J, uint64_t g[64]);

// The same for a member XG_FAMILY_*: g receives member_degree(family) / 64
// words.  False for an unknown family or if P could not be derived.  The
// last 16 distinct (family, J) are kept, so repeated jumps by one J (streams
// split into equal blocks) skip the powering; jump_polynomial_uncached always
// computes.
int member_degree(uint32_t family);
bool jump_polynomial(uint32_t family, uint64_t J, uint64_t *g);
bool jump_polynomial_uncached(uint32_t family, uint64_t J, uint64_t *g);

// table[k] (member_degree(family) / 64 words each) = z^((k + 1) L) mod P for
// k < count.  False for an unknown family, if P could not be derived, or if
// host memory ran out.
bool jump_table(uint32_t family, uint64_t L, uint32_t count, uint64_t *table);

}  // namespace xg
