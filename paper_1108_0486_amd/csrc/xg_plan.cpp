// Host-side batch planner of libxg (xg_plan_batch and the server's variant):
// groups requests by stream (order kept inside a group), gives each segment
// of a split request a group of its own, and orders groups largest first so
// the device's dynamic queue balances uneven lengths.  No HIP here.
#include <algorithm>
#include <cstdint>
#include <new>
#include <unordered_map>
#include <vector>

#include "xg.h"
#include "xg_host.h"

namespace xg {
namespace {

// Relative cost of a request in the planner's balance: words consumed, with
// normals weighted for their transcendental work.
uint64_t request_cost(const xg_request &r) {
  if (r.dtype == XG_NORMAL) return 4 * (r.n + (r.n & 1));
  return r.n;
}

}  // namespace

xg_status plan_batch(const xg_request *h_reqs, uint32_t num_reqs, uint64_t num_streams, uint64_t out_elems,
                     xg_request *h_sorted, uint32_t *h_groups, uint32_t *num_groups, bool allow_segments) {
  if (!h_sorted || !h_groups || !num_groups || (num_reqs && !h_reqs)) return XG_EINVAL;
  *num_groups = 0;
  for (uint32_t i = 0; i < num_reqs; ++i) {
    const xg_request &r = h_reqs[i];
    const bool seg_ok = allow_segments && (r.flags & kReqSegment) && !(r.flags & kReqUndefinedBits);
    if (r.dtype > XG_NORMAL || (r.flags != 0 && !seg_ok)) return XG_EINVAL;
    if (r.stream >= num_streams) return XG_ERANGE;
    if (r.out_offset > out_elems || r.n > out_elems - r.out_offset) return XG_ERANGE;
  }
  try {
    // Group requests by stream, keeping arrival order inside a group; each
    // segment of a split request is a group of its own.
    std::unordered_map<uint64_t, uint32_t> group_of;
    std::vector<std::vector<uint32_t>> members;
    std::vector<uint64_t> cost;
    group_of.reserve(num_reqs * 2 + 1);
    for (uint32_t i = 0; i < num_reqs; ++i) {
      uint32_t g;
      const bool own = (h_reqs[i].flags & kReqSegment) != 0;
      auto it = own ? group_of.end() : group_of.find(h_reqs[i].stream);
      if (it == group_of.end()) {
        g = (uint32_t)members.size();
        if (!own) group_of.emplace(h_reqs[i].stream, g);
        members.emplace_back();
        cost.push_back(0);
      } else {
        g = it->second;
      }
      members[g].push_back(i);
      cost[g] += request_cost(h_reqs[i]);
    }
    // Largest group first (longest-processing-time order for the dynamic queue).
    std::vector<uint32_t> order(members.size());
    for (uint32_t g = 0; g < order.size(); ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(),
                     [&](uint32_t a, uint32_t b) { return cost[a] > cost[b]; });
    uint32_t k = 0;
    for (uint32_t j = 0; j < order.size(); ++j) {
      h_groups[j] = k;
      for (uint32_t i : members[order[j]]) h_sorted[k++] = h_reqs[i];
    }
    h_groups[order.size()] = k;
    *num_groups = (uint32_t)order.size();
  } catch (const std::bad_alloc &) {
    return XG_ENOMEM;
  }
  return XG_OK;
}


}  // namespace xg

extern "C" xg_status xg_plan_batch(const xg_request *h_reqs, uint32_t num_reqs, uint64_t num_streams,
                        uint64_t out_elems, xg_request *h_sorted, uint32_t *h_groups,
                        uint32_t *num_groups) {
  return xg::plan_batch(h_reqs, num_reqs, num_streams, out_elems, h_sorted, h_groups, num_groups, false);
}
