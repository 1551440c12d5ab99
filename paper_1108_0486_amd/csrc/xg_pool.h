// Output pool of libxg's request server: a first-fit allocator over
// [0, capacity) elements whose ranges start and end on 64-element (256-byte)
// boundaries, with frees that coalesce with both neighbours.  The capacity is
// rounded down to a multiple of 64, so every range lies inside the caller's
// buffer and a request of round_elems(n) <= capacity() fits an empty pool.
// Host-only (no HIP), so it is also built and fuzzed with a plain host compiler.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace xg {

constexpr uint64_t kPoolAlignElems = 64;

inline uint64_t round_elems(uint64_t n) { return (n + kPoolAlignElems - 1) / kPoolAlignElems * kPoolAlignElems; }

class Pool {
 public:
  explicit Pool(uint64_t capacity) : capacity_(capacity / kPoolAlignElems * kPoolAlignElems) {
    if (capacity_) free_[0] = capacity_;
  }
  // Returns the offset, or UINT64_MAX if no free range fits.
  uint64_t alloc(uint64_t n) {
    const uint64_t need = round_elems(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        const uint64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > need) free_[off + need] = len - need;
        used_ += need;
        return off;
      }
    }
    return UINT64_MAX;
  }
  // (off, n) must be a live allocation's offset and the n it was made with.
  void release(uint64_t off, uint64_t n) {
    const uint64_t len = round_elems(n);
    used_ -= len;
    auto next = free_.lower_bound(off);
    uint64_t start = off, size = len;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        size += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && start + size == next->first) {
      size += next->second;
      free_.erase(next);
    }
    free_[start] = size;
  }
  uint64_t used() const { return used_; }
  uint64_t capacity() const { return capacity_; }
  const std::map<uint64_t, uint64_t> &free_ranges() const { return free_; }

 private:
  uint64_t capacity_;
  uint64_t used_ = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length
};

}  // namespace xg
