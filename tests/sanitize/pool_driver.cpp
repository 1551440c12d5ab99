// Randomised check of the request server's output pool (xg_pool.h) against a
// brute-force model: one flag per 64-element unit of the capacity.
//
// After every operation:
//   * a successful alloc returns an aligned range inside the capacity that the
//     model holds free, and it is the lowest such start (first fit over fully
//     coalesced free ranges = the lowest start of a free run long enough);
//   * a failed alloc means no free run in the model is long enough;
//   * the pool's free ranges are exactly the model's maximal free runs (so
//     frees coalesce with both neighbours), and used() is the model's count.
// Prints OK on success; any mismatch aborts with a message.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "xg_pool.h"

namespace {

void fail(const char *what, uint64_t a, uint64_t b) {
  std::fprintf(stderr, "pool mismatch: %s (%llu, %llu)\n", what, (unsigned long long)a, (unsigned long long)b);
  std::abort();
}

struct Model {
  std::vector<uint8_t> used;  // per 64-element unit
  explicit Model(uint64_t units) : used(units, 0) {}
  // Lowest start unit of a free run of at least `need` units, or UINT64_MAX.
  uint64_t first_fit(uint64_t need) const {
    uint64_t run = 0;
    for (uint64_t u = 0; u < used.size(); ++u) {
      run = used[u] ? 0 : run + 1;
      if (run == need) return u + 1 - need;
    }
    return UINT64_MAX;
  }
};

void check_state(const xg::Pool &p, const Model &m) {
  uint64_t busy = 0;
  for (uint8_t b : m.used) busy += b;
  if (p.used() != busy * xg::kPoolAlignElems) fail("used()", p.used(), busy * xg::kPoolAlignElems);
  auto it = p.free_ranges().begin();
  uint64_t u = 0;
  const uint64_t units = m.used.size();
  while (u < units) {
    if (m.used[u]) {
      ++u;
      continue;
    }
    uint64_t v = u;
    while (v < units && !m.used[v]) ++v;
    if (it == p.free_ranges().end()) fail("missing free range at", u, v);
    if (it->first != u * xg::kPoolAlignElems || it->second != (v - u) * xg::kPoolAlignElems)
      fail("free range differs", it->first, it->second);
    ++it;
    u = v;
  }
  if (it != p.free_ranges().end()) fail("extra free range", it->first, it->second);
}

void run(uint64_t capacity, uint64_t seed, int ops) {
  xg::Pool pool(capacity);
  if (pool.capacity() != capacity / 64 * 64) fail("capacity", pool.capacity(), capacity);
  const uint64_t units = pool.capacity() / xg::kPoolAlignElems;
  Model model(units);
  std::mt19937_64 rng(seed);
  struct Live { uint64_t off, n; };
  std::vector<Live> live;
  for (int op = 0; op < ops; ++op) {
    const bool do_alloc = live.empty() || rng() % 100 < 55;
    if (do_alloc && pool.capacity()) {
      // Mostly small requests, some large, some exactly at unit boundaries.
      uint64_t n;
      switch (rng() % 4) {
        case 0: n = 1 + rng() % 64; break;
        case 1: n = 64 * (1 + rng() % 4); break;
        case 2: n = 1 + rng() % (pool.capacity() / 4 + 1); break;
        default: n = 1 + rng() % pool.capacity(); break;
      }
      const uint64_t need = xg::round_elems(n) / xg::kPoolAlignElems;
      const uint64_t want = model.first_fit(need);
      const uint64_t off = pool.alloc(n);
      if (off == UINT64_MAX) {
        if (want != UINT64_MAX) fail("alloc failed with room at", want, n);
      } else {
        if (off % xg::kPoolAlignElems) fail("unaligned offset", off, n);
        if (off + n > capacity || off + xg::round_elems(n) > pool.capacity()) fail("range past capacity", off, n);
        if (off != want * xg::kPoolAlignElems) fail("not first fit", off, want);
        for (uint64_t u = off / 64; u < off / 64 + need; ++u) {
          if (model.used[u]) fail("overlap at unit", u, n);
          model.used[u] = 1;
        }
        live.push_back({off, n});
      }
    } else if (!live.empty()) {
      const size_t i = rng() % live.size();
      const Live l = live[i];
      live[i] = live.back();
      live.pop_back();
      pool.release(l.off, l.n);
      for (uint64_t u = l.off / 64; u < (l.off + xg::round_elems(l.n)) / 64; ++u) model.used[u] = 0;
    }
    check_state(pool, model);
  }
  for (const Live &l : live) pool.release(l.off, l.n);
  live.clear();
  std::fill(model.used.begin(), model.used.end(), 0);
  check_state(pool, model);
  // An emptied pool is one free range again: the largest request fits at 0.
  if (pool.capacity() && pool.alloc(pool.capacity()) != 0) fail("emptied pool not whole", pool.capacity(), 0);
}

}  // namespace

int main() {
  const uint64_t capacities[] = {0, 1, 63, 64, 65, 100, 127, 128, 1000, 4096, 4096 + 37, 65536};
  uint64_t seed = 1;
  for (uint64_t c : capacities)
    for (int rep = 0; rep < 4; ++rep) run(c, seed++, 4000);
  std::printf("OK\n");
  return 0;
}
