// Concurrent first use of libxg's jump polynomials (xg_jump.cpp, host only):
// eight threads ask for z^J mod P of every member at once, so the lazily
// built moduli and the cache of recent results race.  Built with
// ThreadSanitizer; every thread's result must equal a single-threaded
// recomputation afterwards that bypasses the cache.  Prints OK.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "xg_host.h"

int main() {
  const uint64_t Js[] = {1, 4097, 123456789, 1ull << 40, ~0ull};
  constexpr int kThreads = 8, kWords = 64;
  std::vector<uint64_t> got((size_t)kThreads * 3 * 5 * kWords, 0);
  std::vector<int> ok((size_t)kThreads, 1);
  std::vector<std::thread> pool;
  for (int t = 0; t < kThreads; ++t) {
    pool.emplace_back([&, t] {
      for (int k = 0; k < 15; ++k) {
        const int f = (k + t) % 3, j = (k / 3 + t) % 5;   // each thread its own order
        uint64_t *g = &got[(((size_t)t * 3 + f) * 5 + j) * kWords];
        if (!xg::jump_polynomial((uint32_t)f, Js[j], g)) ok[t] = 0;
      }
    });
  }
  for (auto &th : pool) th.join();
  for (int t = 0; t < kThreads; ++t)
    if (!ok[t]) { std::printf("thread %d failed\n", t); return 1; }
  for (int f = 0; f < 3; ++f)
    for (int j = 0; j < 5; ++j) {
      uint64_t ref[kWords] = {0};
      if (!xg::jump_polynomial_uncached((uint32_t)f, Js[j], ref)) return 1;
      const int w = xg::member_degree((uint32_t)f) / 64;
      for (int t = 0; t < kThreads; ++t)
        for (int i = 0; i < w; ++i)
          if (got[(((size_t)t * 3 + f) * 5 + j) * kWords + i] != ref[i]) {
            std::printf("mismatch f=%d j=%d t=%d\n", f, j, t);
            return 1;
          }
    }
  std::printf("OK\n");
  return 0;
}
