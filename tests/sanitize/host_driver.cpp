// Exercises libxg's host-only code (the batch planner and the jump
// polynomials) under AddressSanitizer/UndefinedBehaviorSanitizer.  Checks the
// planner's contract on random tables and its error codes, and prints the
// jump polynomials of the (member, J) pairs given on the command line as hex
// words (most-significant word first) for comparison with the oracle.
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "xg_host.h"

#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c);     \
      return 1;                                                   \
    }                                                             \
  } while (0)

static int plan_checks() {
  std::mt19937_64 rng(7);
  for (int trial = 0; trial < 200; ++trial) {
    const uint32_t n = (uint32_t)(rng() % 300);
    const uint64_t streams = 1 + rng() % 40;
    const bool segs = trial & 1;
    std::vector<xg_request> reqs(n);
    uint64_t off = 0;
    for (auto &r : reqs) {
      r.stream = rng() % streams;
      r.n = 1 + rng() % 5000;  // n >= 1: output offsets are distinct and name the request
      r.out_offset = off;
      off += r.n;
      r.dtype = (uint32_t)(rng() % 3);
      r.flags = segs && rng() % 4 == 0 ? (xg::kReqSegment | (uint32_t)(rng() % 256) << 8) : 0;
    }
    std::vector<xg_request> sorted(n + 1);
    std::vector<uint32_t> groups(n + 1);
    uint32_t ng = 12345;
    CHECK(xg::plan_batch(reqs.data(), n, streams, off, sorted.data(), groups.data(), &ng, segs) == XG_OK);
    CHECK(ng <= n && groups[0] == 0 && groups[ng] == n);
    std::vector<int> seen(n, 0);
    uint64_t prev_cost = ~0ull;
    for (uint32_t g = 0; g < ng; ++g) {
      CHECK(groups[g] < groups[g + 1]);
      uint64_t cost = 0;
      int64_t last = -1;
      for (uint32_t k = groups[g]; k < groups[g + 1]; ++k) {
        const xg_request &q = sorted[k];
        CHECK(q.stream == sorted[groups[g]].stream);  // one stream per group
        uint32_t lo = 0, hi = n;                      // find the request by its offset
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) / 2;
          if (reqs[mid].out_offset <= q.out_offset) lo = mid; else hi = mid;
        }
        CHECK(reqs[lo].out_offset == q.out_offset && reqs[lo].n == q.n && reqs[lo].flags == q.flags &&
              reqs[lo].dtype == q.dtype);
        CHECK((int64_t)lo > last);                    // arrival order kept inside a group
        last = lo;
        ++seen[lo];
        cost += q.dtype == XG_NORMAL ? 4 * (q.n + (q.n & 1)) : q.n;
      }
      if (sorted[groups[g]].flags & xg::kReqSegment) CHECK(groups[g + 1] - groups[g] == 1);
      CHECK(cost <= prev_cost);                       // largest group first
      prev_cost = cost;
    }
    for (uint32_t i = 0; i < n; ++i) CHECK(seen[i] == 1);
  }
  // error codes
  xg_request r{3, 10, 0, 0, 0};
  xg_request out[2];
  uint32_t g[3], ng = 0;
  CHECK(xg::plan_batch(&r, 1, 3, 100, out, g, &ng, false) == XG_ERANGE);   // stream
  r.stream = 0;
  CHECK(xg::plan_batch(&r, 1, 3, 9, out, g, &ng, false) == XG_ERANGE);     // output range
  r.out_offset = ~0ull;
  CHECK(xg::plan_batch(&r, 1, 3, 100, out, g, &ng, false) == XG_ERANGE);   // no overflow
  r.out_offset = 0;
  r.dtype = 3;
  CHECK(xg::plan_batch(&r, 1, 3, 100, out, g, &ng, false) == XG_EINVAL);
  r.dtype = 0;
  r.flags = xg::kReqSegment;
  CHECK(xg::plan_batch(&r, 1, 3, 100, out, g, &ng, false) == XG_EINVAL);   // segments not allowed
  CHECK(xg::plan_batch(&r, 1, 3, 100, out, g, &ng, true) == XG_OK && ng == 1);
  r.flags = xg::kReqSegment | 0x4u;
  CHECK(xg::plan_batch(&r, 1, 3, 100, out, g, &ng, true) == XG_EINVAL);    // undefined bits
  CHECK(xg::plan_batch(nullptr, 0, 3, 100, out, g, &ng, false) == XG_OK && ng == 0 && g[0] == 0);
  CHECK(xg::plan_batch(nullptr, 1, 3, 100, out, g, &ng, false) == XG_EINVAL);
  return 0;
}

// Arguments "f:J": the jump polynomial of member f (XG_FAMILY_*) for J.
int main(int argc, char **argv) {
  if (plan_checks()) return 1;
  uint64_t g0[64];
  CHECK(!xg::jump_polynomial(3u, 1, g0) && xg::member_degree(3u) == 0);  // unknown member
  for (int i = 1; i < argc; ++i) {
    char *rest = nullptr;
    const uint32_t f = (uint32_t)std::strtoul(argv[i], &rest, 0);
    CHECK(rest && *rest == ':');
    const uint64_t J = std::strtoull(rest + 1, nullptr, 0);
    const int words = xg::member_degree(f) / 64;
    CHECK(words == 32 || words == 64);
    uint64_t gp[64];
    CHECK(xg::jump_polynomial(f, J, gp));
    if (f == XG_FAMILY_R128_W32) {  // the member-less entry point agrees
      uint64_t gq[64];
      CHECK(xg::jump_polynomial(J, gq));
      for (int w = 0; w < 64; ++w) CHECK(gq[w] == gp[w]);
    }
    std::printf("J %u %" PRIu64 " ", f, J);
    for (int w = words - 1; w >= 0; --w) std::printf("%016" PRIx64, gp[w]);
    std::printf("\n");
  }
  std::printf("OK\n");
  return 0;
}
