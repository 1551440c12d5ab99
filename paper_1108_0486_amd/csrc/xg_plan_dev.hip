// Device-side batch planner of libxg: turns a request table in the caller's
// array order into the table the persistent batch kernels serve.  Requests of
// one stream become one group, kept in array order (that is what makes a
// batched request read the positions it would read alone); a group of one
// long request may become tiles of L words that separate wavefronts run from
// jumped start states (Section 2: independent subsequences of one stream);
// queue items are ordered largest first, so the dynamic queue balances uneven
// lengths.  Everything runs as kernels on the caller's stream, so the call
// needs no host round trip and can be captured in a HIP graph.
//
// Grouping is a sort of 64-bit keys (stream << 32 | request index): the keys
// are distinct, so any correct sort leaves each stream's requests in array
// order.  A bitonic network (compare-exchange passes in LDS within a
// workgroup's 2048 keys, global passes above that) sorts them; the queue items
// are sorted the same way on (inverted cost << 32 | group << 8 | tile).
// Prefix sums are three-kernel block scans.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xg_host.h"
#include "xg_internal.h"
#include "xg_launch.h"
#include "xg_plan_dev.h"

namespace xg {
namespace {

// Keys one workgroup sorts in LDS (1024 threads, two keys each).  8192-key
// blocks (64 KB, eight keys per thread) need fewer launches but measured
// slower: 305 against 249 us of sorting per 65536-request plan.
constexpr uint32_t kSortBlock = 2048;
constexpr uint32_t kScanBlock = 1024;  // elements one scan workgroup covers (256 threads, four each)

// Planner counters (meta words).
constexpr uint32_t kMetaValid = 0;  // requests that passed the checks
constexpr uint32_t kMetaTiles = 1;  // tile slots used (the largest tile prefix sum within max_tiles)
constexpr uint32_t kMetaItems = 2;  // queue items

__device__ __forceinline__ uint64_t words_of(uint64_t n, uint32_t dtype) {
  return dtype == XG_NORMAL ? n + (n & 1u) : n;
}

// Cost of serving n values of dtype in the queue's balance (the host
// planner's measure: words consumed, normals weighted four times for their
// transcendental work).
__device__ __forceinline__ uint64_t cost_of(uint64_t n, uint32_t dtype) {
  return dtype == XG_NORMAL ? 4u * words_of(n, dtype) : n;
}

// Queue item key: larger cost sorts first, then group, then tile.
__device__ __forceinline__ uint64_t item_key(uint64_t cost, uint32_t g, uint32_t k) {
  const uint32_t c = cost > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)cost;
  return ((uint64_t)(0xFFFFFFFFu - c) << 32) | ((uint64_t)g << 8) | k;
}

// ---- bitonic sort of 64-bit keys ------------------------------------------

// One compare-exchange pass of the bitonic network over a[0, n): pair
// (i, i + j) with bit j of i clear, ascending where bit k of i is clear.
__global__ __launch_bounds__(256) void k_bitonic_step(uint64_t *__restrict__ a, uint32_t n, uint32_t k,
                                                      uint32_t j) {
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= n / 2) return;
  const uint32_t i = ((t & ~(j - 1u)) << 1) | (t & (j - 1u));
  const uint32_t l = i | j;
  const bool asc = (i & k) == 0u;
  const uint64_t x = a[i], y = a[l];
  if ((x > y) == asc) {
    a[i] = y;
    a[l] = x;
  }
}

// M consecutive global passes j, j / 2, ..., j / 2^(M-1) of stage k in one
// launch: the 2^M keys whose indices differ only in those M bits are closed
// under these passes (and share the direction, since j < k), so each thread
// loads one such group, runs the M passes in registers and stores it back.
// Consecutive threads take consecutive indices below j / 2^(M-1), so every
// load and store is coalesced.
template <int M>
__global__ __launch_bounds__(256) void k_bitonic_steps(uint64_t *__restrict__ a, uint32_t n, uint32_t k,
                                                       uint32_t j) {
  constexpr uint32_t G = 1u << M;
  const uint32_t t = blockIdx.x * 256u + threadIdx.x;
  if (t >= n / G) return;
  const uint32_t jlo = j >> (M - 1);             // the smallest stride
  const uint32_t i = ((t / jlo) * (jlo * G)) | (t % jlo);  // M zero bits at the strides' positions
  const bool asc = (i & k) == 0u;
  uint64_t v[G];
#pragma unroll
  for (uint32_t b = 0; b < G; ++b) v[b] = a[i + b * jlo];
#pragma unroll
  for (int m = M - 1; m >= 0; --m) {  // stride jlo 2^m: partners differ in bit m of b
#pragma unroll
    for (uint32_t b = 0; b < G; ++b) {
      if (b & (1u << m)) continue;
      const uint32_t c = b | (1u << m);
      const uint64_t x = v[b], y = v[c];
      if ((x > y) == asc) {
        v[b] = y;
        v[c] = x;
      }
    }
  }
#pragma unroll
  for (uint32_t b = 0; b < G; ++b) a[i + b * jlo] = v[b];
}

// The passes with j < kSortBlock, in LDS, on each workgroup's kSortBlock
// keys: the whole network up to k = kSortBlock when k == 0, else the passes
// j = kSortBlock / 2 .. 1 of stage k.  Each of the 1024 threads takes
// kSortBlock / 2048 of a pass's kSortBlock / 2 pairs.
__global__ __launch_bounds__(1024) void k_bitonic_block(uint64_t *__restrict__ a, uint32_t k_stage) {
  constexpr uint32_t kPer = kSortBlock / 1024u, kPairs = kSortBlock / 2048u;
  __shared__ uint64_t s[kSortBlock];
  const uint32_t t = threadIdx.x;
  const uint32_t base = blockIdx.x * kSortBlock;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) s[t + 1024u * q] = a[base + t + 1024u * q];
  __syncthreads();
  const uint32_t k_lo = k_stage ? k_stage : 2u, k_hi = k_stage ? k_stage : kSortBlock;
  for (uint32_t k = k_lo; k <= k_hi; k <<= 1) {
    for (uint32_t j = (k_stage ? kSortBlock : k) >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (uint32_t q = 0; q < kPairs; ++q) {
        const uint32_t pr = t + 1024u * q;  // pair number in the block
        const uint32_t i = ((pr & ~(j - 1u)) << 1) | (pr & (j - 1u));
        const uint32_t l = i | j;
        const bool asc = ((base + i) & k) == 0u;
        const uint64_t x = s[i], y = s[l];
        if ((x > y) == asc) {
          s[i] = y;
          s[l] = x;
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) a[base + t + 1024u * q] = s[t + 1024u * q];
}

// Sorts a[0, n) ascending; n is a power of two >= kSortBlock.  The global
// passes of a stage go three at a time (k_bitonic_steps<3>), then the rest.
hipError_t bitonic_sort(uint64_t *a, uint32_t n, hipStream_t stream) {
  hipError_t e = launch(k_bitonic_block, dim3(n / kSortBlock), dim3(1024), 0, stream, a, 0u);
  for (uint32_t k = 2 * kSortBlock; k <= n && e == hipSuccess; k <<= 1) {
    uint32_t j = k >> 1;
    while (j >= kSortBlock && e == hipSuccess) {
      const uint32_t left = 31u - (uint32_t)__builtin_clz(j / kSortBlock) + 1u;  // passes j .. kSortBlock
      if (left >= 3) {
        e = launch(k_bitonic_steps<3>, dim3((n / 8 + 255) / 256), dim3(256), 0, stream, a, n, k, j);
        j >>= 3;
      } else if (left == 2) {
        e = launch(k_bitonic_steps<2>, dim3((n / 4 + 255) / 256), dim3(256), 0, stream, a, n, k, j);
        j >>= 2;
      } else {
        e = launch(k_bitonic_step, dim3((n / 2 + 255) / 256), dim3(256), 0, stream, a, n, k, j);
        j >>= 1;
      }
    }
    if (e == hipSuccess) e = launch(k_bitonic_block, dim3(n / kSortBlock), dim3(1024), 0, stream, a, k);
  }
  return e;
}

// ---- exclusive prefix sums in place, total at a[n] ---------------------------

// Exclusive scan of the block's 256 values v (one per thread); *total gets
// their sum.  lds holds 256 values.
template <typename T>
__device__ __forceinline__ T block_exclusive(T v, T *lds, T *total) {
  const uint32_t t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (uint32_t d = 1; d < 256u; d <<= 1) {
    const T add = t >= d ? lds[t - d] : T(0);
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  const T incl = lds[t];
  *total = lds[255];
  __syncthreads();  // lds may be reused after this
  return incl - v;
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_reduce(const T *__restrict__ a, uint32_t n, T *__restrict__ sums) {
  __shared__ T lds[256];
  const uint32_t i0 = blockIdx.x * kScanBlock + 4u * threadIdx.x;
  T v = 0;
  for (uint32_t q = 0; q < 4u; ++q)
    if (i0 + q < n) v += a[i0 + q];
  T total;
  (void)block_exclusive(v, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of nb <= 1024 block sums in one workgroup (four per thread).
template <typename T>
__global__ __launch_bounds__(256) void k_scan_sums(T *__restrict__ sums, uint32_t nb) {
  __shared__ T lds[256];
  const uint32_t i0 = 4u * threadIdx.x;
  T x[4], v = 0;
  for (uint32_t q = 0; q < 4u; ++q) {
    x[q] = i0 + q < nb ? sums[i0 + q] : T(0);
    v += x[q];
  }
  T total;
  T run = block_exclusive(v, lds, &total);
  for (uint32_t q = 0; q < 4u; ++q) {
    if (i0 + q < nb) sums[i0 + q] = run;
    run += x[q];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_scan_apply(T *__restrict__ a, uint32_t n, const T *__restrict__ sums,
                                                    uint32_t nb) {
  __shared__ T lds[256];
  const uint32_t i0 = blockIdx.x * kScanBlock + 4u * threadIdx.x;
  T x[4], v = 0;
  for (uint32_t q = 0; q < 4u; ++q) {
    x[q] = i0 + q < n ? a[i0 + q] : T(0);
    v += x[q];
  }
  T total;
  T run = block_exclusive(v, lds, &total) + sums[blockIdx.x];
  for (uint32_t q = 0; q < 4u; ++q) {
    if (i0 + q < n) a[i0 + q] = run;
    run += x[q];
  }
  if (blockIdx.x == nb - 1u && threadIdx.x == 0) a[n] = sums[blockIdx.x] + total;
}

// Exclusive prefix sums of a[0, n) in place and their total at a[n]
// (n <= kPlanMaxElems; sums holds 1024 values of T).
template <typename T>
hipError_t scan(T *a, uint32_t n, T *sums, hipStream_t stream) {
  const uint32_t nb = n ? (n + kScanBlock - 1) / kScanBlock : 1u;
  hipError_t e = launch(k_scan_reduce<T>, dim3(nb), dim3(256), 0, stream, a, n, sums);
  if (e == hipSuccess) e = launch(k_scan_sums<T>, dim3(1), dim3(256), 0, stream, sums, nb);
  if (e == hipSuccess) e = launch(k_scan_apply<T>, dim3(nb), dim3(256), 0, stream, a, n, sums, nb);
  return e;
}

// ---- planner steps -----------------------------------------------------------

__global__ void k_plan_start(uint32_t *__restrict__ work, uint32_t *__restrict__ meta) {
  if (threadIdx.x < 64) {
    work[threadIdx.x] = 0u;
    meta[threadIdx.x] = 0u;
  }
}

// keys[i] for i < key_n: request i's (stream << 32 | i), with stream
// 0xFFFFFFFF (sorted after every valid stream) for a request that fails the
// checks, and all ones past the table.
__global__ __launch_bounds__(256) void k_plan_keys(const xg_request *__restrict__ reqs, uint32_t num_reqs,
                                                   uint64_t num_streams, uint64_t *__restrict__ keys,
                                                   uint32_t key_n, uint32_t *__restrict__ work,
                                                   uint32_t *__restrict__ meta) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= key_n) return;
  uint64_t key = ~0ull;
  bool valid = false;
  if (i < num_reqs) {
    const xg_request q = reqs[i];
    valid = q.stream < num_streams && q.dtype <= XG_NORMAL && q.flags == 0u;
    key = ((valid ? q.stream : 0xFFFFFFFFull) << 32) | i;
    if (!valid) atomicOr(&work[1], 1u);
  }
  keys[i] = key;
  const uint64_t mask = __ballot(valid);
  if ((threadIdx.x & 63u) == 0 && mask) atomicAdd(&meta[kMetaValid], (uint32_t)__popcll(mask));
}

// For sorted position i: heads[i] = 1 where a group starts, costs[i] = the
// request's cost (both 0 past the valid requests).
__global__ __launch_bounds__(256) void k_plan_heads(const xg_request *__restrict__ reqs, uint32_t num_reqs,
                                                    const uint64_t *__restrict__ keys,
                                                    const uint32_t *__restrict__ meta, uint32_t *__restrict__ heads,
                                                    uint64_t *__restrict__ costs) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= num_reqs) return;
  const uint32_t valid = meta[kMetaValid];
  uint32_t head = 0;
  uint64_t cost = 0;
  if (i < valid) {
    const uint64_t k = keys[i];
    head = i == 0 || (k >> 32) != (keys[i - 1] >> 32);
    const xg_request q = reqs[(uint32_t)k];
    cost = cost_of(q.n, q.dtype);
  }
  heads[i] = head;
  costs[i] = cost;
}

// After the scan of heads: hp[g] = first sorted position of group g, and
// hp[G] = the number of valid requests.
__global__ __launch_bounds__(256) void k_plan_groups(uint32_t num_reqs, const uint32_t *__restrict__ heads,
                                                     const uint32_t *__restrict__ meta, uint32_t *__restrict__ hp) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i >= num_reqs) return;
  if (heads[i + 1] != heads[i]) hp[heads[i]] = i;
  if (i == 0) hp[heads[num_reqs]] = meta[kMetaValid];
}

// tiles[g] = the tiles group g asks for: ceil(words / L) for a group of one
// request split into 2 .. kMaxSegments tiles, else 0.
__global__ __launch_bounds__(256) void k_plan_want(const xg_request *__restrict__ reqs, uint32_t num_reqs,
                                                   const uint64_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ heads,
                                                   const uint32_t *__restrict__ hp, uint64_t tile_words,
                                                   uint32_t *__restrict__ tiles) {
  const uint32_t g = blockIdx.x * 256u + threadIdx.x;
  if (g >= num_reqs) return;
  uint32_t want = 0;
  if (g < heads[num_reqs] && tile_words && hp[g + 1] - hp[g] == 1u) {
    const xg_request q = reqs[(uint32_t)keys[hp[g]]];
    const uint64_t parts = (words_of(q.n, q.dtype) + tile_words - 1) / tile_words;
    if (parts > 1 && parts <= kMaxSegments) want = (uint32_t)parts;
  }
  tiles[g] = want;
}

// After the scan of tiles: groups split in order while their tiles fit
// max_tiles slots; meta[kMetaTiles] = the slots so used.
__global__ __launch_bounds__(256) void k_plan_budget(uint32_t num_reqs, const uint32_t *__restrict__ tiles,
                                                     uint32_t max_tiles, uint32_t *__restrict__ meta) {
  const uint32_t g = blockIdx.x * 256u + threadIdx.x;
  if (g > num_reqs) return;
  const uint32_t v = tiles[g];
  if (v <= max_tiles && v) atomicMax(&meta[kMetaTiles], v);
}

__device__ __forceinline__ bool group_split(const uint32_t *tiles, uint32_t g, uint32_t used) {
  return tiles[g + 1] != tiles[g] && tiles[g + 1] <= used;
}

__global__ __launch_bounds__(256) void k_fill_ones(uint64_t *__restrict__ a, uint32_t n) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) a[i] = ~0ull;
}

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t *__restrict__ a, uint32_t n) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) a[i] = 0u;
}

// Queue items: tile k of split group g at slot tiles[g] + k, every other group
// g at tile_cap + g (unused places keep all ones and sort last).
__global__ __launch_bounds__(256) void k_plan_items(const xg_request *__restrict__ reqs, uint32_t num_reqs,
                                                    const uint64_t *__restrict__ keys,
                                                    const uint32_t *__restrict__ heads,
                                                    const uint64_t *__restrict__ costs,
                                                    const uint32_t *__restrict__ hp,
                                                    const uint32_t *__restrict__ tiles, uint64_t tile_words,
                                                    uint32_t tile_cap, uint32_t *__restrict__ meta,
                                                    uint64_t *__restrict__ items) {
  const uint32_t g = blockIdx.x * 256u + threadIdx.x;
  if (g >= num_reqs || g >= heads[num_reqs]) return;
  if (group_split(tiles, g, meta[kMetaTiles])) {
    const xg_request q = reqs[(uint32_t)keys[hp[g]]];
    const uint32_t t = tiles[g + 1] - tiles[g];
    for (uint32_t k = 0; k < t; ++k) {
      const uint64_t first = k * tile_words;
      const uint64_t nk = q.n - first < tile_words ? q.n - first : tile_words;
      items[tiles[g] + k] = item_key(cost_of(nk, q.dtype), g, k);
    }
    atomicAdd(&meta[kMetaItems], t);
  } else {
    items[tile_cap + g] = item_key(costs[hp[g + 1]] - costs[hp[g]], g, 0);
    atomicAdd(&meta[kMetaItems], 1u);
  }
}

// offs[p] = table entries of sorted item p (0 past the items).
__global__ __launch_bounds__(256) void k_plan_counts(uint32_t item_n, const uint64_t *__restrict__ items,
                                                     const uint32_t *__restrict__ hp,
                                                     const uint32_t *__restrict__ tiles,
                                                     const uint32_t *__restrict__ meta, uint32_t *__restrict__ offs) {
  const uint32_t p = blockIdx.x * 256u + threadIdx.x;
  if (p >= item_n) return;
  uint32_t cnt = 0;
  if (p < meta[kMetaItems]) {
    const uint32_t g = (uint32_t)items[p] >> 8;
    cnt = group_split(tiles, g, meta[kMetaTiles]) ? 1u : hp[g + 1] - hp[g];
  }
  offs[p] = cnt;
}

// Table entry e: the j-th request of its item's group, or the item's tile as a
// segment entry.  Entry 0 also publishes the counts for the batch kernel.
__global__ __launch_bounds__(256) void k_plan_emit(const xg_request *__restrict__ reqs,
                                                   const uint64_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ hp,
                                                   const uint32_t *__restrict__ tiles, uint64_t tile_words,
                                                   const uint64_t *__restrict__ items, uint32_t item_n,
                                                   const uint32_t *__restrict__ offs,
                                                   const uint32_t *__restrict__ meta,
                                                   xg_request *__restrict__ table, uint32_t *__restrict__ work) {
  const uint32_t e = blockIdx.x * 256u + threadIdx.x;
  const uint32_t num_items = meta[kMetaItems], entries = offs[item_n];
  if (e == 0) {
    work[2] = num_items;
    work[3] = entries;
  }
  if (e >= entries) return;
  // The item holding entry e: the last p < num_items with offs[p] <= e.
  uint32_t lo = 0, hi = num_items;  // offs[lo] <= e < offs[hi]
  while (hi - lo > 1u) {
    const uint32_t mid = (lo + hi) >> 1;
    if (offs[mid] <= e) lo = mid;
    else hi = mid;
  }
  const uint64_t it = items[lo];
  const uint32_t g = (uint32_t)it >> 8, k = (uint32_t)it & 0xFFu;
  if (group_split(tiles, g, meta[kMetaTiles])) {
    xg_request q = reqs[(uint32_t)keys[hp[g]]];
    const uint64_t first = k * tile_words;
    const uint32_t t = tiles[g + 1] - tiles[g], slot = tiles[g] + k;
    q.n = q.n - first < tile_words ? q.n - first : tile_words;
    q.out_offset += first;
    q.flags = kReqSegment | (k << 8) | (slot << 16) | (k + 1 == t ? kReqLast : 0u);
    table[e] = q;
  } else {
    table[e] = reqs[(uint32_t)keys[hp[g] + (e - offs[lo])]];
  }
}

// ---- small tables: the whole plan in one workgroup ---------------------------

// Table entries plus tile slots that one workgroup of 1024 threads plans in
// LDS with a single launch instead of the multi-kernel sequence above (the
// plan is the same): EPT consecutive elements per thread, EPT = 1, 2 or 4, at
// most 4096 elements (128 KB of LDS; gfx950 gives a workgroup 160 KB).
constexpr uint32_t kPlanThreads = 1024;
constexpr uint32_t kSmallPlanMax = 4 * kPlanThreads;

// Exclusive prefix sums of the workgroup's values, EPT consecutive ones per
// thread (v[e] is element EPT t + e): on return v[e] holds the sum of every
// element before it, and *total the sum of all.  wsum holds 16 values of T.
template <typename T, int EPT>
__device__ __forceinline__ void wg_exclusive(T (&v)[EPT], T *wsum, T *total) {
  const uint32_t t = threadIdx.x, lane = t & 63u, w = t >> 6;
  T mine = 0;
#pragma unroll
  for (int e = 0; e < EPT; ++e) mine += v[e];
  T x = mine;
#pragma unroll
  for (uint32_t d = 1; d < 64u; d <<= 1) {
    const T y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63u) wsum[w] = x;
  __syncthreads();
  if (w == 0) {
    T s = lane < 16u ? wsum[lane] : T(0);
#pragma unroll
    for (uint32_t d = 1; d < 16u; d <<= 1) {
      const T y = __shfl_up(s, d);
      if (lane >= d) s += y;
    }
    if (lane < 16u) wsum[lane] = s;
  }
  __syncthreads();
  T run = (w ? wsum[w - 1] : T(0)) + x - mine;
  *total = wsum[15];
  __syncthreads();  // wsum is reused by the next scan
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const T here = v[e];
    v[e] = run;
    run += here;
  }
}

// Ascending bitonic sort of N keys in LDS (EPT / 2 pairs per thread and pass,
// or half the threads with one pair each when EPT == 1).
template <uint32_t N>
__device__ __forceinline__ void wg_sort(uint64_t *s) {
  const uint32_t t = threadIdx.x;
  constexpr uint32_t kPairs = N / 2;
  for (uint32_t k = 2; k <= N; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (uint32_t pr = t; pr < kPairs; pr += kPlanThreads) {
        const uint32_t i = ((pr & ~(j - 1u)) << 1) | (pr & (j - 1u));
        const uint32_t l = i | j;
        const bool asc = (i & k) == 0u;
        const uint64_t x = s[i], y = s[l];
        if ((x > y) == asc) {
          s[i] = y;
          s[l] = x;
        }
      }
      __syncthreads();
    }
  }
}

// The planner for num_reqs + tile_cap <= N = 1024 EPT: the steps of the
// kernels above (keys, sort, group heads and cost sums, tiles and their
// budget, queue items, their sort, entry counts, table) on EPT consecutive
// elements per thread, with the arrays in LDS.  Writes offs[0 .. num_reqs +
// tile_cap], the table and work[0 .. 63] (counts in work[2], work[3], the
// error word in work[1]).
template <int EPT>
__global__ __launch_bounds__(kPlanThreads) void k_plan_small(const xg_request *__restrict__ reqs,
                                                             uint32_t num_reqs, uint64_t num_streams,
                                                             uint64_t tile_words, uint32_t tile_cap,
                                                             uint32_t *__restrict__ work,
                                                             uint32_t *__restrict__ offs_out,
                                                             xg_request *__restrict__ table) {
  constexpr uint32_t N = kPlanThreads * EPT;
  __shared__ uint64_t keys[N];       // sort keys, then queue item keys
  __shared__ uint64_t costs[N + 1];  // cost prefix sums over sorted requests
  __shared__ uint32_t idx[N];        // request index at each sorted position
  __shared__ uint32_t heads[N + 1];  // group prefix sums, then entry offsets of items
  __shared__ uint32_t hp[N + 1];     // first sorted position of each group
  __shared__ uint32_t tiles[N + 1];  // tile prefix sums per group
  __shared__ uint64_t wsum[16];
  __shared__ uint32_t cnt[4];        // valid requests, error, tile slots used, items
  const uint32_t t = threadIdx.x, n = num_reqs, i0 = t * EPT;
  uint32_t *wsum32 = reinterpret_cast<uint32_t *>(wsum);
  if (t >= 4u && t < 64u) work[t] = 0u;
  if (t < 4u) cnt[t] = 0u;
  __syncthreads();

#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const uint32_t i = i0 + e;
    uint64_t key = ~0ull;
    if (i < n) {
      const xg_request q = reqs[i];
      const bool valid = q.stream < num_streams && q.dtype <= XG_NORMAL && q.flags == 0u;
      key = ((valid ? q.stream : 0xFFFFFFFFull) << 32) | i;
      if (valid) atomicAdd(&cnt[0], 1u);
      else atomicOr(&cnt[1], 1u);
    }
    keys[i] = key;
  }
  __syncthreads();
  wg_sort<N>(keys);

  const uint32_t valid_n = cnt[0];
  uint32_t head[EPT], hx[EPT];
  uint64_t cx[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const uint32_t i = i0 + e;
    const uint64_t k = keys[i];
    idx[i] = (uint32_t)k;
    head[e] = 0;
    cx[e] = 0;
    if (i < valid_n) {
      head[e] = i == 0 || (k >> 32) != (keys[i - 1] >> 32);
      const xg_request q = reqs[(uint32_t)k];
      cx[e] = cost_of(q.n, q.dtype);
    }
    hx[e] = head[e];
  }
  uint32_t num_groups;
  wg_exclusive<uint32_t, EPT>(hx, wsum32, &num_groups);
  uint64_t cost_total;
  wg_exclusive<uint64_t, EPT>(cx, wsum, &cost_total);
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    heads[i0 + e] = hx[e];
    costs[i0 + e] = cx[e];
  }
  if (t == kPlanThreads - 1u) {
    heads[N] = num_groups;
    costs[N] = cost_total;
  }
  __syncthreads();
#pragma unroll
  for (int e = 0; e < EPT; ++e)
    if (i0 + e < n && head[e]) hp[hx[e]] = i0 + e;
  if (t == 0) hp[num_groups] = valid_n;
  __syncthreads();

  uint32_t want[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const uint32_t g = i0 + e;
    want[e] = 0;
    if (tile_cap && g < num_groups && hp[g + 1] - hp[g] == 1u) {
      const xg_request q = reqs[idx[hp[g]]];
      const uint64_t parts = (words_of(q.n, q.dtype) + tile_words - 1) / tile_words;
      if (parts > 1 && parts <= kMaxSegments) want[e] = (uint32_t)parts;
    }
  }
  uint32_t tile_total;
  wg_exclusive<uint32_t, EPT>(want, wsum32, &tile_total);
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    tiles[i0 + e] = want[e];
    if (want[e] && want[e] <= tile_cap) atomicMax(&cnt[2], want[e]);
  }
  if (t == kPlanThreads - 1u) tiles[N] = tile_total;
  if (t == 0 && tile_total && tile_total <= tile_cap) atomicMax(&cnt[2], tile_total);
#pragma unroll
  for (int e = 0; e < EPT; ++e) keys[i0 + e] = ~0ull;  // idx holds the request indices now
  __syncthreads();

  const uint32_t used = cnt[2];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const uint32_t g = i0 + e;
    if (g >= num_groups) continue;
    if (group_split(tiles, g, used)) {
      const xg_request q = reqs[idx[hp[g]]];
      const uint32_t parts = tiles[g + 1] - tiles[g];
      for (uint32_t k = 0; k < parts; ++k) {
        const uint64_t first = k * tile_words;
        const uint64_t nk = q.n - first < tile_words ? q.n - first : tile_words;
        keys[tiles[g] + k] = item_key(cost_of(nk, q.dtype), g, k);
      }
      atomicAdd(&cnt[3], parts);
    } else {
      keys[tile_cap + g] = item_key(costs[hp[g + 1]] - costs[hp[g]], g, 0);
      atomicAdd(&cnt[3], 1u);
    }
  }
  __syncthreads();
  wg_sort<N>(keys);

  const uint32_t num_items = cnt[3];
  uint32_t ox[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const uint32_t q = i0 + e;
    ox[e] = 0;
    if (q < num_items) {
      const uint32_t g = (uint32_t)keys[q] >> 8;
      ox[e] = group_split(tiles, g, used) ? 1u : hp[g + 1] - hp[g];
    }
  }
  uint32_t entries;
  wg_exclusive<uint32_t, EPT>(ox, wsum32, &entries);
  const uint32_t items = n + tile_cap;
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    heads[i0 + e] = ox[e];  // heads now holds the items' table offsets
    if (i0 + e <= items) offs_out[i0 + e] = ox[e];
  }
  if (t == kPlanThreads - 1u) {
    heads[N] = entries;
    if (items == N) offs_out[N] = entries;
  }
  __syncthreads();

#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const uint32_t en = i0 + e;
    if (en >= entries) continue;
    uint32_t lo = 0, hi = num_items;  // heads[lo] <= en < heads[hi]
    while (hi - lo > 1u) {
      const uint32_t mid = (lo + hi) >> 1;
      if (heads[mid] <= en) lo = mid;
      else hi = mid;
    }
    const uint64_t it = keys[lo];
    const uint32_t g = (uint32_t)it >> 8, k = (uint32_t)it & 0xFFu;
    if (group_split(tiles, g, used)) {
      xg_request q = reqs[idx[hp[g]]];
      const uint64_t first = k * tile_words;
      const uint32_t parts = tiles[g + 1] - tiles[g], slot = tiles[g] + k;
      q.n = q.n - first < tile_words ? q.n - first : tile_words;
      q.out_offset += first;
      q.flags = kReqSegment | (k << 8) | (slot << 16) | (k + 1 == parts ? kReqLast : 0u);
      table[en] = q;
    } else {
      table[en] = reqs[idx[hp[g] + (en - heads[lo])]];
    }
  }
  if (t == 0) {
    work[0] = 0u;
    work[1] = cnt[1];
    work[2] = num_items;
    work[3] = entries;
  }
}

uint32_t pow2_at_least(uint32_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

}  // namespace

PlanLayout plan_layout(uint32_t max_reqs, uint32_t max_tiles, uint32_t state_bytes, uint32_t jump_bytes) {
  PlanLayout l;
  l.key_cap = pow2_at_least(max_reqs > kSortBlock ? max_reqs : kSortBlock);
  const uint32_t items = max_reqs + max_tiles;
  l.item_cap = pow2_at_least(items > kSortBlock ? items : kSortBlock);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  l.work = take(256);
  l.meta = take(256);
  l.keys = take((size_t)l.key_cap * 8);
  l.heads = take(((size_t)max_reqs + 1) * 4);
  l.costs = take(((size_t)max_reqs + 1) * 8);
  l.hp = take(((size_t)max_reqs + 1) * 4);
  l.tiles = take(((size_t)max_reqs + 1) * 4);
  l.items = take((size_t)l.item_cap * 8);
  l.offs = take(((size_t)items + 1) * 4);
  l.table = take((size_t)items * sizeof(xg_request));
  l.sums = take(1024 * 8);
  l.stage = take((size_t)max_tiles * state_bytes);
  l.jump = take(max_tiles ? (size_t)(kMaxSegments - 1) * jump_bytes : 0);
  l.total = o;
  return l;
}

PlanPtrs plan_ptrs(void *base, const PlanLayout &l) {
  char *b = static_cast<char *>(base);
  PlanPtrs p;
  p.work = reinterpret_cast<uint32_t *>(b + l.work);
  p.meta = reinterpret_cast<uint32_t *>(b + l.meta);
  p.keys = reinterpret_cast<uint64_t *>(b + l.keys);
  p.heads = reinterpret_cast<uint32_t *>(b + l.heads);
  p.costs = reinterpret_cast<uint64_t *>(b + l.costs);
  p.hp = reinterpret_cast<uint32_t *>(b + l.hp);
  p.tiles = reinterpret_cast<uint32_t *>(b + l.tiles);
  p.items = reinterpret_cast<uint64_t *>(b + l.items);
  p.offs = reinterpret_cast<uint32_t *>(b + l.offs);
  p.table = reinterpret_cast<xg_request *>(b + l.table);
  p.sums = reinterpret_cast<uint64_t *>(b + l.sums);
  p.stage = reinterpret_cast<uint32_t *>(b + l.stage);
  p.jump = reinterpret_cast<uint64_t *>(b + l.jump);
  return p;
}

hipError_t launch_plan(const PlanPtrs &p, const PlanLayout &l, const xg_request *reqs, uint32_t num_reqs,
                       uint64_t num_streams, uint64_t tile_words, uint32_t max_tiles, hipStream_t stream) {
  const uint32_t tile_cap = tile_words ? max_tiles : 0u;
  const uint64_t elems = (uint64_t)num_reqs + tile_cap;
  if (elems <= kSmallPlanMax) {
    if (elems + 1 > (uint64_t)(l.table - l.offs) / 4) return hipErrorInvalidValue;
    auto run = [&](auto kernel) {
      return launch(kernel, dim3(1), dim3(kPlanThreads), 0, stream, reqs, num_reqs, num_streams, tile_words,
                    tile_cap, p.work, p.offs, p.table);
    };
    if (elems <= kPlanThreads) return run(k_plan_small<1>);
    if (elems <= 2 * kPlanThreads) return run(k_plan_small<2>);
    return run(k_plan_small<4>);
  }
  const uint32_t key_n = pow2_at_least(num_reqs > kSortBlock ? num_reqs : kSortBlock);
  const uint32_t items = num_reqs + tile_cap;
  const uint32_t item_n = pow2_at_least(items > kSortBlock ? items : kSortBlock);
  if (key_n > l.key_cap || item_n > l.item_cap || items > kPlanMaxElems) return hipErrorInvalidValue;
  const dim3 b256(256);
  auto grid = [](uint32_t n) { return dim3(n ? (n + 255) / 256 : 1u); };
  uint32_t *u32sums = reinterpret_cast<uint32_t *>(p.sums);
  hipError_t e = launch(k_plan_start, dim3(1), dim3(64), 0, stream, p.work, p.meta);
  if (e == hipSuccess)
    e = launch(k_plan_keys, grid(key_n), b256, 0, stream, reqs, num_reqs, num_streams, p.keys, key_n, p.work, p.meta);
  if (e == hipSuccess) e = bitonic_sort(p.keys, key_n, stream);
  if (e == hipSuccess)
    e = launch(k_plan_heads, grid(num_reqs), b256, 0, stream, reqs, num_reqs, p.keys, p.meta, p.heads, p.costs);
  if (e == hipSuccess) e = scan<uint32_t>(p.heads, num_reqs, u32sums, stream);
  if (e == hipSuccess) e = scan<uint64_t>(p.costs, num_reqs, p.sums, stream);
  if (e == hipSuccess) e = launch(k_plan_groups, grid(num_reqs), b256, 0, stream, num_reqs, p.heads, p.meta, p.hp);
  if (tile_cap) {
    if (e == hipSuccess)
      e = launch(k_plan_want, grid(num_reqs), b256, 0, stream, reqs, num_reqs, p.keys, p.heads, p.hp, tile_words,
                 p.tiles);
    if (e == hipSuccess) e = scan<uint32_t>(p.tiles, num_reqs, u32sums, stream);
    if (e == hipSuccess)
      e = launch(k_plan_budget, grid(num_reqs + 1), b256, 0, stream, num_reqs, p.tiles, tile_cap, p.meta);
  } else if (e == hipSuccess) {
    // no tiles: every group's tile prefix sum is 0
    e = launch(k_fill_zero, grid(num_reqs + 1), b256, 0, stream, p.tiles, num_reqs + 1);
  }
  if (e == hipSuccess) e = launch(k_fill_ones, grid(item_n), b256, 0, stream, p.items, item_n);
  if (e == hipSuccess)
    e = launch(k_plan_items, grid(num_reqs), b256, 0, stream, reqs, num_reqs, p.keys, p.heads, p.costs, p.hp,
               p.tiles, tile_words, tile_cap, p.meta, p.items);
  if (e == hipSuccess) e = bitonic_sort(p.items, item_n, stream);
  if (e == hipSuccess)
    e = launch(k_plan_counts, grid(items), b256, 0, stream, items, p.items, p.hp, p.tiles, p.meta, p.offs);
  if (e == hipSuccess) e = scan<uint32_t>(p.offs, items, u32sums, stream);
  if (e == hipSuccess)
    e = launch(k_plan_emit, grid(items), b256, 0, stream, reqs, p.keys, p.hp, p.tiles, tile_words, p.items, items,
               p.offs, p.meta, p.table, p.work);
  return e;
}

}  // namespace xg
