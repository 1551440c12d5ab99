// Request server of libxg (include/xg.h, "serving"): continuous batching of
// (stream, n, dtype) requests over device-resident streams.
//
// One host thread drives it through xg_server_poll:
//   reap    - a lane whose event has fired has finished its batch: its
//             requests complete and their streams become free;
//   admit   - pending requests are taken in submission order; a request waits
//             while its stream is inside a batch still in flight, and admission
//             stops at the first request whose output does not fit in the pool
//             (memory admission, no overtaking);
//   launch  - the admitted set is planned (same-stream requests grouped in
//             order, largest groups first), copied to the lane's device table and
//             served by one persistent batched launch on the lane's HIP stream.
// Lanes are independent HIP streams, so a batch admitted while others run
// overlaps with them on the device.  A stream is never in two in-flight
// batches, so every request reads the exact positions it would read alone.
// With segment_words = L, a request of more than L words becomes segments of
// L words, each its own group (so separate wavefronts run them at once):
// segment k starts from the request's start state jumped by k L words, staged
// before the batch kernel; only the last one writes the stream's end state.
// A split request is alone on its stream within its batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <deque>
#include <new>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "xg.h"
#include "xg_internal.h"
#include "xg_pool.h"
#include "xg_fam_batch.h"

namespace {

constexpr size_t kAlignBytes = 256;

uint64_t now_ns() {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

uint64_t words_consumed(uint64_t n, uint32_t dtype) { return dtype == XG_NORMAL ? n + (n & 1) : n; }

struct Pending {
  uint64_t id, stream, n;
  uint32_t dtype;
  uint64_t t_submit;
};

struct Lane {
  uint32_t *d_stage = nullptr;   // max_batch staged start states (segments)
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  bool busy = false;
  xg_request *h_reqs = nullptr;  // pinned staging
  uint32_t *h_groups = nullptr;
  xg_request *h_scratch = nullptr;
  xg_request *d_reqs = nullptr;  // in the caller's table buffer
  uint32_t *d_groups = nullptr;
  uint32_t *d_work = nullptr;
  std::vector<xg_completion> reqs;
  uint64_t t_launch = 0;
};

struct TableLayout {
  size_t reqs, groups, work, stage, per_lane, jump;
};

// Jump table entries: z^(k L) mod P for k = 1 .. kMaxSegments - 1.
constexpr uint32_t kJumpEntries = xg::kMaxSegments - 1;

TableLayout table_layout(const xg_server_config *c) {
  TableLayout t;
  t.reqs = round_up((size_t)c->max_batch * sizeof(xg_request), kAlignBytes);
  t.groups = round_up(((size_t)c->max_batch + 1) * sizeof(uint32_t), kAlignBytes);
  t.work = round_up(xg_batch_workspace_bytes(), kAlignBytes);
  t.stage = c->segment_words ? round_up((size_t)c->max_batch * XG_STATE_WORDS * 4, kAlignBytes) : 0;
  t.per_lane = t.reqs + t.groups + t.work + t.stage;
  t.jump = c->segment_words ? (size_t)kJumpEntries * 64 * sizeof(uint64_t) : 0;
  return t;
}

bool config_valid(const xg_server_config *c) {
  const bool seg_ok = c && (c->segment_words == 0 ||
                            (c->segment_words % 64 == 0 && c->segment_words >= (1ull << 12) &&
                             c->segment_words <= (1ull << 30)));
  return c && seg_ok && c->num_lanes >= 1 && c->num_lanes <= 8 && c->max_batch >= 1 && c->max_batch <= 65536;
}

}  // namespace

struct xg_server {
  xg_ctx *ctx = nullptr;
  uint64_t seg_words = 0;            // 0: no splitting
  uint64_t *d_jump = nullptr;        // kJumpEntries x 64 words
  uint32_t *d_pool = nullptr;
  uint64_t pool_elems = 0;
  uint32_t max_batch = 0;
  xg_tune tune{};
  bool default_tune = true;
  xg::Pool pool{0};
  std::vector<Lane> lanes;
  std::deque<Pending> pending;
  // 0 free; 1 inside an in-flight batch; 2 in the batch being built;
  // 3 in the batch being built as a split request (closed to further requests)
  std::vector<uint8_t> busy_stream;
  std::vector<uint64_t> pos;          // each stream's position after all admitted work
  std::unordered_map<uint64_t, std::pair<uint64_t, uint64_t>> finished;  // id -> (offset, n)
  std::unordered_set<uint64_t> live;  // ids submitted and not yet released
  std::deque<xg_completion> ready;    // completions not yet handed out
  xg_server_stats stats{};
  uint64_t outstanding = 0;
  // Set when a poll fails part-way (a HIP error, or no memory while moving
  // requests between queues): the host view of streams, pool and queues may
  // then disagree with the device, so every later call but destroy refuses.
  xg_status failed = XG_OK;
};

namespace {

void destroy_lanes(xg_server *s) {
  for (Lane &l : s->lanes) {
    if (l.stream) (void)hipStreamSynchronize(l.stream);
    if (l.done) (void)hipEventDestroy(l.done);
    if (l.stream) (void)hipStreamDestroy(l.stream);
    if (l.h_reqs) (void)hipHostFree(l.h_reqs);
    if (l.h_groups) (void)hipHostFree(l.h_groups);
    delete[] l.h_scratch;
  }
  s->lanes.clear();
}

// Reaps lanes whose batch has finished.
xg_status reap(xg_server *s) {
  for (uint32_t li = 0; li < s->lanes.size(); ++li) {
    Lane &l = s->lanes[li];
    if (!l.busy) continue;
    const hipError_t q = hipEventQuery(l.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) return XG_EHIP;
    const uint64_t t = now_ns();
    for (xg_completion &c : l.reqs) {
      c.t_done_ns = t;
      s->busy_stream[c.stream] = 0;
      s->finished[c.id] = {c.out_offset, c.n};
      s->ready.push_back(c);
      ++s->stats.completed;
      --s->outstanding;
    }
    l.reqs.clear();
    l.busy = false;
  }
  return XG_OK;
}

// Admits pending requests into lane l and launches them; returns the number
// admitted (0: nothing to do).
xg_status admit_and_launch(xg_server *s, uint32_t li, uint32_t *admitted) {
  Lane &l = s->lanes[li];
  *admitted = 0;
  std::vector<uint64_t> in_this_batch;
  uint32_t k = 0, nreq = 0;
  bool any_split = false;
  bool waited = false;
  for (auto it = s->pending.begin(); it != s->pending.end() && k < s->max_batch;) {
    const Pending &p = *it;
    const uint8_t bs = s->busy_stream[p.stream];
    const uint64_t words = words_consumed(p.n, p.dtype);
    const uint64_t parts = s->seg_words ? (words + s->seg_words - 1) / s->seg_words : 1;
    // Split only when the segments fit one table (and the jump table): a request of
    // more parts than max_batch would otherwise never be admitted.  Others run unsplit.
    const bool split = parts > 1 && parts <= xg::kMaxSegments && parts <= s->max_batch;
    const uint64_t nseg = split ? parts : 1;
    // Wait (keeping this stream's order) when the stream is busy elsewhere,
    // closed by a split request in this batch, or would mix a split request
    // with others in this batch.
    if (bs == 1 || bs == 3) {
      ++it;
      continue;
    }
    if (split && bs == 2) {
      // The split request waits for a later batch, so every later request on
      // its stream must wait too: close the stream for the rest of this pass
      // (it is already listed in in_this_batch and becomes busy after it).
      s->busy_stream[p.stream] = 3;
      ++it;
      continue;
    }
    if (k + nseg > s->max_batch) break;
    const uint64_t off = s->pool.alloc(p.n);
    if (off == UINT64_MAX) {
      waited = true;
      break;
    }
    if (bs == 0) in_this_batch.push_back(p.stream);
    s->busy_stream[p.stream] = split ? 3 : 2;
    xg_completion c{};
    c.id = p.id;
    c.stream = p.stream;
    c.n = p.n;
    c.dtype = p.dtype;
    c.out_offset = off;
    c.start_pos = s->pos[p.stream];
    c.t_submit_ns = p.t_submit;
    c.lane = li;
    s->pos[p.stream] += words;
    if (!split) {
      l.h_scratch[k++] = xg_request{p.stream, p.n, off, p.dtype, 0};
    } else {
      // Segment j's start state goes to staging slot k (its place in
      // this table before planning; k < max_batch <= 65536).
      any_split = true;
      for (uint64_t j = 0; j < nseg; ++j) {
        const uint64_t first = j * s->seg_words;
        const uint64_t n_j = std::min<uint64_t>(s->seg_words, p.n - first);
        uint32_t flags = xg::kReqSegment | ((uint32_t)j << 8) | (k << 16);
        if (j + 1 == nseg) flags |= xg::kReqLast;
        l.h_scratch[k++] = xg_request{p.stream, n_j, off + first, p.dtype, flags};
      }
    }
    l.reqs.push_back(c);
    ++nreq;
    it = s->pending.erase(it);
  }
  if (waited) ++s->stats.admission_waits;
  for (uint64_t st : in_this_batch) s->busy_stream[st] = 1;
  if (k == 0) return XG_OK;
  uint32_t num_groups = 0;
  xg_status st = xg::plan_batch(l.h_scratch, k, s->ctx->num_streams, s->pool_elems, l.h_reqs, l.h_groups,
                                &num_groups, true);
  if (st != XG_OK) return st;
  if (hipMemcpyAsync(l.d_reqs, l.h_reqs, (size_t)k * sizeof(xg_request), hipMemcpyHostToDevice, l.stream) !=
          hipSuccess ||
      hipMemcpyAsync(l.d_groups, l.h_groups, ((size_t)num_groups + 1) * sizeof(uint32_t),
                     hipMemcpyHostToDevice, l.stream) != hipSuccess)
    return XG_EHIP;
  xg::Shape shape = xg::default_batch_shape(num_groups, s->ctx->num_cus);
  if (!s->default_tune)
    shape = xg::Shape{s->tune.waves_per_block, s->tune.unroll, s->tune.blocks_per_cu,
                      s->tune.store_words ? s->tune.store_words : (s->tune.unroll >= 4 ? 4u : 1u)};
  if (xg::launch_work_init(l.d_work, num_groups, k, l.stream) != hipSuccess) return XG_EHIP;
  if (s->ctx->family != XG_FAMILY_R128_W32) {  // a further member (no segments)
    if (xg::launch_family_batch(s->ctx->family, shape, s->ctx->num_cus,
                                reinterpret_cast<unsigned char *>(s->ctx->d_state), s->ctx->num_streams, l.d_reqs,
                                l.d_groups, num_groups, s->d_pool, s->pool_elems, l.d_work, l.stream) != hipSuccess)
      return XG_EHIP;
  } else {
    const xg::SegmentArgs seg{s->d_jump, s->seg_words, s->d_jump ? kJumpEntries : 0u, l.d_stage, s->max_batch};
    if (any_split &&
        xg::launch_seg_starts(s->ctx->d_state, s->ctx->num_streams, l.d_reqs, k, l.d_work, seg, s->ctx->num_cus,
                              l.stream) != hipSuccess)
      return XG_EHIP;
    if (xg::launch_batch(shape, s->ctx->num_cus, s->ctx->d_state, s->ctx->num_streams, l.d_reqs, l.d_groups,
                         num_groups, s->d_pool, s->pool_elems, l.d_work, l.stream,
                         s->seg_words ? &seg : nullptr) != hipSuccess)
      return XG_EHIP;
  }
  if (hipEventRecord(l.done, l.stream) != hipSuccess) return XG_EHIP;
  l.t_launch = now_ns();
  for (xg_completion &c : l.reqs) c.t_launch_ns = l.t_launch;
  l.busy = true;
  *admitted = nreq;
  ++s->stats.batches;
  s->stats.admitted += nreq;
  s->stats.max_batch_seen = std::max<uint64_t>(s->stats.max_batch_seen, nreq);
  s->stats.pool_high_water = std::max<uint64_t>(s->stats.pool_high_water, s->pool.used());
  uint64_t busy = 0;
  for (const Lane &x : s->lanes) busy += x.busy;
  s->stats.max_lanes_busy = std::max<uint64_t>(s->stats.max_lanes_busy, busy);
  return XG_OK;
}

}  // namespace

extern "C" {

size_t xg_server_device_bytes(const xg_server_config *cfg) {
  if (!config_valid(cfg)) return 0;
  const TableLayout t = table_layout(cfg);
  return t.per_lane * cfg->num_lanes + t.jump;
}

xg_status xg_server_create(xg_server **out, xg_ctx *ctx, const xg_server_config *cfg, void *d_pool,
                           uint64_t pool_elems, void *d_tables, size_t tables_bytes) {
  if (!out) return XG_EINVAL;
  *out = nullptr;
  if (!ctx || !config_valid(cfg) || !d_pool || !d_tables || pool_elems < xg::kPoolAlignElems) return XG_EINVAL;
  // The further members are served without jump-ahead segments.
  if (ctx->family != XG_FAMILY_R128_W32 &&
      ((ctx->family != XG_FAMILY_R64_W32 && ctx->family != XG_FAMILY_R64_W64) || cfg->segment_words != 0))
    return XG_ENOTSUP;
  if (tables_bytes < xg_server_device_bytes(cfg)) return XG_ERANGE;
  if (reinterpret_cast<uintptr_t>(d_pool) % kAlignBytes || reinterpret_cast<uintptr_t>(d_tables) % kAlignBytes)
    return XG_EALIGN;
  bool default_tune = cfg->tune.waves_per_block == 0 && cfg->tune.unroll == 0 &&
                      cfg->tune.blocks_per_cu == 0 && cfg->tune.store_words == 0;
  xg_tune tune = cfg->tune;
  if (default_tune && cfg->tune_key) {  // the tuning cache's shape for this device, member and key
    const xg_status st = xg_tune_cache_get(ctx->arch, (uint32_t)ctx->num_cus, ctx->family, cfg->tune_key, &tune,
                                           nullptr);
    if (st == XG_EINVAL || st == XG_ENOMEM) return st;
    default_tune = st != XG_OK;
  }
  if (!default_tune) {
    xg::Shape sh{tune.waves_per_block, tune.unroll, tune.blocks_per_cu,
                 tune.store_words ? tune.store_words : (tune.unroll >= 4 ? 4u : 1u)};
    if (!xg::shape_valid(sh)) return XG_EINVAL;
  }
  xg_server *s = new (std::nothrow) xg_server;
  if (!s) return XG_ENOMEM;
  try {
    s->ctx = ctx;
    s->d_pool = static_cast<uint32_t *>(d_pool);
    s->pool_elems = pool_elems;
    s->max_batch = cfg->max_batch;
    s->tune = tune;
    s->default_tune = default_tune;
    s->pool = xg::Pool(pool_elems);
    s->busy_stream.assign(ctx->num_streams, 0);
    s->pos.assign(ctx->num_streams, 0);
    s->lanes.resize(cfg->num_lanes);
  } catch (const std::bad_alloc &) {
    delete s;
    return XG_ENOMEM;
  }
  // Positions of every stream (and completion of any prior work on the state).
  if (hipDeviceSynchronize() != hipSuccess) {
    delete s;
    return XG_EHIP;
  }
  {
    const size_t per = xg::family_state_bytes(ctx->family);
    const size_t pos_off = xg::family_pos_offset(ctx->family);
    std::vector<unsigned char> state;
    try {
      state.resize((size_t)ctx->num_streams * per);
    } catch (const std::bad_alloc &) {
      delete s;
      return XG_ENOMEM;
    }
    if (hipMemcpy(state.data(), ctx->d_state, state.size(), hipMemcpyDeviceToHost) != hipSuccess) {
      delete s;
      return XG_EHIP;
    }
    for (uint64_t i = 0; i < ctx->num_streams; ++i) std::memcpy(&s->pos[i], state.data() + i * per + pos_off, 8);
  }
  const TableLayout tl = table_layout(cfg);
  char *base = static_cast<char *>(d_tables);
  if (cfg->segment_words) {
    // z^(k L) mod P for k = 1 .. kJumpEntries, computed on the host once.
    s->seg_words = cfg->segment_words;
    s->d_jump = reinterpret_cast<uint64_t *>(base + tl.per_lane * cfg->num_lanes);
    std::vector<uint64_t> table;
    try {
      table.resize((size_t)kJumpEntries * 64);
    } catch (const std::bad_alloc &) {
      delete s;
      return XG_ENOMEM;
    }
    if (!xg::jump_table(XG_FAMILY_R128_W32, cfg->segment_words, kJumpEntries, table.data())) {
      delete s;
      return XG_ENOTSUP;
    }
    if (hipMemcpy(s->d_jump, table.data(), table.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess) {
      delete s;
      return XG_EHIP;
    }
  }
  for (uint32_t li = 0; li < cfg->num_lanes; ++li) {
    Lane &l = s->lanes[li];
    char *lb = base + li * tl.per_lane;
    l.d_reqs = reinterpret_cast<xg_request *>(lb);
    l.d_groups = reinterpret_cast<uint32_t *>(lb + tl.reqs);
    l.d_work = reinterpret_cast<uint32_t *>(lb + tl.reqs + tl.groups);
    l.d_stage = tl.stage ? reinterpret_cast<uint32_t *>(lb + tl.reqs + tl.groups + tl.work) : nullptr;
    l.h_scratch = new (std::nothrow) xg_request[cfg->max_batch];
    bool reserved = l.h_scratch != nullptr;
    try {
      if (reserved) l.reqs.reserve(cfg->max_batch);
    } catch (const std::bad_alloc &) {
      reserved = false;
    }
    if (!reserved) {
      destroy_lanes(s);
      delete s;
      return XG_ENOMEM;
    }
    if (hipStreamCreateWithFlags(&l.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&l.h_reqs), (size_t)cfg->max_batch * sizeof(xg_request),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&l.h_groups), ((size_t)cfg->max_batch + 1) * sizeof(uint32_t),
                      hipHostMallocDefault) != hipSuccess) {
      destroy_lanes(s);
      delete s;
      return XG_EHIP;
    }
  }
  *out = s;
  return XG_OK;
}

xg_status xg_server_submit(xg_server *s, uint64_t id, uint64_t stream, uint64_t n, uint32_t dtype) {
  if (!s || n == 0 || dtype > XG_NORMAL) return XG_EINVAL;
  if (s->failed != XG_OK) return s->failed;
  if (stream >= s->ctx->num_streams || xg::round_elems(n) > s->pool.capacity()) return XG_ERANGE;
  if (s->live.count(id)) return XG_EINVAL;
  try {
    s->live.insert(id);
    s->pending.push_back(Pending{id, stream, n, dtype, now_ns()});
  } catch (const std::bad_alloc &) {
    s->live.erase(id);
    return XG_ENOMEM;
  }
  ++s->stats.submitted;
  ++s->outstanding;
  return XG_OK;
}

namespace {

xg_status poll_body(xg_server *s, xg_completion *out, uint32_t max_out, uint32_t *num_out) {
  xg_status st = reap(s);
  if (st != XG_OK) return st;
  for (uint32_t li = 0; li < s->lanes.size() && !s->pending.empty(); ++li) {
    if (s->lanes[li].busy) continue;
    uint32_t admitted = 0;
    st = admit_and_launch(s, li, &admitted);
    if (st != XG_OK) return st;
    if (admitted == 0) break;  // the oldest request waits for memory or its stream
  }
  uint32_t k = 0;
  while (k < max_out && !s->ready.empty()) {
    out[k++] = s->ready.front();
    s->ready.pop_front();
  }
  *num_out = k;
  return XG_OK;
}

}  // namespace

xg_status xg_server_poll(xg_server *s, xg_completion *out, uint32_t max_out, uint32_t *num_out) {
  if (!s || !num_out || (max_out && !out)) return XG_EINVAL;
  *num_out = 0;
  if (s->failed != XG_OK) return s->failed;
  xg_status st;
  try {
    st = poll_body(s, out, max_out, num_out);
  } catch (const std::bad_alloc &) {
    st = XG_ENOMEM;
  }
  if (st != XG_OK) {
    s->failed = st;
    *num_out = 0;
  }
  return st;
}

xg_status xg_server_release(xg_server *s, uint64_t id) {
  if (!s) return XG_EINVAL;
  if (s->failed != XG_OK) return s->failed;
  auto it = s->finished.find(id);
  if (it == s->finished.end()) return XG_EINVAL;
  s->pool.release(it->second.first, it->second.second);
  s->finished.erase(it);
  s->live.erase(id);
  return XG_OK;
}

uint64_t xg_server_outstanding(const xg_server *s) { return s ? s->outstanding : 0; }

xg_status xg_server_get_stats(const xg_server *s, xg_server_stats *out) {
  if (!s || !out) return XG_EINVAL;
  *out = s->stats;
  return XG_OK;
}

xg_status xg_server_get_tune(const xg_server *s, xg_tune *out) {
  if (!s || !out) return XG_EINVAL;
  *out = s->default_tune ? xg_tune{0, 0, 0, 0} : s->tune;
  return XG_OK;
}

void xg_server_destroy(xg_server *s) {
  if (!s) return;
  destroy_lanes(s);
  delete s;
}

}  // extern "C"
