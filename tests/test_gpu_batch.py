"""Batched requests in one persistent launch: the one-call path (the table in
the caller's order, grouped and ordered on the device, long single requests
split into jumped tiles) and the host-planned path, captured and replayed in a
HIP graph, and the autotuner with its tuning cache: identical bits to the
oracle and to the plain launch."""
import numpy as np
import pytest

from gpu_helpers import needs_gpu, ulp32_error
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402
from paper_1108_0486_amd.batch import Batch, PlannedBatch  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams  # noqa: E402

PATHS = ["device", "planned"]


def _batch(path, gs, reqs, total, **kw):
    return Batch(gs, reqs, total, **kw) if path == "device" else PlannedBatch(gs, reqs, total, **kw)


def _requests(rng, num_streams, num_reqs, max_n=5000, same_stream_every=5):
    reqs = []
    off = 0
    for i in range(num_reqs):
        s = int(rng.integers(0, num_streams)) if i % same_stream_every else 7
        n = int(rng.integers(0, max_n))
        dt = int(rng.integers(0, 3))
        reqs.append((s, n, off, dt))
        off += n + int(rng.integers(0, 3))
    return reqs, off


def _oracle_serve(ref: O.OracleStreams, reqs, out_elems=None):
    """Serves requests in order on the oracle; returns per-request expected arrays."""
    want = []
    for s, n, off, dt in reqs:
        one = ref.subset([s])
        if dt == 0:
            v = one.u32(n)[0]
        elif dt == 1:
            v = one.f32(n)[0]
        else:
            v = one.normal(n)[0]
        ref.ring[s], ref.weyl[s], ref.pos[s] = one.ring[0], one.weyl[0], one.pos[0]
        want.append(v)
    return want


def _check_outputs(out_i32: np.ndarray, reqs, want):
    for (s, n, off, dt), w in zip(reqs, want):
        if n == 0:
            continue
        got = out_i32[off:off + n]
        if dt == 0:
            assert (got.view(np.uint32) == w).all(), (s, n, dt)
        elif dt == 1:
            assert (got.view(np.float32) == w).all(), (s, n, dt)
        else:
            assert ulp32_error(got.view(np.float32), w).max() <= 4.0, (s, n, dt)


def _check_state(gs, ref):
    ring, weyl, pos = gs.host_state()
    assert (ring == ref.ring).all() and (weyl == ref.weyl).all() and (pos == ref.pos).all()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("tune", [None, (1, 1, 1), (4, 4, 8), (16, 8, 2), (2, 2, 32), (4, 8, 4, 4),
                                  (1, 4, 8, 4), (8, 8, 4, 1)])
def test_batch_matches_oracle(path, tune):
    rng = np.random.default_rng(17)
    reqs, total = _requests(rng, 300, 700)
    gs = XorgensStreams(300, seed=42)
    ref = O.OracleStreams(42, 300)
    b = _batch(path, gs, reqs, total)
    b.run(tune=tune)
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    want = _oracle_serve(ref, b.requests_in_order(), total)
    _check_outputs(b.out.cpu().numpy(), b.requests_in_order(), want)
    _check_state(gs, ref)


def test_planned_bad_request_is_skipped_and_flagged():
    """A planned table corrupted on the device after planning (a stream beyond
    the handle) trips the kernel's own bounds check: the request is skipped,
    the error word is set, the other requests are served."""
    gs = XorgensStreams(10, seed=1)
    ref = O.OracleStreams(1, 10)
    b = PlannedBatch(gs, [(2, 100, 0, 0), (3, 50, 100, 1)], 200)
    good, corrupt = b.requests_in_order()
    d = b.d_reqs.view(torch.int64).view(-1, 4)    # stream, n, out_offset, dtype | flags
    d[1, 0] = 10
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 1
    out = b.out.cpu().numpy()
    one = ref.subset([good[0]])
    assert (out[good[2]:good[2] + good[1]].view(np.uint32) == one.u32(good[1])[0]).all()
    _, _, pos = gs.host_state()
    assert pos[corrupt[0]] == 0 and pos[good[0]] == good[1]


def test_device_batch_skips_and_flags_bad_requests():
    """The device planner drops requests with a stream beyond the handle, an
    unknown dtype or nonzero flags, sets the error word, and serves the rest."""
    gs = XorgensStreams(10, seed=1)
    ref = O.OracleStreams(1, 10)
    reqs = [(2, 100, 0, 0), (10, 50, 100, 0), (3, 60, 150, 1), (4, 10, 210, 3), (2, 30, 220, 2)]
    b = Batch(gs, reqs, 300)
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 1
    good = [reqs[0], reqs[2], reqs[4]]
    want = _oracle_serve(ref, good)
    _check_outputs(b.out.cpu().numpy(), good, want)
    _check_state(gs, ref)
    # flags != 0 alone is also refused
    b2 = Batch(gs, [(5, 8, 0, 0)], 8)
    b2.d_reqs.view(torch.int32).view(-1, 8)[0, 7] = 1
    b2.run()
    torch.cuda.synchronize()
    assert b2.error_flag() == 1
    assert gs.host_state()[2][5] == 0
    # and a clean call clears the word again
    b3 = Batch(gs, [(5, 8, 0, 0)], 8)
    b3.run()
    torch.cuda.synchronize()
    assert b3.error_flag() == 0


@pytest.mark.parametrize("path", PATHS)
def test_batch_graph_replay(path):
    rng = np.random.default_rng(5)
    reqs, total = _requests(rng, 64, 128, max_n=3000)
    gs = XorgensStreams(64, seed=9)
    ref = O.OracleStreams(9, 64)
    b = _batch(path, gs, reqs, total)
    g = b.capture_graph(tune=(4, 4, 4))
    for replay in range(4):
        g.replay()
        torch.cuda.synchronize()
        # eager work between replays
        _ = torch.arange(1000, device="cuda").sum().item()
        assert b.error_flag() == 0
        want = _oracle_serve(ref, b.requests_in_order(), total)
        _check_outputs(b.out.cpu().numpy(), b.requests_in_order(), want)
        _check_state(gs, ref)


def test_autotune_keeps_state_and_bits_and_fills_the_cache():
    rng = np.random.default_rng(3)
    reqs, total = _requests(rng, 200, 400, max_n=20000)
    gs = XorgensStreams(200, seed=4)
    before = gs.checkpoint()
    b = Batch(gs, reqs, total)
    key = "test/autotune/200x400"
    best, recs = b.autotune(reps=1, tune_key=key)
    torch.cuda.synchronize()
    assert torch.equal(before, gs.state)
    assert len(recs) > 10 and all(r[4] > 0 for r in recs)
    assert best in [r[:4] for r in recs]
    assert {r[3] for r in recs} == {1, 4}
    arch, cus = xg.xg_tune_identity(gs.ctx)
    cached = xg.xg_tune_cache_get(arch, cus, xg.XG_FAMILY_R128_W32, key)
    assert cached is not None and cached[0] == best
    assert abs(cached[1] - min(r[4] for r in recs)) < 1e-6
    b.run(tune_key=key)
    out_best = b.out.clone()
    gs.restore(before)
    b.run()
    assert torch.equal(out_best, b.out)


@pytest.mark.parametrize("path", PATHS)
def test_batch_equals_plain_launch(path):
    gs_a = XorgensStreams(128, seed=42)
    gs_b = XorgensStreams(128, seed=42)
    n = 4096 + 17
    plain = gs_a.u32(n)
    reqs = [(i, n, i * n, 0) for i in range(128)]
    b = _batch(path, gs_b, reqs, 128 * n)
    b.run()
    assert torch.equal(plain.view(-1), b.out)
    assert torch.equal(gs_a.state, gs_b.state)


@pytest.mark.parametrize("path", PATHS)
def test_batch_degenerate_tables(path):
    """An empty table launches nothing and leaves the state alone; a table of
    one-word requests (uint32, FP32, and a normal that consumes a pair) and
    zero-length requests serves exactly those words."""
    gs = XorgensStreams(5, seed=3)
    saved = gs.checkpoint()
    empty = _batch(path, gs, [], 0)
    empty.run()
    torch.cuda.synchronize()
    assert torch.equal(gs.state, saved) and empty.error_flag() == 0
    reqs = [(0, 1, 0, 0), (1, 1, 1, 1), (2, 1, 2, 2), (3, 0, 3, 0), (4, 0, 3, 2), (0, 1, 3, 0)]
    b = _batch(path, gs, reqs, 4)
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    ref = O.OracleStreams(3, 5)
    want = _oracle_serve(ref, b.requests_in_order(), 4)
    _check_outputs(b.out.cpu().numpy(), b.requests_in_order(), want)
    _, _, pos = gs.host_state()
    assert list(pos) == [2, 1, 2, 0, 0]


def _cost(n, dt):
    return 4 * (n + (n & 1)) if dt == 2 else n


def _check_plan(reqs, rows, groups, num_streams, tile_words=0):
    """The served table holds every valid request once: each stream's requests
    in table order, as one group, or a lone long request as consecutive tiles
    of tile_words values; items (groups and tiles) in nonincreasing cost."""
    assert groups[0] == 0 and groups[-1] == len(rows)
    by_stream = {}
    for r in reqs:
        if r[0] < num_streams:
            by_stream.setdefault(r[0], []).append(r)
    seen = {}
    costs = []
    for g in range(len(groups) - 1):
        items = rows[groups[g]:groups[g + 1]]
        assert items, g
        s = items[0][0]
        assert all(it[0] == s for it in items)
        if items[0][4]:                                  # a tile: one segment entry
            assert len(items) == 1 and tile_words
            st, n, off, dt, fl = items[0]
            k = (fl >> 8) & 0xFF
            assert fl & 1 and (fl & 0xFC) == 0
            seen.setdefault(s, {})[k] = (n, off, dt, bool(fl & 2))
            costs.append(_cost(n, dt))
        else:
            assert s not in seen
            seen[s] = [it[:4] for it in items]
            costs.append(sum(_cost(it[1], it[3]) for it in items))
    assert sorted(seen) == sorted(by_stream)
    for s, want in by_stream.items():
        got = seen[s]
        if isinstance(got, dict):                        # tiles of one request
            assert len(want) == 1
            st, n, off, dt = want[0]
            t = len(got)
            assert sorted(got) == list(range(t)) and t == -(-(n + (n & 1 if dt == 2 else 0)) // tile_words) > 1
            for k in range(t):
                nk, offk, dtk, last = got[k]
                assert (nk, offk, dtk, last) == (min(tile_words, n - k * tile_words), off + k * tile_words, dt,
                                                 k == t - 1)
        else:
            assert got == [tuple(r) for r in want], s
    capped = [min(c, 2**32 - 1) for c in costs]
    assert all(a >= b for a, b in zip(capped, capped[1:]))


def test_device_plan_groups_in_table_order_largest_first():
    """More requests than one LDS sort block (2048), repeated streams, one
    stream holding 3000 requests: the planned table, read back, groups every
    stream's requests in table order and serves the costliest items first;
    the outputs and end states equal the oracle's."""
    rng = np.random.default_rng(23)
    S = 500
    reqs, off = [], 0
    for i in range(9000):
        s = 11 if i % 3 == 0 else int(rng.integers(0, S))
        n = int(rng.integers(0, 700))
        dt = int(rng.integers(0, 3))
        reqs.append((s, n, off, dt))
        off += n
    gs = XorgensStreams(S, seed=77)
    ref = O.OracleStreams(77, S)
    b = Batch(gs, reqs, off)
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    rows, groups = b.served_plan()
    assert len(rows) == len(reqs) and len(groups) - 1 == len({r[0] for r in reqs})
    _check_plan(reqs, rows, groups, S)
    want = _oracle_serve(ref, reqs)
    _check_outputs(b.out.cpu().numpy(), reqs, want)
    _check_state(gs, ref)


def _tile_requests(rng, S, L):
    """Streams with one long request (some past 256 tiles, some odd normals),
    streams with several requests, and short ones."""
    reqs, off = [], 0
    for s in range(S):
        kind = s % 4
        if kind == 0:                                     # one long request: tiles
            n = int(rng.integers(L + 1, 9 * L))
            reqs.append((s, n, off, int(rng.integers(0, 3)))); off += n
        elif kind == 1:                                   # several requests on the stream: no tiles
            for _ in range(3):
                n = int(rng.integers(1, 2 * L))
                reqs.append((s, n, off, int(rng.integers(0, 3)))); off += n
        elif kind == 2:                                   # one short request
            n = int(rng.integers(1, L))
            reqs.append((s, n, off, int(rng.integers(0, 3)))); off += n
        else:                                             # an odd normal count just past a tile boundary
            n = 2 * L + 1
            reqs.append((s, n, off, 2)); off += n
    # one request longer than 256 tiles runs whole
    reqs.append((S, 256 * L + 5, off, 0)); off += 256 * L + 5
    return reqs, off


def test_device_batch_tiles_match_oracle():
    """Long lone requests split into tiles of L words (each started from the
    request's start state jumped by k L words on the device): every value and
    every end state equals the oracle's, and the plan's tiles are the expected
    ones."""
    L = 4096
    rng = np.random.default_rng(31)
    S = 40
    reqs, total = _tile_requests(rng, S, L)
    gs = XorgensStreams(S + 1, seed=5)
    ref = O.OracleStreams(5, S + 1)
    b = Batch(gs, reqs, total, tile_words=L, max_tiles=4096)
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    rows, groups = b.served_plan()
    _check_plan(reqs, rows, groups, S + 1, tile_words=L)
    assert sum(1 for r in rows if r[4]) > 10
    want = _oracle_serve(ref, reqs)
    _check_outputs(b.out.cpu().numpy(), reqs, want)
    _check_state(gs, ref)


def test_device_batch_tile_budget():
    """With room for only a few tile slots, groups split in table-stream order
    while their tiles fit and the rest run whole; the bits do not change."""
    L = 4096
    reqs, off = [], 0
    for s in range(8):                                    # 3 tiles each
        reqs.append((s, 3 * L - 7, off, s % 3)); off += 3 * L - 7
    gs = XorgensStreams(8, seed=12)
    ref = O.OracleStreams(12, 8)
    b = Batch(gs, reqs, off, tile_words=L, max_tiles=7)
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    rows, groups = b.served_plan()
    tiles = [r for r in rows if r[4]]
    assert sorted({r[0] for r in tiles}) == [0, 1] and len(tiles) == 6
    assert len(groups) - 1 == 6 + 6
    want = _oracle_serve(ref, reqs)
    _check_outputs(b.out.cpu().numpy(), reqs, want)
    _check_state(gs, ref)


def _plan_pair(reqs, total, S, seed, small_kw, grid_kw):
    """The same table through two handles: one whose table fits the
    one-workgroup planner (requests plus tile slots at most 1024), one whose
    tile capacity sends it through the multi-kernel planner."""
    out = []
    for kw in (small_kw, grid_kw):
        gs = XorgensStreams(S, seed=seed)
        # words no request writes (dropped and empty requests) keep this fill
        buf = torch.full((max(1, total),), -1, dtype=torch.int32, device="cuda")
        b = Batch(gs, reqs, total, out=buf, **kw)
        b.run()
        torch.cuda.synchronize()
        out.append((b.served_plan(), b.error_flag(), b.out.cpu().numpy(), gs.host_state()))
    return out


@pytest.mark.parametrize("num_reqs", [0, 1, 37, 500, 1023, 1024, 1025, 1500, 2048, 2049, 3000, 4096, 4097])
def test_small_table_planner_equals_multi_kernel_planner(num_reqs):
    """Tables of up to 4096 requests are planned by one workgroup in LDS (1, 2
    or 4 elements per thread); the same table sent through the multi-kernel
    planner (a tile capacity that no request uses puts it there) gives the
    same table, item offsets, error word, outputs and end states, with
    repeated streams, all three dtypes, empty requests and requests that fail
    the checks."""
    rng = np.random.default_rng(1000 + num_reqs)
    S = 97
    reqs, off = [], 0
    for i in range(num_reqs):
        s = 5 if i % 7 == 0 else int(rng.integers(0, S + 3))   # a few streams past S: dropped
        n = int(rng.integers(0, 900))
        dt = int(rng.integers(0, 3)) if i % 50 != 49 else 3    # dtype 3: dropped
        reqs.append((s, n, off, dt))
        off += n
    (plan_a, err_a, out_a, st_a), (plan_b, err_b, out_b, st_b) = _plan_pair(
        reqs, off, S, 41, {}, {"tile_words": 1 << 30, "max_tiles": 4096})
    assert plan_a == plan_b
    assert err_a == err_b == int(any(r[0] >= S or r[3] > 2 for r in reqs))
    assert (out_a == out_b).all()
    assert all((x == y).all() for x, y in zip(st_a, st_b))
    rows, groups = plan_a
    _check_plan([r for r in reqs if r[3] <= 2], rows, groups, S)


@pytest.mark.parametrize("n_req", [1024, 4096])
@pytest.mark.parametrize("kind", ["one_stream", "all_invalid", "distinct_streams", "mostly_empty"])
def test_small_table_planner_edge_tables(kind, n_req):
    """Edge tables at the one-workgroup planner's limits (1024 requests at one
    element per thread, 4096 at four), each against the multi-kernel
    planner: one stream holding every request (one group), every request
    failing the checks, distinct streams (one group each, in cost order), and
    mostly empty requests."""
    S = n_req + 76
    rng = np.random.default_rng(77)
    reqs, off = [], 0
    for i in range(n_req):
        if kind == "one_stream":
            st, n, dt = 0, int(rng.integers(1, 300)), i % 3
        elif kind == "all_invalid":
            st, n, dt = S + i, 10, 0
        elif kind == "distinct_streams":
            st, n, dt = (i * 37) % n_req, 64 + (i * 7919) % 2000, i % 3
        else:
            st, n, dt = int(rng.integers(0, 50)), (int(rng.integers(1, 100)) if i % 5 == 0 else 0), i % 3
        reqs.append((st, n, off, dt))
        off += n
    (plan_a, err_a, out_a, st_a), (plan_b, err_b, out_b, st_b) = _plan_pair(
        reqs, off, S, 8, {}, {"tile_words": 1 << 30, "max_tiles": 4096})
    assert plan_a == plan_b
    assert err_a == err_b == int(kind == "all_invalid")
    assert (out_a == out_b).all()
    assert all((x == y).all() for x, y in zip(st_a, st_b))
    rows, groups = plan_a
    if kind == "all_invalid":
        assert rows == [] and groups == [0]
    else:
        _check_plan(reqs, rows, groups, S)
        assert len(groups) - 1 == len({r[0] for r in reqs})


@pytest.mark.parametrize("slots", [1000, 3000])
def test_small_table_planner_tiles_equal_multi_kernel_planner(slots):
    """Tiles in the one-workgroup planner (19 requests with 1000 or 3000 tile
    slots: one and four elements per thread) and in the multi-kernel planner
    (5000 slots): the same plan, outputs and states, and the oracle's
    values."""
    L = 4096
    rng = np.random.default_rng(12)
    S = 12
    reqs, total = _tile_requests(rng, S, L)
    assert len(reqs) + slots <= 4096 and len(reqs) + 5000 > 4096
    (plan_a, err_a, out_a, st_a), (plan_b, err_b, out_b, st_b) = _plan_pair(
        reqs, total, S + 1, 6, {"tile_words": L, "max_tiles": slots}, {"tile_words": L, "max_tiles": 5000})
    assert err_a == err_b == 0
    assert plan_a == plan_b
    rows, groups = plan_a
    _check_plan(reqs, rows, groups, S + 1, tile_words=L)
    assert sum(1 for r in rows if r[4]) > 10
    assert (out_a == out_b).all()
    assert all((x == y).all() for x, y in zip(st_a, st_b))
    ref = O.OracleStreams(6, S + 1)
    want = _oracle_serve(ref, reqs)
    _check_outputs(out_a, reqs, want)
    ring, weyl, pos = st_a
    assert (ring == ref.ring).all() and (weyl == ref.weyl).all() and (pos == ref.pos).all()


def test_device_batch_tiles_graph_replay():
    """The whole call with tiles (planning, start states by jump, batch)
    captured once and replayed three times, with eager work in between: every
    replay against the oracle."""
    L = 4096
    rng = np.random.default_rng(8)
    S = 24
    reqs, total = _tile_requests(rng, S, L)
    gs = XorgensStreams(S + 1, seed=21)
    ref = O.OracleStreams(21, S + 1)
    b = Batch(gs, reqs, total, tile_words=L, max_tiles=1024)
    g = b.capture_graph(tune=(2, 2, 4))
    for replay in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = torch.ones(4096, device="cuda").cumsum(0)[-1].item()
        assert b.error_flag() == 0
        want = _oracle_serve(ref, reqs)
        _check_outputs(b.out.cpu().numpy(), reqs, want)
        _check_state(gs, ref)


def test_device_batch_refuses_more_requests_than_its_scratch():
    gs = XorgensStreams(4, seed=1)
    b = Batch(gs, [(0, 10, 0, 0), (1, 10, 10, 0)], 20)
    saved = gs.checkpoint()
    with pytest.raises(xg.XgError) as e:
        xg.xg_generate_batch(gs.ctx, b.d_reqs.data_ptr(), gs._batch_cfg[0] + 1, b.out.data_ptr())
    assert e.value.status == xg.XG_EBUSY
    torch.cuda.synchronize()
    assert torch.equal(saved, gs.state)
