"""The request server: continuous batching with memory admission and
per-stream order.  Every request's values equal the oracle's from the
position it was admitted at, and equal the same request run alone."""
import time

import numpy as np
import pytest

from gpu_helpers import needs_gpu, ulp32_error
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402
from paper_1108_0486_amd import workloads as W  # noqa: E402
from paper_1108_0486_amd.serve import Server, run_trace, run_trace_plain_fifo  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams, as_u32  # noqa: E402

SEED = 42


def _check_against_oracle(done, outputs, num_streams):
    by_stream = {}
    for c in done:
        by_stream.setdefault(c.stream, []).append(c)
    for s, cs in by_stream.items():
        cs.sort(key=lambda c: c.start_pos)
        # requests on one stream are served in submission order (ids are
        # given in submission order by every caller here)
        ids = [c.id for c in cs]
        assert ids == sorted(ids), (s, ids)
        ref = O.OracleStreams(SEED + s, 1)
        pos = 0
        for c in cs:
            assert c.start_pos == pos, (s, c.id, c.start_pos, pos)   # requests chain on their stream
            got = outputs[c.id].cpu().numpy()
            if c.dtype == xg.XG_U32:
                assert (got.view(np.uint32) == ref.u32(c.n)[0]).all(), c
            elif c.dtype == xg.XG_F32:
                assert (got == ref.f32(c.n)[0]).all(), c
            else:
                assert ulp32_error(got, ref.normal(c.n)[0]).max() <= 4.0, c
            pos += c.n + (c.n & 1 if c.dtype == xg.XG_NORMAL else 0)


def _dense_trace(num_reqs, num_streams, seed, lo=4, hi=14, rate=50_000.0):
    trace = W.serving_trace(num_reqs, num_streams=num_streams, rate=rate, seed=seed, lo_exp=lo, hi_exp=hi)
    # a long request first, so that later arrivals are admitted while it runs
    trace[0].n = 1 << 20
    trace[0].dtype = 0
    return trace


def test_serving_matches_oracle_and_overlaps():
    S = 40                                   # few streams: many same-stream requests
    gs = XorgensStreams(S, seed=SEED)
    srv = Server(gs, pool_elems=1 << 22, num_lanes=4, max_batch=32)
    trace = _dense_trace(300, S, seed=3)
    summary, done, outputs = run_trace(srv, trace, keep_outputs=True)
    st = summary["server"]
    assert st["completed"] == 300 and st["submitted"] == 300
    assert st["max_lanes_busy"] >= 2          # batches overlapped on the device
    assert st["batches"] > 1 and st["max_batch_seen"] > 1
    _check_against_oracle(done, outputs, S)
    # final device positions agree with the host's bookkeeping
    _, _, pos = gs.host_state()
    want = np.zeros(S, dtype=np.uint64)
    for c in done:
        want[c.stream] = max(want[c.stream], c.start_pos + c.n + (c.n & 1 if c.dtype == 2 else 0))
    assert (pos == want).all()
    srv.close()


def test_alone_equals_in_the_mix():
    S = 64
    gs = XorgensStreams(S, seed=SEED)
    srv = Server(gs, pool_elems=1 << 22, num_lanes=3, max_batch=16)
    summary, done, outputs = run_trace(srv, _dense_trace(200, S, seed=9), keep_outputs=True)
    srv.close()
    rng = np.random.default_rng(1)
    for c in [done[i] for i in rng.choice(len(done), size=24, replace=False)]:
        alone = XorgensStreams(1, seed=SEED + c.stream)
        if c.start_pos:
            alone.u32(c.start_pos)           # advance to the admitted position
        if c.dtype == xg.XG_U32:
            ref = alone.u32(c.n)[0]
        elif c.dtype == xg.XG_F32:
            ref = alone.f32(c.n)[0]
        else:
            ref = alone.normal(c.n)[0]
        assert torch.equal(ref.view(torch.int32), outputs[c.id].view(torch.int32)), c


def test_memory_admission_queues_instead_of_failing():
    S = 30
    gs = XorgensStreams(S, seed=SEED)
    srv = Server(gs, pool_elems=1 << 15, num_lanes=2, max_batch=8)   # far less than the trace needs
    trace = W.serving_trace(120, num_streams=S, rate=1e6, seed=5, lo_exp=10, hi_exp=15)
    summary, done, outputs = run_trace(srv, trace, keep_outputs=True)
    st = summary["server"]
    assert st["completed"] == 120
    assert st["admission_waits"] > 0
    assert st["pool_high_water"] <= 1 << 15
    _check_against_oracle(done, outputs, S)
    srv.close()


def test_oversize_and_bad_requests_rejected():
    gs = XorgensStreams(4, seed=SEED)
    srv = Server(gs, pool_elems=1 << 12, num_lanes=1, max_batch=4)
    with pytest.raises(xg.XgError) as e:
        srv.submit(1, 0, (1 << 12) + 1, 0)
    assert e.value.status == xg.XG_ERANGE
    with pytest.raises(xg.XgError) as e:
        srv.submit(2, 4, 10, 0)
    assert e.value.status == xg.XG_ERANGE
    with pytest.raises(xg.XgError) as e:
        srv.submit(3, 0, 0, 0)
    assert e.value.status == xg.XG_EINVAL
    with pytest.raises(xg.XgError) as e:
        srv.submit(4, 0, 10, 3)
    assert e.value.status == xg.XG_EINVAL
    with pytest.raises(xg.XgError) as e:
        srv.release(12345)
    assert e.value.status == xg.XG_EINVAL
    assert srv.outstanding == 0
    # an id may not be reused until its request is released
    srv.submit(7, 0, 16, 0)
    with pytest.raises(xg.XgError) as e:
        srv.submit(7, 1, 16, 0)
    assert e.value.status == xg.XG_EINVAL
    deadline = time.monotonic() + 20.0
    got = []
    while not got and time.monotonic() < deadline:
        got = srv.poll()
    assert [c.id for c in got] == [7]
    with pytest.raises(xg.XgError):
        srv.submit(7, 1, 16, 0)                                    # completed, not yet released
    srv.release(7)
    srv.submit(7, 1, 16, 0)                                        # free again
    srv.close()


def test_plain_fifo_baseline_runs():
    S = 16
    gs = XorgensStreams(S, seed=SEED)
    trace = W.serving_trace(50, num_streams=S, rate=20_000.0, seed=2, lo_exp=8, hi_exp=14)
    summary = run_trace_plain_fifo(gs, trace, max_n=1 << 14)
    assert summary["requests"] == 50 and summary["p99_ms"] > 0


@pytest.mark.parametrize("seg", [4096, 1 << 14])
def test_segmented_serving_matches_oracle(seg):
    """Requests longer than the segment length run as jumped segments on
    separate wavefronts; every value still equals the oracle's from the
    request's start position, and the stream ends where the unsplit request
    would leave it."""
    S = 24
    gs = XorgensStreams(S, seed=SEED)
    srv = Server(gs, pool_elems=1 << 22, num_lanes=4, max_batch=512, segment_words=seg)
    trace = W.serving_trace(150, num_streams=S, rate=30_000.0, seed=21, lo_exp=6, hi_exp=17)
    trace[0].n, trace[0].dtype = (1 << 20) + 77, 2          # long, odd normal request
    trace[1].n, trace[1].dtype = 5 * seg, 0                # an exact multiple of the segment
    summary, done, outputs = run_trace(srv, trace, keep_outputs=True)
    assert summary["server"]["completed"] == 150
    _check_against_oracle(done, outputs, S)
    _, _, pos = gs.host_state()
    want = np.zeros(S, dtype=np.uint64)
    for c in done:
        want[c.stream] = max(want[c.stream], c.start_pos + c.n + (c.n & 1 if c.dtype == 2 else 0))
    assert (pos == want).all()
    srv.close()


def test_segmented_alone_equals_in_the_mix():
    S = 16
    gs = XorgensStreams(S, seed=SEED)
    srv = Server(gs, pool_elems=1 << 22, num_lanes=2, max_batch=256, segment_words=8192)
    trace = W.serving_trace(60, num_streams=S, rate=20_000.0, seed=4, lo_exp=10, hi_exp=17)
    summary, done, outputs = run_trace(srv, trace, keep_outputs=True)
    srv.close()
    for c in sorted(done, key=lambda c: -c.n)[:10]:
        alone = XorgensStreams(1, seed=SEED + c.stream)
        if c.start_pos:
            alone.skip(c.start_pos)
        ref = {0: alone.u32, 1: alone.f32, 2: alone.normal}[c.dtype](c.n)[0]
        assert torch.equal(ref.view(torch.int32), outputs[c.id].view(torch.int32)), c


def test_invalid_segment_length_rejected():
    gs = XorgensStreams(4, seed=SEED)
    for seg in (100, 64, 1 << 31):
        with pytest.raises(ValueError):
            Server(gs, pool_elems=1 << 12, num_lanes=1, max_batch=4, segment_words=seg)


def test_request_with_more_segments_than_a_batch_runs_unsplit():
    """A request that would split into more segments than one batch table
    holds (max_batch = 4, 10 segments) is served unsplit instead of waiting
    forever, and the requests behind it still complete."""
    gs = XorgensStreams(3, seed=SEED)
    srv = Server(gs, pool_elems=1 << 17, num_lanes=1, max_batch=4, segment_words=4096)
    for rid, (stream, n, dt) in enumerate([(0, 10 * 4096, 0), (1, 3 * 4096 + 5, 1), (2, 100, 2), (0, 77, 0)]):
        srv.submit(rid, stream, n, dt)
    done, outputs = [], {}
    deadline = time.monotonic() + 20.0
    while len(done) < 4 and time.monotonic() < deadline:
        for c in srv.poll():
            outputs[c.id] = srv.output(c).clone()
            srv.release(c.id)
            done.append(c)
    assert len(done) == 4, [c.id for c in done]
    _check_against_oracle(done, outputs, 3)
    srv.close()


def test_split_request_keeps_its_streams_order():
    """A(short), B(long enough to split into segments), C(short), all on
    one stream and submitted together: B cannot share a batch with A, and C
    must not overtake it, so the three read consecutive positions in
    submission order (C after B)."""
    gs = XorgensStreams(2, seed=SEED)
    srv = Server(gs, pool_elems=1 << 17, num_lanes=1, max_batch=64, segment_words=4096)
    plan = [(0, 100, 0), (0, 3 * 4096 + 5, 1), (0, 50, 0), (1, 7, 2), (0, 64, 2)]
    for rid, (stream, n, dt) in enumerate(plan):
        srv.submit(rid, stream, n, dt)
    done, outputs = [], {}
    deadline = time.monotonic() + 20.0
    while len(done) < len(plan) and time.monotonic() < deadline:
        for c in srv.poll():
            outputs[c.id] = srv.output(c).clone()
            srv.release(c.id)
            done.append(c)
    assert len(done) == len(plan), [c.id for c in done]
    start = {c.id: c.start_pos for c in done}
    assert start[0] == 0 and start[1] == 100 and start[2] == 100 + 3 * 4096 + 5 and start[4] == start[2] + 50
    _check_against_oracle(done, outputs, 2)
    srv.close()


def test_pool_not_a_multiple_of_64():
    """The server uses floor(pool_elems / 64) * 64 elements of its pool (its
    ranges are 64-element aligned): a request that rounds up past that is
    rejected at submit instead of waiting forever, one that fits is served,
    and a pool of fewer than 64 elements is refused."""
    gs = XorgensStreams(2, seed=SEED)
    with pytest.raises(xg.XgError) as e:
        Server(gs, pool_elems=63, num_lanes=1, max_batch=4)
    assert e.value.status == xg.XG_EINVAL
    srv = Server(gs, pool_elems=100, num_lanes=1, max_batch=4)
    with pytest.raises(xg.XgError) as e:
        srv.submit(0, 0, 65, 0)
    assert e.value.status == xg.XG_ERANGE
    for rid, (stream, n, dt) in enumerate([(0, 64, 0), (1, 1, 1), (0, 33, 2)]):
        srv.submit(rid, stream, n, dt)
    done, outputs = [], {}
    deadline = time.monotonic() + 20.0
    while len(done) < 3 and time.monotonic() < deadline:
        for c in srv.poll():
            assert c.out_offset + c.n <= 64
            outputs[c.id] = srv.output(c).clone()
            srv.release(c.id)
            done.append(c)
    assert len(done) == 3, [c.id for c in done]
    _check_against_oracle(done, outputs, 2)
    srv.close()


def _oracle_at(stream: int, q: int, P: int):
    """The oracle's stream `stream` (seed SEED + stream) moved to word q: by
    stepping for short moves, else by its own polynomial jump (z^q mod P on
    the x-part, q omega on the Weyl word)."""
    ref = O.OracleStreams(SEED + stream, 1)
    if q == 0:
        return ref
    if q < (1 << 16):
        ref.skip(q)
        return ref
    g = O.poly_to_words(O.z_pow_mod(q, P), 64)
    ring = O.xpart_jump_poly(O.PAPER, ref.ring[0], g)
    weyl = (int(ref.weyl[0]) + q * O.PAPER.omega) % 2**32
    return O.OracleStreams.from_state(ring[None, :], np.array([weyl], dtype=np.uint32), np.array([q], dtype=np.uint64))


def test_server_takes_its_shape_from_the_tuning_cache():
    """A server created with a tuning-cache key and no explicit shape runs
    the cached shape (and its values still equal the oracle's); an absent key
    leaves the default; a malformed key is refused."""
    S = 16
    gs = XorgensStreams(S, seed=SEED)
    arch, cus = xg.xg_tune_identity(gs.ctx)
    xg.xg_tune_cache_put(arch, cus, xg.XG_FAMILY_R128_W32, "test/serve/small", (2, 4, 3, 1), 0.5)
    srv = Server(gs, pool_elems=1 << 20, num_lanes=2, max_batch=16, tune_key="test/serve/small")
    assert xg.xg_server_get_tune(srv.srv) == (2, 4, 3, 1)
    trace = W.serving_trace(60, num_streams=S, rate=100_000.0, seed=4, lo_exp=2, hi_exp=13)
    summary, done, outputs = run_trace(srv, trace, keep_outputs=True, timeout_s=60)
    assert summary["server"]["completed"] == len(trace)
    _check_against_oracle(done, outputs, S)
    srv.close()
    gs2 = XorgensStreams(S, seed=SEED)
    srv2 = Server(gs2, pool_elems=1 << 20, num_lanes=1, max_batch=16, tune_key="test/serve/absent")
    assert xg.xg_server_get_tune(srv2.srv) == (0, 0, 0, 0)
    srv2.close()
    with pytest.raises(xg.XgError) as e:
        Server(gs2, pool_elems=1 << 20, num_lanes=1, max_batch=16, tune_key='bad"key')
    assert e.value.status == xg.XG_EINVAL


def _check_request(c, host, P):
    """A completed request's values against the oracle from its start
    position; returns None or a description of the mismatch."""
    ref = _oracle_at(c.stream, c.start_pos, P)
    if c.dtype == xg.XG_U32:
        ok = np.array_equal(host.view(np.uint32), ref.u32(c.n)[0])
    elif c.dtype == xg.XG_F32:
        ok = np.array_equal(host.view(np.float32), ref.f32(c.n)[0])
    else:
        ok = bool(ulp32_error(host.view(np.float32), ref.normal(c.n)[0]).max() <= 4.0)
    return None if ok else (c.id, c.stream, c.start_pos, c.n, c.dtype)


def test_serving_full_size_every_value():
    """The serving workload at full size: 10^5 resident streams, the bench's
    server (8 GiB pool, 4 lanes, batches of up to 8192 entries, requests over
    2^16 words split into jumped segments) and the first 1500 requests of the
    seed-11 trace (N up to 2^24, all three dtypes, 2.3 x 10^9 values),
    submitted at once so the batches mix.  Every value of every request equals
    the oracle's from the request's start position (checked on host threads
    while the server runs), and every touched stream ends in the oracle's
    state after the words its requests consumed."""
    from concurrent.futures import ThreadPoolExecutor

    trace = W.serving_trace(1500)
    gs = XorgensStreams(W.SERVE_STREAMS, seed=SEED)
    srv = Server(gs, pool_elems=1 << 31, num_lanes=4, max_batch=8192, segment_words=1 << 16)
    for r in trace:
        srv.submit(r.rid, r.stream, r.n, r.dtype)
    P = O.charpoly(O.PAPER)
    done, futures, values = [], [], 0
    with ThreadPoolExecutor(max_workers=O.default_threads()) as pool:
        deadline = time.monotonic() + 300.0
        while len(done) < len(trace) and time.monotonic() < deadline:
            for c in srv.poll():
                host = srv.output(c).cpu().numpy().copy()
                srv.release(c.id)
                done.append(c)
                values += c.n
                futures.append(pool.submit(_check_request, c, host, P))
        bad = [f.result() for f in futures]
    srv.close()
    assert len(done) == len(trace)
    bad = [x for x in bad if x is not None]
    assert not bad, bad[:10]
    assert values == sum(r.n for r in trace) and values > 2 * 10**9
    assert sum(1 for c in done if c.n > (1 << 16)) > 100     # many requests ran as jumped segments
    # End state of every stream the trace touched: it depends on every word
    # its requests (and their jumped segments) generated.
    used = {}
    for c in done:
        used[c.stream] = used.get(c.stream, 0) + c.n + (c.n & 1 if c.dtype == xg.XG_NORMAL else 0)
    touched = sorted(used)
    ring, weyl, pos = gs.host_state(touched)
    for j, st in enumerate(touched):
        ref = _oracle_at(st, used[st], P)
        assert int(pos[j]) == used[st], st
        assert (ring[j] == ref.ring[0]).all() and int(weyl[j]) == int(ref.weyl[0]), st


@pytest.mark.parametrize("seed,seg,pool,lanes,max_batch", [
    (21, None, 1 << 16, 2, 8),          # small pool: admission waits; small tables
    (22, 4096, 1 << 17, 3, 6),          # segments; some requests too long to split into 6
    (23, 4096, 1 << 20, 4, 64),         # segments, roomy
    (24, None, 1 << 20, 1, 1),          # one request per batch
])
def test_serving_random_traces_match_oracle(seed, seg, pool, lanes, max_batch):
    """Randomised traces (few streams, so requests chain on a stream; N from 1
    to 2^15; all three dtypes) through servers configured to hit the
    admission paths: a pool far smaller than the trace, tables that hold
    fewer entries than a split request has segments, a single lane.  Every
    value of every request equals the oracle's from its start position, and
    each stream's requests chain without gaps."""
    S = 12
    gs = XorgensStreams(S, seed=SEED)
    kw = {} if seg is None else {"segment_words": seg}
    srv = Server(gs, pool_elems=pool, num_lanes=lanes, max_batch=max_batch, **kw)
    trace = W.serving_trace(250, num_streams=S, rate=200_000.0, seed=seed, lo_exp=0, hi_exp=15)
    summary, done, outputs = run_trace(srv, trace, keep_outputs=True, timeout_s=60)
    assert summary["server"]["completed"] == len(trace)
    _check_against_oracle(done, outputs, S)
    srv.close()
