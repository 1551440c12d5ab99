"""The persistent batched launch for the two further members: two request
groups per wavefront (one per half), identical bits to the oracle for words
and reals and normals within 4 ulp, after graph replays and under every
launch shape, with bad and empty requests skipped."""
import numpy as np
import pytest

from gpu_helpers import check_ragged_every_word, needs_gpu, ulp32_error, ulp64_error
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402
from paper_1108_0486_amd.batch import Batch, PlannedBatch  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams  # noqa: E402

R64W32, R64W64 = xg.XG_FAMILY_R64_W32, xg.XG_FAMILY_R64_W64
FAMILIES = [R64W32, R64W64]
PARAMS = {R64W32: O.R64, R64W64: O.W64}


def _oracle(fam, seed, count):
    p = PARAMS[fam]
    if fam == R64W64:
        return O.OracleStreams64(seed, count, p)
    return O.OracleStreams(seed, count, params=p)


def _one(fam, ref, s):
    if fam == R64W64:
        return O.OracleStreams64.from_state(ref.ring[[s]], ref.weyl[[s]], ref.pos[[s]], ref.params)
    return ref.subset([s])


def _oracle_serve(fam, ref, reqs):
    """Serves the requests in the given order on the oracle (each stream's
    requests in that order); returns the expected words of each."""
    want = []
    for s, n, off, dt in reqs:
        one = _one(fam, ref, s)
        if dt == 2:
            v = one.normal(n)[0]
        elif fam == R64W64:
            v = one.u64(n)[0] if dt == 0 else one.f64(n)[0].view(np.uint64)
        else:
            v = one.u32(n)[0] if dt == 0 else one.f32(n)[0].view(np.uint32)
        ref.ring[s], ref.weyl[s], ref.pos[s] = one.ring[0], one.weyl[0], one.pos[0]
        want.append(np.asarray(v))
    return want


def _requests(rng, num_streams, num_reqs, max_n, mixed=True):
    reqs, off = [], 0
    for i in range(num_reqs):
        s = int(rng.integers(0, num_streams)) if i % 4 else 3
        n = int(rng.integers(0, max_n))
        dt = int(rng.integers(0, 3)) if mixed else 0
        reqs.append((s, n, off, dt))
        off += n + int(rng.integers(0, 3))
    return reqs, off


def _check(fam, out, reqs, want):
    words = out.cpu().numpy().view(np.uint64 if fam == R64W64 else np.uint32)
    for (s, n, off, dt), w in zip(reqs, want):
        if n == 0:
            continue
        got = words[off:off + n]
        if dt == 2:  # normals: FP32 / FP64 against the oracle's higher precision
            err = ulp64_error(got.view(np.float64), w) if fam == R64W64 else ulp32_error(got.view(np.float32), w)
            assert err.max() <= 4.0, (s, n, off, dt)
        else:
            assert (got == w).all(), (s, n, off, dt)


@pytest.mark.parametrize("path", ["device", "planned"])
@pytest.mark.parametrize("fam", FAMILIES)
@pytest.mark.parametrize("tune", [None, (1, 1, 1), (2, 2, 4), (4, 4, 8), (16, 8, 2), (1, 8, 32)])
def test_member_batch_matches_oracle(fam, tune, path):
    rng = np.random.default_rng(17)
    S = 37
    reqs, out_elems = _requests(rng, S, 120, 3000)
    gs = XorgensStreams(S, seed=9, family=fam)
    b = (Batch if path == "device" else PlannedBatch)(gs, reqs, out_elems)
    b.run(tune=None if tune is None else (tune[0], tune[1], tune[2], 1))
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    # Each stream serves its requests in table order.
    ref = _oracle(fam, 9, S)
    want = _oracle_serve(fam, ref, b.requests_in_order())
    _check(fam, b.out, b.requests_in_order(), want)
    # End states equal the oracle's after every request.
    ring, weyl, pos = gs.host_state()
    assert (ring == ref.ring).all() and (weyl == ref.weyl).all() and (pos == ref.pos).all()


@pytest.mark.parametrize("fam", FAMILIES)
def test_member_batch_equals_plain_launches(fam):
    # One request per stream of equal length: the same words as one plain
    # stream-major launch over all streams.
    S, n = 64, 4133
    reqs = [(i, n, i * n, 0) for i in range(S)]
    a = XorgensStreams(S, seed=4, family=fam)
    b = XorgensStreams(S, seed=4, family=fam)
    bt = Batch(a, reqs, S * n)
    bt.run()
    plain = b.u64(n) if fam == R64W64 else b.u32(n)
    torch.cuda.synchronize()
    assert bt.error_flag() == 0
    assert torch.equal(bt.out.view(plain.dtype).view(S, n), plain)
    assert torch.equal(a.state, b.state)


@pytest.mark.parametrize("fam", FAMILIES)
def test_member_batch_graph_replay(fam):
    rng = np.random.default_rng(5)
    S = 21
    reqs, out_elems = _requests(rng, S, 40, 2000)
    gs = XorgensStreams(S, seed=13, family=fam)
    b = Batch(gs, reqs, out_elems)
    g = b.capture_graph()
    ref = _oracle(fam, 13, S)
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert b.error_flag() == 0
        want = _oracle_serve(fam, ref, b.requests_in_order())
        _check(fam, b.out, b.requests_in_order(), want)


@pytest.mark.parametrize("fam", FAMILIES)
def test_member_batch_skips_bad_requests(fam):
    # An empty request is skipped without a flag; a request with an unknown
    # dtype is flagged and skipped.
    S = 6
    gs = XorgensStreams(S, seed=2, family=fam)
    good = [(0, 100, 0, 0), (1, 33, 100, 1), (2, 0, 133, 0), (0, 31, 133, 2)]
    b = Batch(gs, good, 200)
    raw = b.d_reqs.cpu().numpy().copy().view(np.uint64).reshape(-1, 4)
    ref = _oracle(fam, 2, S)
    want = _oracle_serve(fam, ref, b.requests_in_order())
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    _check(fam, b.out, b.requests_in_order(), want)
    # Now corrupt one request on the device: dtype 3 (no such type).
    bad = raw.copy()
    bad[0, 3] = (bad[0, 3] & ~np.uint64(0xFFFFFFFF)) | np.uint64(3)
    b.d_reqs.copy_(torch.from_numpy(bad.view(np.int32).reshape(-1)))
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 1


@pytest.mark.parametrize("fam", FAMILIES)
def test_member_batch_autotune_keeps_state(fam):
    rng = np.random.default_rng(8)
    S = 40
    reqs, out_elems = _requests(rng, S, 80, 4000, mixed=False)
    gs = XorgensStreams(S, seed=21, family=fam)
    before = gs.state.clone()
    b = Batch(gs, reqs, out_elems)
    best, times = b.autotune(reps=1)
    torch.cuda.synchronize()
    assert torch.equal(gs.state, before)
    assert all(t[3] == 1 for t in times)  # store_words: no wide stores for these members
    b.run(tune=best)
    torch.cuda.synchronize()
    ref = _oracle(fam, 21, S)
    want = _oracle_serve(fam, ref, b.requests_in_order())
    _check(fam, b.out, b.requests_in_order(), want)


@pytest.mark.parametrize("fam", FAMILIES)
def test_member_batch_odd_normal_pieces(fam):
    # Two groups in one wavefront, both normals, with odd lengths that end
    # inside the partner's request: the trips shorten to even counts, and a
    # count of one runs only the half that finishes (the pair is kept whole).
    S = 2
    reqs = [(0, 5, 0, 2), (1, 10, 5, 2), (0, 3, 15, 2), (1, 7, 18, 0), (0, 1, 25, 2)]
    gs = XorgensStreams(S, seed=77, family=fam)
    b = Batch(gs, reqs, 26)
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    assert b.served_counts() == (2, 5)
    ref = _oracle(fam, 77, S)
    want = _oracle_serve(fam, ref, b.requests_in_order())
    _check(fam, b.out, b.requests_in_order(), want)
    ring, weyl, pos = gs.host_state()
    assert (ring == ref.ring).all() and (weyl == ref.weyl).all() and (pos == ref.pos).all()


@pytest.mark.parametrize("fam", FAMILIES)
@pytest.mark.parametrize("pool,lanes,max_batch", [(1 << 20, 4, 64), (1 << 14, 2, 8), (1 << 20, 1, 1)])
def test_member_serving_matches_oracle(fam, pool, lanes, max_batch):
    """A randomised trace (few streams, so requests chain on a stream; N from 1
    to 2^13; all three dtypes) through a member's server: every request reads
    from where the stream's previous request ended, and every value equals
    the oracle's."""
    from paper_1108_0486_amd import workloads as W
    from paper_1108_0486_amd.serve import Server, run_trace

    S = 10
    gs = XorgensStreams(S, seed=31, family=fam)
    srv = Server(gs, pool_elems=pool, num_lanes=lanes, max_batch=max_batch)
    trace = W.serving_trace(200, num_streams=S, rate=200_000.0, seed=5, lo_exp=0, hi_exp=13)
    summary, done, outputs = run_trace(srv, trace, keep_outputs=True, timeout_s=60)
    assert summary["server"]["completed"] == len(trace)
    ref = _oracle(fam, 31, S)
    pos = [0] * S
    for c in sorted(done, key=lambda c: (c.stream, c.start_pos)):
        assert c.start_pos == pos[c.stream], (c.id, c.stream)
        w = _oracle_serve(fam, ref, [(c.stream, c.n, 0, c.dtype)])[0]
        _check(fam, outputs[c.id], [(c.stream, c.n, 0, c.dtype)], [w])
        pos[c.stream] += c.n + (c.n & 1 if c.dtype == xg.XG_NORMAL else 0)
    srv.close()


def test_member_batch_full_size_ragged():
    """The 65536-stream ragged workload (uint32, dense CSR offsets) on the
    n = 2048 member, with the autotuned shape in a replayed graph, as the
    bench times it: every word of every stream against the oracle, every end
    position, and the end states of 256 streams against the oracle stepped
    through them."""
    from paper_1108_0486_amd import workloads as W

    lengths = W.ragged_lengths()
    off = W.csr_offsets(lengths)
    total = int(off[-1])
    S = len(lengths)
    gs = XorgensStreams(S, seed=W.SEED, family=R64W32)
    b = Batch(gs, [(i, int(lengths[i]), int(off[i]), 0) for i in range(S)], total)
    best, _ = b.autotune(reps=1)
    g = b.capture_graph(tune=best)
    g.replay()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    _, _, pos = gs.host_state()
    assert (pos == lengths).all()
    check_ragged_every_word(b.out, lengths, off, W.SEED, params=O.R64)
    rng = np.random.default_rng(1)
    more = sorted(rng.choice(S, size=256, replace=False).tolist())
    ring, weyl, _ = gs.host_state(more)
    for j, i in enumerate(more):
        n = int(lengths[i])
        end = O.OracleStreams(W.SEED + i, 1, params=O.R64)
        end.skip(n)                                      # the oracle steps through all n words
        assert (ring[j] == end.ring[0]).all(), i
        assert int(weyl[j]) == int(end.weyl[0]), i
