"""The persistent batched launch (request groups from a device queue),
captured and replayed in a HIP graph, and its autotuner: identical bits to
the oracle and to the plain launch."""
import numpy as np
import pytest

from gpu_helpers import needs_gpu, ulp32_error
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402
from paper_1108_0486_amd.batch import Batch  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams  # noqa: E402


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


def _oracle_serve(ref: O.OracleStreams, reqs, out_elems):
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


@pytest.mark.parametrize("tune", [None, (1, 1, 1), (4, 4, 8), (16, 8, 2), (2, 2, 32), (4, 8, 4, 4),
                                  (1, 4, 8, 4), (8, 8, 4, 1)])
def test_batch_matches_oracle(tune):
    rng = np.random.default_rng(17)
    reqs, total = _requests(rng, 300, 700)
    gs = XorgensStreams(300, seed=42)
    ref = O.OracleStreams(42, 300)
    b = Batch(gs, reqs, total)
    b.run(tune=tune)
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    want = _oracle_serve(ref, b.requests_in_order(), total)
    _check_outputs(b.out.cpu().numpy(), b.requests_in_order(), want)
    ring, weyl, pos = gs.host_state()
    assert (ring == ref.ring).all() and (weyl == ref.weyl).all() and (pos == ref.pos).all()


def test_batch_bad_request_is_skipped_and_flagged():
    """A request table corrupted on the device after planning (a stream beyond
    the handle) trips the kernel's own bounds check: the request is skipped,
    the error word is set, the other requests are served."""
    gs = XorgensStreams(10, seed=1)
    ref = O.OracleStreams(1, 10)
    b = Batch(gs, [(2, 100, 0, 0), (3, 50, 100, 1)], 200)
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


def test_batch_graph_replay():
    rng = np.random.default_rng(5)
    reqs, total = _requests(rng, 64, 128, max_n=3000)
    gs = XorgensStreams(64, seed=9)
    ref = O.OracleStreams(9, 64)
    b = Batch(gs, reqs, total)
    g = b.capture_graph(tune=(4, 4, 4))
    for replay in range(4):
        g.replay()
        torch.cuda.synchronize()
        # eager work between replays
        _ = torch.arange(1000, device="cuda").sum().item()
        assert b.error_flag() == 0
        want = _oracle_serve(ref, b.requests_in_order(), total)
        _check_outputs(b.out.cpu().numpy(), b.requests_in_order(), want)
        ring, weyl, pos = gs.host_state()
        assert (pos == ref.pos).all() and (ring == ref.ring).all(), replay


def test_autotune_keeps_state_and_bits():
    rng = np.random.default_rng(3)
    reqs, total = _requests(rng, 200, 400, max_n=20000)
    gs = XorgensStreams(200, seed=4)
    before = gs.checkpoint()
    b = Batch(gs, reqs, total)
    best, recs = b.autotune(reps=1)
    torch.cuda.synchronize()
    assert torch.equal(before, gs.state)
    assert len(recs) > 10 and all(r[4] > 0 for r in recs)
    assert best in [r[:4] for r in recs]
    assert {r[3] for r in recs} == {1, 4}
    b.run(tune=best)
    out_best = b.out.clone()
    gs.restore(before)
    b.run(tune=None)
    assert torch.equal(out_best, b.out)


def test_batch_equals_plain_launch():
    gs_a = XorgensStreams(128, seed=42)
    gs_b = XorgensStreams(128, seed=42)
    n = 4096 + 17
    plain = gs_a.u32(n)
    reqs = [(i, n, i * n, 0) for i in range(128)]
    b = Batch(gs_b, reqs, 128 * n)
    b.run()
    assert torch.equal(plain.view(-1), b.out)
    assert torch.equal(gs_a.state, gs_b.state)


def test_batch_degenerate_tables():
    """An empty table launches nothing and leaves the state alone; a table of
    one-word requests (uint32, FP32, and a normal that consumes a pair) and
    zero-length requests serves exactly those words."""
    gs = XorgensStreams(5, seed=3)
    saved = gs.checkpoint()
    empty = Batch(gs, [], 0)
    empty.run()
    torch.cuda.synchronize()
    assert torch.equal(gs.state, saved) and empty.error_flag() == 0
    reqs = [(0, 1, 0, 0), (1, 1, 1, 1), (2, 1, 2, 2), (3, 0, 3, 0), (4, 0, 3, 2), (0, 1, 3, 0)]
    b = Batch(gs, reqs, 4)
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    ref = O.OracleStreams(3, 5)
    want = _oracle_serve(ref, b.requests_in_order(), 4)
    _check_outputs(b.out.cpu().numpy(), b.requests_in_order(), want)
    _, _, pos = gs.host_state()
    assert list(pos) == [2, 1, 2, 0, 0]
