"""xg_generate_batch_static, the batch entry point that allocates nothing
(its planner scratch is a file-scope device array of the library), against
xg_generate_batch with attached scratch: identical outputs, end states and
error words, on two calls in a row, the second with a smaller table."""
import numpy as np
import pytest

from gpu_helpers import needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402
from paper_1108_0486_amd.batch import Batch  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams, _stream_handle  # noqa: E402


def _table(rng, num_streams, num_reqs, max_n):
    reqs, off = [], 0
    for i in range(num_reqs):
        s = int(rng.integers(0, num_streams)) if i % 4 else 3
        n = int(rng.integers(0, max_n))
        dt = int(rng.integers(0, 3))
        reqs.append((s, n, off, dt))
        off += n + int(rng.integers(0, 5))
    return reqs, off


def _static_call(gs, b, out, err, key=None):
    xg.xg_generate_batch_static(gs.ctx, b.d_reqs.data_ptr(), b.num_reqs, out.data_ptr(), key, err.data_ptr(),
                                _stream_handle(None))


@pytest.mark.parametrize("family", [xg.XG_FAMILY_R128_W32, xg.XG_FAMILY_R64_W32, xg.XG_FAMILY_R64_W64])
def test_static_batch_equals_attached_scratch_twice(family):
    S = 300
    rng = np.random.default_rng(41 + family)
    a = XorgensStreams(S, seed=42, family=family)   # xg_generate_batch, attached scratch
    s = XorgensStreams(S, seed=42, family=family)   # xg_generate_batch_static
    err = torch.full((1,), 7, dtype=torch.int32, device=a.device)
    dtype = torch.int64 if family == xg.XG_FAMILY_R64_W64 else torch.int32
    for call, (num_reqs, max_n) in enumerate([(3000, 6000), (500, 900)]):   # the second table is smaller
        reqs, total = _table(rng, S, num_reqs, max_n)
        # both outputs start equal, so the gaps between requests compare too
        b = Batch(a, reqs, total, out=torch.full((max(1, total),), -1, dtype=dtype, device=a.device))
        b.run()
        out = torch.full((max(1, total),), -1, dtype=dtype, device=a.device)
        _static_call(s, b, out, err)
        torch.cuda.synchronize()
        assert b.error_flag() == 0 and int(err.item()) == 0, call
        assert torch.equal(out[:total], b.out[:total]), call
        assert torch.equal(a.state, s.state), call


def test_static_batch_reports_skipped_requests_and_refuses_oversize():
    a = XorgensStreams(10, seed=1)
    s = XorgensStreams(10, seed=1)
    reqs = [(2, 100, 0, 0), (10, 50, 100, 0), (3, 60, 150, 1), (4, 10, 210, 3), (2, 30, 220, 2)]
    b = Batch(a, reqs, 300, out=torch.zeros(300, dtype=torch.int32, device=a.device))
    b.run()
    out = torch.zeros(300, dtype=torch.int32, device=a.device)
    err = torch.zeros(1, dtype=torch.int32, device=a.device)
    _static_call(s, b, out, err)
    torch.cuda.synchronize()
    assert b.error_flag() == 1 and int(err.item()) == 1
    assert torch.equal(out, b.out) and torch.equal(a.state, s.state)
    # more requests than the static array holds: refused before anything runs
    big = torch.zeros((xg.XG_STATIC_MAX_REQS + 1) * 8, dtype=torch.int32, device=a.device)
    saved = s.checkpoint()
    with pytest.raises(xg.XgError) as e:
        xg.xg_generate_batch_static(s.ctx, big.data_ptr(), xg.XG_STATIC_MAX_REQS + 1, out.data_ptr())
    assert e.value.status == xg.XG_EBUSY
    torch.cuda.synchronize()
    assert torch.equal(saved, s.state)
    # and a clean call after it clears the error word again
    b2 = Batch(a, [(1, 64, 0, 0)], 64)
    b2.run()
    _static_call(s, b2, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and torch.equal(out[:64], b2.out[:64])


def test_static_batch_full_table_in_a_graph():
    """XG_STATIC_MAX_REQS requests (the array's limit), captured in a HIP graph
    and replayed twice with eager work between: each replay equals the
    attached-scratch call."""
    S = 4096
    rng = np.random.default_rng(9)
    n = rng.integers(1, 300, size=xg.XG_STATIC_MAX_REQS)
    st = rng.integers(0, S, size=xg.XG_STATIC_MAX_REQS)
    off = np.concatenate([[0], np.cumsum(n)])
    reqs = [(int(st[i]), int(n[i]), int(off[i]), int(i % 3)) for i in range(len(n))]
    total = int(off[-1])
    a = XorgensStreams(S, seed=3)
    s = XorgensStreams(S, seed=3)
    b = Batch(a, reqs, total)
    out = torch.zeros(total, dtype=torch.int32, device=a.device)
    err = torch.zeros(1, dtype=torch.int32, device=a.device)
    b.run()                                  # eager first: both advance by one table
    _static_call(s, b, out, err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0 and torch.equal(out, b.out[:total]) and torch.equal(a.state, s.state)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _static_call(s, b, out, err)
    for replay in range(2):
        b.run()
        g.replay()
        torch.cuda.synchronize()
        _ = torch.arange(100, device=a.device).sum().item()
        assert int(err.item()) == 0
        assert torch.equal(out, b.out[:total]), replay
        assert torch.equal(a.state, s.state), replay
