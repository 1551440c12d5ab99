"""Edge cases at the limits of the method and of the index arithmetic.

- The degenerate state: an all-zero x-part ring stays zero (Section 2's
  recurrence is linear), so the outputs are the tempered Weyl sequence alone
  (Section 1.5, Eq. (1)); the GPU must reproduce it from an attached state.
- Offsets beyond 2^32 elements: two streams of 2^31 + 77 words each, in the
  stream-major and the bulk-fill layouts (4 * (2^32 + 154) bytes of output),
  checked against the oracle at the start, the ragged end and the far end of
  each stream, so a 32-bit index overflow anywhere shows.
- Batch requests placed past 2^32 elements of the output (one crossing it,
  one long request split into tiles beyond it), through the one-call and the
  host-planned batch paths.
"""
import numpy as np
import pytest

from gpu_helpers import needs_gpu
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams, as_u32  # noqa: E402


def test_zero_ring_gives_the_tempered_weyl_sequence():
    S = 3
    words = np.zeros((S, xg.XG_STATE_WORDS), dtype=np.uint32)
    weyl = np.array([0, 0x9E3779B9, 0xFFFFFFFF], dtype=np.uint32)
    words[:, 128] = weyl
    words[:, 130] = [0, 5, 1 << 20]                          # positions (low words)
    state = torch.from_numpy(words.view(np.int32).ravel().copy()).cuda()
    gs = XorgensStreams.attach(state, S)
    got = as_u32(gs.u32(4133))
    ref = O.OracleStreams.from_state(np.zeros((S, 128), dtype=np.uint32), weyl,
                                     np.array([0, 5, 1 << 20], dtype=np.uint64))
    want = ref.u32(4133)
    assert (got == want).all()
    k = np.arange(1, 4134, dtype=np.uint64)
    W = ((weyl[:, None].astype(np.uint64) + k[None, :] * np.uint64(0x9E3779B9)) & np.uint64(0xFFFFFFFF))
    assert (want == (W ^ (W >> np.uint64(16))).astype(np.uint32)).all()   # x-part contributes nothing
    ring, _, pos = gs.host_state()
    assert (ring == 0).all() and (pos == np.array([4133, 4138, (1 << 20) + 4133])).all()


def _oracle_slices(seed, count, n, starts, length):
    """Oracle words [s, s + length) of each stream for each start s (in order)."""
    out = {}
    ref = O.OracleStreams(seed, count)
    pos = 0
    for s in sorted(starts):
        assert s >= pos, "slices must not overlap"
        if s > pos:
            ref.skip(s - pos)
        out[s] = ref.u32(length)
        pos = s + length
    return out


@pytest.mark.parametrize("layout", ["stream_major", "fill"])
def test_offsets_beyond_2p32_elements(layout):
    count, n = 2, (1 << 31) + 77
    L = 4096
    gs = XorgensStreams(count, seed=99)
    if layout == "stream_major":
        out = gs.u32(n).view(-1)                            # [count * n], element k n + t
        at = lambda k, t: k * n + t                         # noqa: E731
    else:
        out = gs.fill_u32(n)
        full, rem = n // 64, n % 64
        at = lambda k, t: (t // 64) * 64 * count + k * 64 + t % 64 if t < 64 * full else \
            64 * full * count + k * rem + (t - 64 * full)   # noqa: E731
    assert out.numel() == count * n and count * n > 2**32
    starts = [0, (1 << 31) - 3 * L, n - L]                 # the last slice crosses 2^31 words
    ref = _oracle_slices(99, count, n, starts, L)
    for s in starts:
        for k in range(count):
            idx = torch.as_tensor([at(k, t) for t in range(s, s + L)], dtype=torch.int64, device="cuda")
            got = as_u32(out[idx])
            assert (got == ref[s][k]).all(), (layout, k, s)
    del out
    torch.cuda.synchronize()
    _, _, pos = gs.host_state()
    assert (pos == n).all()


@pytest.mark.parametrize("words", [1, 3, 4, 5, 1000, 1 << 20, (1 << 26) + 7])
def test_fill_value_reference_kernel(words):
    out = torch.full((words + 8,), -1, dtype=torch.int32, device="cuda")
    xg.xg_fill_value(out.data_ptr(), words, 0x12345678, torch.cuda.current_stream().cuda_stream)
    a = out.cpu().numpy().view(np.uint32)
    assert (a[:words] == 0x12345678).all() and (a[words:] == 0xFFFFFFFF).all()
    with pytest.raises(xg.XgError) as e:
        xg.xg_fill_value(out.data_ptr() + 4, 8, 1)
    assert e.value.status == xg.XG_EALIGN


@pytest.mark.parametrize("path", ["device", "planned"])
def test_batch_offsets_beyond_2p32_elements(path):
    """A request that straddles element 2^32 of a 16 GiB output, one that
    starts past it (FP32), and one long request whose tiles of 2^16 words all
    lie past it (one-call path only; the planned path serves it whole): every
    word equals the oracle's and nothing else in the buffer changes."""
    from paper_1108_0486_amd.batch import Batch, PlannedBatch
    L = 1 << 16
    base = 1 << 32
    reqs = [(0, 5000, base - 100, 0), (1, 3000, base + 12345, 1), (2, 3 * L + 17, base + 50000, 0)]
    total = base + 50000 + 3 * L + 17 + 64
    out = torch.full((total,), -1, dtype=torch.int32, device="cuda")
    gs = XorgensStreams(3, seed=5)
    if path == "device":
        b = Batch(gs, reqs, total, out=out, tile_words=L, max_tiles=64)
    else:
        b = PlannedBatch(gs, reqs, total, out=out)
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    if path == "device":
        rows, _ = b.served_plan()
        assert sum(1 for r in rows if r[4]) == 4              # stream 2's request as 4 tiles
    ref = O.OracleStreams(5, 3)
    for st, n, off, dt in reqs:
        one = ref.subset([st])
        want = one.u32(n)[0] if dt == 0 else one.f32(n)[0].view(np.uint32)
        got = as_u32(out[off - 8:off + n + 8]).astype(np.uint32)
        assert (got[8:8 + n] == want).all(), (st, off)
        assert (got[:8] == 0xFFFFFFFF).all() and (got[8 + n:] == 0xFFFFFFFF).all(), st   # neighbours untouched
    _, _, pos = gs.host_state()
    assert list(pos) == [5000, 3000, 3 * L + 17]
    del out, b
    torch.cuda.empty_cache()
