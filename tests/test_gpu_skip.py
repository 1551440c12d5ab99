"""xg_skip: advancing streams by J words, by stepping (J < 2^15) and by the
polynomial jump (J >= 2^15), against the oracle's stepping and, for J too
large to step, the oracle's matrix form (and its own polynomial jump)."""
import numpy as np
import pytest

from gpu_helpers import huge_skip_digests, needs_gpu, ring_digest
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd.streams import XorgensStreams, as_u32  # noqa: E402


def _assert_state(gs, ref):
    ring, weyl, pos = gs.host_state()
    assert (ring == ref.ring).all() and (weyl == ref.weyl).all() and (pos == ref.pos).all()


@pytest.mark.parametrize("J", [1, 63, 64, 65, 1000, 32767, 32768, 32769, 100_000, (1 << 20) + 7])
def test_skip_equals_stepping(J):
    gs = XorgensStreams(37, seed=42)
    gs.u32(129)                     # start from a position that is not chunk-aligned
    ref = O.OracleStreams(42, 37)
    ref.u32(129)
    gs.skip(J)
    ref.skip(J)
    _assert_state(gs, ref)
    assert (as_u32(gs.u32(300)) == ref.u32(300)).all()


@pytest.mark.parametrize("J", [2**32 + 5, 2**50 + 3, 2**63 + 1])
def test_skip_huge_equals_matrix_form(J):
    """Skips far beyond stepping.  The expected rings are the oracle's matrix
    form (T^J by binary powering of the one-step bit matrix; stored digests
    written by tests/golden/make_golden.py), which shares no method with the
    library's jump polynomial; the oracle's own polynomial jump must agree."""
    gs = XorgensStreams(5, seed=7)
    ref = O.OracleStreams(7, 5)
    want = huge_skip_digests()
    P = O.charpoly(O.PAPER)
    g = O.poly_to_words(O.z_pow_mod(J, P), 64)
    gs.skip(J)
    ring, weyl, pos = gs.host_state()
    for i in range(5):
        assert ring_digest(ring[i]) == want[("r128_w32", 7, i, J)], i
        assert (ring[i] == O.xpart_jump_poly(O.PAPER, ref.ring[i], g)).all()
    assert (weyl == ((ref.weyl.astype(np.uint64) + np.uint64(J % 2**32) * np.uint64(O.PAPER.omega))
                     % np.uint64(2**32)).astype(np.uint32)).all()
    assert (pos == np.uint64(J)).all()


def test_skip_subset_only():
    gs = XorgensStreams(10, seed=3)
    ref = O.OracleStreams(3, 10)
    gs.skip(50_000, first=4, count=3)
    sub = ref.subset(range(4, 7))
    sub.skip(50_000)
    ring, weyl, pos = gs.host_state()
    assert (ring[4:7] == sub.ring).all() and (pos[4:7] == 50_000).all()
    assert (pos[:4] == 0).all() and (pos[7:] == 0).all() and (ring[:4] == ref.ring[:4]).all()


def test_skip_then_generate_equals_generate_then_discard():
    a = XorgensStreams(64, seed=11)
    b = XorgensStreams(64, seed=11)
    a.skip(3 * 2**17 + 5)
    b.u32(3 * 2**17 + 5)
    assert torch.equal(a.state, b.state)
    assert torch.equal(a.u32(5000), b.u32(5000))


@pytest.mark.parametrize("J", [(1 << 20) + 3, 2**40 + 777, 2**64 - 1])
def test_skip_both_jump_kernels_agree(J):
    """Jumps of at most 3 streams per compute unit run one workgroup per
    stream (the window sums split over its wavefronts); larger launches run
    one wavefront per stream.  The same streams through both launch forms
    end in the same states, which equal the oracle's polynomial jump on
    sampled streams and its stepping where that is short enough."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    S = 3 * cus + 1
    a = XorgensStreams(S, seed=13)
    b = XorgensStreams(S, seed=13)
    a.skip(J)                                   # one wavefront per stream
    b.skip(J, first=0, count=S - 1)             # one workgroup per stream
    b.skip(J, first=S - 1, count=1)
    assert torch.equal(a.state, b.state)
    rows = [0, 1, S // 2, S - 2, S - 1]
    ref = O.OracleStreams(13, S).subset(rows)
    g = O.poly_to_words(O.z_pow_mod(J, O.charpoly(O.PAPER)), 64)
    ring, _, pos = a.host_state(rows)
    for j in range(len(rows)):
        assert (ring[j] == O.xpart_jump_poly(O.PAPER, ref.ring[j], g)).all(), rows[j]
    assert (pos == J).all()
    if J < 1 << 21:
        ref.skip(J)
        assert (ring == ref.ring).all()
