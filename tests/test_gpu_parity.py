"""HIP path against the CPU oracle, through the C ABI, element by element.

Sizes span several 64-word chunks, unroll groups and ragged tails; every
launch shape is checked to give identical bits.  u32 and f32 are bit-exact;
normals are within 4 FP32 ulp of the FP64 oracle; moments are within the
stated bound.
"""
import numpy as np
import pytest

from gpu_helpers import needs_gpu, ulp32_error
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams, as_u32  # noqa: E402

RAGGED_NS = [1, 2, 31, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 513, 1000, 4133]


def _assert_state(gs: XorgensStreams, os_: O.OracleStreams, idx=None):
    ring, weyl, pos = gs.host_state(idx)
    assert (ring == os_.ring).all()
    assert (weyl == os_.weyl).all()
    assert (pos == os_.pos).all()


def test_seeding_matches_oracle():
    gs = XorgensStreams(257, seed=42)
    torch.cuda.synchronize()
    _assert_state(gs, O.OracleStreams(42, 257))


def test_seeding_large_seed_wraps():
    gs = XorgensStreams(5, seed=2**64 - 2)
    torch.cuda.synchronize()
    _assert_state(gs, O.OracleStreams(2**64 - 2, 5))


@pytest.mark.parametrize("n", RAGGED_NS)
def test_u32_ragged_lengths(n):
    gs = XorgensStreams(70, seed=1234)
    ref = O.OracleStreams(1234, 70)
    sub = ref.subset(range(3, 70))
    out = gs.u32(n, first=3, count=67)
    torch.cuda.synchronize()
    assert (as_u32(out) == sub.u32(n)).all()
    ref_after = O.OracleStreams.from_state(np.concatenate([ref.ring[:3], sub.ring]),
                                           np.concatenate([ref.weyl[:3], sub.weyl]),
                                           np.concatenate([ref.pos[:3], sub.pos]))
    _assert_state(gs, ref_after)


@pytest.mark.parametrize("n", [1, 64, 65, 1000, 4133])
def test_f32_ragged_lengths(n):
    gs = XorgensStreams(33, seed=77)
    ref = O.OracleStreams(77, 33)
    out = gs.f32(n).cpu().numpy()
    want = ref.f32(n)
    assert out.dtype == np.float32 and (out.view(np.uint32) == want.view(np.uint32)).all()
    _assert_state(gs, ref)


def test_zero_length_is_noop():
    gs = XorgensStreams(4, seed=5)
    before = gs.checkpoint()
    out = torch.empty((4, 0), dtype=torch.int32, device="cuda")
    gs.u32(0, out=out)
    torch.cuda.synchronize()
    assert torch.equal(before, gs.state)


def test_sequential_calls_mixed_types():
    gs = XorgensStreams(9, seed=99)
    ref = O.OracleStreams(99, 9)
    for kind, n in [("u32", 100), ("f32", 777), ("normal", 333), ("u32", 64), ("normal", 128),
                    ("f32", 1), ("u32", 5000)]:
        if kind == "u32":
            assert (as_u32(gs.u32(n)) == ref.u32(n)).all(), (kind, n)
        elif kind == "f32":
            assert (gs.f32(n).cpu().numpy() == ref.f32(n)).all(), (kind, n)
        else:
            err = ulp32_error(gs.normal(n).cpu().numpy(), ref.normal(n))
            assert err.max() <= 4.0, (kind, n, err.max())
        _assert_state(gs, ref)


PLAIN_SHAPES = [(w, u, 1) for w in (1, 2, 4, 8, 16) for u in (1, 2, 4, 8)] + \
               [(w, u, 4) for w in (1, 2, 4, 8, 16) for u in (4, 8)]


@pytest.mark.parametrize("wpb,unroll,store_words", PLAIN_SHAPES)
def test_plain_shapes_identical(wpb, unroll, store_words):
    n = 64 * 37 + 37
    gs = XorgensStreams(37, seed=3)
    gs.set_plain_tune(wpb, unroll, store_words)
    assert gs.plain_tune() == (wpb, unroll, store_words)
    ref = O.OracleStreams(3, 37)
    assert (as_u32(gs.u32(n)) == ref.u32(n)).all()
    assert (gs.f32(n).cpu().numpy() == ref.f32(n)).all()
    z = gs.normal(2 * 64 * 9 + 77).cpu().numpy()
    assert ulp32_error(z, ref.normal(2 * 64 * 9 + 77)).max() <= 4.0
    _assert_state(gs, ref)


@pytest.mark.parametrize("n", [256 * 5, 256 * 5 + 64, 256 * 9 + 3])
def test_wide_stores_with_unaligned_output(n):
    """16-byte stores are used only while the output is 16-byte aligned; a
    4-byte-aligned output takes the 4-byte path with the same bits."""
    gs = XorgensStreams(6, seed=21)
    gs.set_plain_tune(1, 8, 4)
    ref = O.OracleStreams(21, 6)
    buf = torch.zeros(6 * n + 1, dtype=torch.int32, device="cuda")
    out = buf[1:].view(6, n)
    gs.u32(n, out=out)
    assert (as_u32(out) == ref.u32(n)).all() and buf[0].item() == 0
    _assert_state(gs, ref)


def test_default_plain_shape():
    gs = XorgensStreams(2, seed=1)
    assert gs.plain_tune() == (0, 0, 4)
    gs.set_plain_tune(0, 4, 1)
    assert gs.plain_tune() == (0, 4, 1)
    gs.set_plain_tune(2, 0, 0)                 # automatic unroll, default store width
    assert gs.plain_tune() == (2, 0, 4)


@pytest.mark.parametrize("full", [False, True])
@pytest.mark.parametrize("kind", ["fill_u32", "fill_f32", "u32", "f32"])
def test_automatic_unroll_matches_oracle(kind, full):
    """The automatic shape gives the oracle's bits, with a ragged length
    (13 chunks and 5 words: an odd chunk count leaves a remainder for every
    unroll), like every explicit shape.  `full`: a wavefront on every SIMD,
    where the uint32 fill takes unroll 4 and stream-major unroll 2 with
    4-byte stores (the uint32 one paced); otherwise unroll 8."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    count, n = (4 * cus + 5 if full else 9), 64 * 13 + 5
    gs = XorgensStreams(count, seed=77)
    ref = O.OracleStreams(77, count)
    want = ref.u32(n) if kind.endswith("u32") else ref.f32(n)
    if kind.startswith("fill"):
        got = getattr(gs, kind)(n)
        idx = torch.as_tensor(xg.fill_index(count, n), device="cuda")
        got = got[idx].view(count, n)
    else:
        got = getattr(gs, kind)(n)
    got = as_u32(got) if kind.endswith("u32") else got.cpu().numpy()
    assert (got == want).all()
    _assert_state(gs, ref)


@pytest.mark.parametrize("count", [1, 255, 256, 511, 512, 1023, 1024, 1025, 2049])
def test_auto_shape_counts(count):
    """The automatic waves-per-block choice around the compute-unit multiples
    gives the same bits (and touches only the selected streams)."""
    gs = XorgensStreams(count + 2, seed=13)
    ref = O.OracleStreams(13, count + 2)
    sub = ref.subset(range(1, 1 + count))
    n = 130
    assert (as_u32(gs.u32(n, first=1, count=count)) == sub.u32(n)).all()
    flat = as_u32(gs.fill_u32(n, first=1, count=count))
    assert (flat[xg.fill_index(count, n)] == sub.u32(n)).all()
    _, _, pos = gs.host_state()
    assert pos[0] == 0 and pos[-1] == 0 and (pos[1:-1] == 2 * n).all()


def test_split_calls_equal_one_call():
    a = XorgensStreams(16, seed=8)
    b = XorgensStreams(16, seed=8)
    whole = as_u32(a.u32(10_000))
    parts = np.concatenate([as_u32(b.u32(k)) for k in (1, 63, 64, 65, 3000, 6807)], axis=1)
    assert (whole == parts).all()
    assert torch.equal(a.state, b.state)


@pytest.mark.parametrize("n", [1, 2, 3, 127, 128, 129, 130, 255, 256, 1001, 10_001])
def test_normals_within_4_ulp(n):
    gs = XorgensStreams(33, seed=2024)
    ref = O.OracleStreams(2024, 33)
    z = gs.normal(n).cpu().numpy()
    err = ulp32_error(z, ref.normal(n))
    assert err.max() <= 4.0, err.max()
    _assert_state(gs, ref)


def test_normals_unaligned_output_pointer():
    n = 1001
    gs = XorgensStreams(5, seed=31)
    ref = O.OracleStreams(31, 5)
    buf = torch.zeros(5 * n + 1, dtype=torch.float32, device="cuda")
    out = buf[1:].view(5, n)              # 4-byte but not 8-byte aligned
    gs.normal(n, out=out)
    z = out.cpu().numpy()
    assert ulp32_error(z, ref.normal(n)).max() <= 4.0
    assert buf[0].item() == 0.0


def test_normals_many_variates_ulp():
    gs = XorgensStreams(64, seed=42)
    ref = O.OracleStreams(42, 64)
    z = gs.normal(1 << 16).cpu().numpy()
    err = ulp32_error(z, ref.normal(1 << 16))
    assert err.max() <= 4.0, err.max()


def test_moments_bound():
    n = 1 << 16
    gs = XorgensStreams(64, seed=42)
    ref = O.OracleStreams(42, 64)
    zref = ref.copy().normal(n)
    m = gs.moments(n).cpu().numpy().astype(np.float64)
    mref = ref.moments(n)
    tau = 27 * 2.0**-24
    assert (np.abs(m[:, 0] - mref[:, 0]) <= tau * np.abs(zref).sum(axis=1)).all()
    assert (np.abs(m[:, 1] - mref[:, 1]) <= tau * (zref * zref).sum(axis=1)).all()
    _assert_state(gs, ref)


def test_moments_odd_and_tiny():
    for n in (1, 3, 129, 1001):
        gs = XorgensStreams(7, seed=6)
        ref = O.OracleStreams(6, 7)
        zref = ref.normal(n)
        m = gs.moments(n).cpu().numpy().astype(np.float64)
        assert np.allclose(m[:, 0], zref.sum(axis=1), rtol=0, atol=27 * 2.0**-24 * np.abs(zref).sum() + 1e-7)
        _assert_state(gs, ref)


@pytest.mark.parametrize("n", [1, 2, 127, 128, 129, 301, 1000])
def test_normals_same_bits_under_both_pair_gathers(n):
    """A launch of at least eight streams per compute unit (two wavefronts per
    SIMD) gathers each Box-Muller pair through LDS; smaller launches gather it
    with a DPP lane swap.  The same streams in one launch and in launches of
    a quarter of that size give identical normals and end states, equal to
    the oracle's within 4 ulp on sampled streams; the fused moments of both
    forms are within the bound."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    S = 8 * cus
    big = XorgensStreams(S, seed=19)
    small = XorgensStreams(S, seed=19)
    za = big.normal(n)
    zb = torch.cat([small.normal(n, first=k, count=S // 4) for k in range(0, S, S // 4)])
    torch.cuda.synchronize()
    assert torch.equal(za.view(torch.int32), zb.view(torch.int32))
    assert torch.equal(big.state, small.state)
    rows = [0, 1, 2, S // 4 - 1, S // 2 + 3, S - 1]
    ref = O.OracleStreams(19, S).subset(rows)
    err = ulp32_error(za.cpu().numpy()[rows], ref.normal(n))
    assert err.max() <= 4.0, err.max()
    tau = 27 * 2.0**-24
    for launches in (1, 4):
        gs = XorgensStreams(S, seed=23)
        m = torch.cat([gs.moments(n, first=k, count=S // launches) for k in range(0, S, S // launches)])
        m = m.cpu().numpy().astype(np.float64)[rows]
        zref = O.OracleStreams(23, S).subset(rows).normal(n)
        assert (np.abs(m[:, 0] - zref.sum(axis=1)) <= tau * np.abs(zref).sum(axis=1) + 1e-30).all()
        assert (np.abs(m[:, 1] - (zref * zref).sum(axis=1)) <= tau * (zref * zref).sum(axis=1) + 1e-30).all()


def test_range_errors_leave_state_untouched():
    gs = XorgensStreams(8, seed=1)
    before = gs.checkpoint()
    out = torch.empty((8, 16), dtype=torch.int32, device="cuda")
    with pytest.raises(xg.XgError) as e:
        xg.xg_generate_u32(gs.ctx, 4, 5, 16, out.data_ptr(), 0)
    assert e.value.status == xg.XG_ERANGE
    with pytest.raises(xg.XgError) as e:
        xg.xg_generate_u32(gs.ctx, 0, 8, 16, out.data_ptr() + 2, 0)
    assert e.value.status == xg.XG_EALIGN
    with pytest.raises(xg.XgError) as e:
        xg.xg_generate_u32(gs.ctx, 0, 0, 16, out.data_ptr(), 0)
    assert e.value.status == xg.XG_EINVAL
    with pytest.raises(xg.XgError):
        gs.set_plain_tune(3, 4)
    torch.cuda.synchronize()
    assert torch.equal(before, gs.state)


def test_checkpoint_resume():
    gs = XorgensStreams(12, seed=10)
    gs.u32(999)
    saved = gs.checkpoint()
    first = as_u32(gs.u32(4321))
    gs.restore(saved)
    again = as_u32(gs.u32(4321))
    assert (first == again).all()
    # attach a fresh handle to a copy of the saved state
    other = XorgensStreams.attach(saved.clone(), 12)
    assert (as_u32(other.u32(4321)) == first).all()


def test_streams_are_independent_of_neighbours():
    a = XorgensStreams(100, seed=500)
    b = XorgensStreams(1, seed=537)
    assert (as_u32(a.u32(3000, first=37, count=1)) == as_u32(b.u32(3000))).all()


@pytest.mark.parametrize("count,n", [(1, 1), (5, 64), (7, 65), (33, 1000), (67, 64 * 19 + 37), (3, 8 * 64)])
def test_fill_layout_matches_oracle(count, n):
    gs = XorgensStreams(70, seed=55)
    ref = O.OracleStreams(55, 70)
    sub = ref.subset(range(2, 2 + count))
    flat = as_u32(gs.fill_u32(n, first=2, count=count))
    assert flat.shape == (count * n,)
    want = sub.u32(n)
    assert (flat[xg.fill_index(count, n)] == want).all()
    f = gs.fill_f32(n, first=2, count=count).cpu().numpy()
    assert (f[xg.fill_index(count, n)] == sub.f32(n)).all()
    ring, weyl, pos = gs.host_state(list(range(2, 2 + count)))
    assert (ring == sub.ring).all() and (weyl == sub.weyl).all() and (pos == sub.pos).all()


@pytest.mark.parametrize("wpb,unroll", [(1, 1), (2, 2), (4, 4), (16, 8), (1, 8)])
def test_fill_shapes_identical(wpb, unroll):
    gs = XorgensStreams(40, seed=8)
    gs.set_plain_tune(wpb, unroll, 1)
    ref = O.OracleStreams(8, 40)
    n = 64 * 21 + 5
    flat = as_u32(gs.fill_u32(n))
    assert (flat[xg.fill_index(40, n)] == ref.u32(n)).all()


def test_fill_unaligned_buffer():
    gs = XorgensStreams(9, seed=2)
    ref = O.OracleStreams(2, 9)
    n = 300
    buf = torch.zeros(9 * n + 1, dtype=torch.int32, device="cuda")
    gs.fill_u32(n, out=buf[1:])
    flat = as_u32(buf)[1:]
    assert (flat[xg.fill_index(9, n)] == ref.u32(n)).all() and buf[0].item() == 0
