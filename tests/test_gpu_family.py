"""The further family members on the GPU against the oracle, through the C ABI.

XG_FAMILY_R64_W32 (w = 32, r = 64, s = 33) and XG_FAMILY_R64_W64 (w = 64,
r = 64, s = 33) run two streams per wavefront, 32 words per stream per step.
Sizes span several steps, unroll groups and ragged tails, odd stream counts
(a wavefront with one stream) and offsets; every value is bit-exact against
the oracle, and so is the state left behind.
"""
import numpy as np
import pytest

from gpu_helpers import huge_skip_digests, needs_gpu, ring_digest, ulp32_error, ulp64_error
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams  # noqa: E402

R64W32, R64W64 = xg.XG_FAMILY_R64_W32, xg.XG_FAMILY_R64_W64
PARAMS = {R64W32: O.R64, R64W64: O.W64}
FAMS = [R64W32, R64W64]
RAGGED = [1, 2, 31, 32, 33, 63, 64, 65, 255, 256, 257, 1000, 4133]


def _oracle(fam, seed, count, first=0):
    p = PARAMS[fam]
    if p.w == 64:
        return O.OracleStreams64(seed, count, p, first=first)
    return O.OracleStreams(seed, count, first=first, params=p)


def _sub(ref, lo, hi):
    if isinstance(ref, O.OracleStreams64):
        return O.OracleStreams64.from_state(ref.ring[lo:hi], ref.weyl[lo:hi], ref.pos[lo:hi], ref.params)
    return ref.subset(range(lo, hi))


def _bits(t):
    a = t.cpu().numpy()
    return a.view(np.uint64) if a.dtype.itemsize == 8 else a.view(np.uint32)


def _words(gs, fam, n, first=0, count=None, fp=False, fill=False):
    if fam == R64W64:
        f = {(False, False): gs.u64, (True, False): gs.f64, (False, True): gs.fill_u64, (True, True): gs.fill_f64}
    else:
        f = {(False, False): gs.u32, (True, False): gs.f32, (False, True): gs.fill_u32, (True, True): gs.fill_f32}
    return f[(fp, fill)](n, first=first, count=count)


def _ref_words(ref, fam, n, fp=False):
    if fam == R64W64:
        return ref.f64(n) if fp else ref.u64(n)
    return ref.f32(n) if fp else ref.u32(n)


def _assert_state(gs, ref, idx=None):
    ring, weyl, pos = gs.host_state(idx)
    assert (ring == ref.ring).all() and (weyl == ref.weyl).all() and (pos == ref.pos).all()


@pytest.mark.parametrize("fam", FAMS)
@pytest.mark.parametrize("count", [1, 2, 7, 258])
def test_family_seeding_matches_oracle(fam, count):
    gs = XorgensStreams(count, seed=42, family=fam)
    torch.cuda.synchronize()
    assert xg.xg_family(gs.ctx) == fam
    _assert_state(gs, _oracle(fam, 42, count))


@pytest.mark.parametrize("fam", FAMS)
def test_family_seed_wraps(fam):
    gs = XorgensStreams(3, seed=2**64 - 2, family=fam)
    torch.cuda.synchronize()
    _assert_state(gs, _oracle(fam, 2**64 - 2, 3))


@pytest.mark.parametrize("fam", FAMS)
@pytest.mark.parametrize("n", RAGGED)
def test_family_words_ragged(fam, n):
    """Streams 3 .. 35 of 37 (33 streams: the last wavefront holds one)."""
    gs = XorgensStreams(37, seed=1234, family=fam)
    ref = _oracle(fam, 1234, 37)
    sub = _sub(ref, 3, 36)
    got = _bits(_words(gs, fam, n, first=3, count=33))
    assert (got == _ref_words(sub, fam, n)).all()
    gotf = _words(gs, fam, n, first=3, count=33, fp=True).cpu().numpy()
    assert (gotf == _ref_words(sub, fam, n, fp=True)).all()
    torch.cuda.synchronize()
    _assert_state(gs, sub, idx=list(range(3, 36)))
    _assert_state(gs, _sub(ref, 0, 3), idx=[0, 1, 2])          # untouched neighbours
    _assert_state(gs, _sub(ref, 36, 37), idx=[36])


@pytest.mark.parametrize("fam", FAMS)
@pytest.mark.parametrize("n", [1, 31, 32, 33, 100, 1024, 4133])
@pytest.mark.parametrize("count", [1, 6, 9])
def test_family_fill_layout(fam, n, count):
    gs = XorgensStreams(count + 2, seed=5, family=fam)
    ref = _sub(_oracle(fam, 5, count + 2), 1, count + 1)
    flat = _bits(_words(gs, fam, n, first=1, count=count, fill=True))
    idx = xg.fill_index(count, n, chunk=32)
    assert (flat[idx] == _ref_words(ref, fam, n)).all()
    assert np.array_equal(np.sort(idx.ravel()), np.arange(count * n))
    flatf = _words(gs, fam, n, first=1, count=count, fp=True, fill=True).cpu().numpy()
    assert (flatf[idx] == _ref_words(ref, fam, n, fp=True)).all()
    torch.cuda.synchronize()
    _assert_state(gs, ref, idx=list(range(1, count + 1)))


@pytest.mark.parametrize("fam", FAMS)
def test_family_launch_shapes_identical(fam):
    outs = []
    for wpb, unroll in [(1, 1), (2, 2), (4, 4), (16, 8), (0, 8)]:
        gs = XorgensStreams(45, seed=9, family=fam)
        gs.set_plain_tune(wpb, unroll, 1)
        outs.append(_bits(_words(gs, fam, 2049)))
        outs.append(_bits(_words(gs, fam, 300, fill=True)))
    for k in range(2, len(outs), 2):
        assert (outs[k] == outs[0]).all() and (outs[k + 1] == outs[1]).all()
    ref = _oracle(fam, 9, 45)
    assert (outs[0] == _ref_words(ref, fam, 2049)).all()


@pytest.mark.parametrize("fam", FAMS)
def test_family_split_calls_and_checkpoint(fam):
    gs = XorgensStreams(10, seed=3, family=fam)
    saved = gs.checkpoint()
    whole = _bits(_words(gs, fam, 1000))
    gs.restore(saved)
    parts = np.concatenate([_bits(_words(gs, fam, k)) for k in (31, 1, 500, 468)], axis=1)
    assert (parts == whole).all()
    again = XorgensStreams.attach(saved.clone(), 10, family=fam)
    assert (_bits(_words(again, fam, 1000)) == whole).all()


@pytest.mark.parametrize("fam", FAMS)
def test_family_unsupported_calls_are_rejected(fam):
    gs = XorgensStreams(4, seed=1, family=fam)
    out = torch.empty(4 * 64, dtype=torch.float64, device="cuda")
    p = out.data_ptr()
    if fam == R64W64:
        calls = [lambda: xg.xg_generate_normal(gs.ctx, 0, 4, 8, p), lambda: xg.xg_normal_moments(gs.ctx, 0, 4, 8, p),
                 lambda: xg.xg_generate_u32(gs.ctx, 0, 4, 8, p), lambda: xg.xg_fill_f32(gs.ctx, 0, 4, 8, p)]
    else:
        calls = [lambda: xg.xg_generate_u64(gs.ctx, 0, 4, 8, p), lambda: xg.xg_fill_f64(gs.ctx, 0, 4, 8, p),
                 lambda: xg.xg_generate_normal_f64(gs.ctx, 0, 4, 8, p),
                 lambda: xg.xg_normal_moments_f64(gs.ctx, 0, 4, 8, p)]
    for c in calls:
        with pytest.raises(xg.XgError) as e:
            c()
        assert e.value.status == xg.XG_ENOTSUP
    from paper_1108_0486_amd.serve import Server
    with pytest.raises(xg.XgError) as e:  # served, but without jump-ahead segments
        Server(gs, pool_elems=1 << 12, num_lanes=1, max_batch=4, segment_words=1 << 12)
    assert e.value.status == xg.XG_ENOTSUP
    paper = XorgensStreams(4, seed=1)
    for c in (xg.xg_generate_u64, xg.xg_generate_normal_f64, xg.xg_normal_moments_f64):
        with pytest.raises(xg.XgError) as e:
            c(paper.ctx, 0, 4, 8, p)
        assert e.value.status == xg.XG_ENOTSUP
    torch.cuda.synchronize()
    _assert_state(gs, _oracle(fam, 1, 4))                      # nothing ran


def test_w64_bulk_full_size_sampled():
    """2048 streams x 2^18 uint64 in the bulk-fill layout (4 GiB, the launch
    the benchmark times), then FP64; sampled streams against the oracle, and
    every stream's end position."""
    count, n = 2048, 1 << 18
    gs = XorgensStreams(count, seed=42, family=R64W64)
    flat = gs.fill_u64(n)
    picks = [0, 1, 2, 777, 1024, 2046, 2047]
    t = np.arange(n, dtype=np.int64)                          # n is a multiple of 32: no ragged tail
    idx = np.stack([(t // 32) * 32 * count + k * 32 + t % 32 for k in picks])
    ref = O.OracleStreams64(42, count, O.W64)
    sel = O.OracleStreams64.from_state(ref.ring[picks], ref.weyl[picks], ref.pos[picks], O.W64)
    want = sel.u64(n)
    pos = torch.as_tensor(idx.ravel(), device="cuda")
    got = flat[pos].cpu().numpy().view(np.uint64).reshape(len(picks), n)
    assert (got == want).all()
    del flat
    f = gs.fill_f64(n)
    gotf = f[pos].cpu().numpy().reshape(len(picks), n)
    assert (gotf == sel.f64(n)).all()
    del f
    torch.cuda.synchronize()
    _, _, p = gs.host_state()
    assert (p == 2 * n).all()


def _oracle_after_skip(fam, seed, count, J, idx):
    """Oracle state of streams idx after skipping J words: by stepping for
    small J, else by the oracle's own polynomial jump (pinned to stepping by
    the oracle tests) with W advanced by J omega."""
    p = PARAMS[fam]
    ref = _oracle(fam, seed, count)
    if J <= 2_000_000:
        sub = _sub(ref, idx[0], idx[-1] + 1)
        sub.skip(J)
        return sub
    P = O.charpoly(p)
    g = O.poly_to_words(O.z_pow_mod(J, P), p.n // 64)
    mask = (1 << p.w) - 1
    wt = np.uint64 if p.w == 64 else np.uint32
    rings = np.stack([O.xpart_jump_poly(p, ref.ring[i], g) for i in idx]).astype(wt)
    weyl = np.array([(int(ref.weyl[i]) + J * p.omega) & mask for i in idx], dtype=wt)
    pos = np.array([int(ref.pos[i]) + J for i in idx], dtype=np.uint64)
    if p.w == 64:
        return O.OracleStreams64.from_state(rings, weyl, pos, p)
    return O.OracleStreams.from_state(rings, weyl, pos, params=p)


@pytest.mark.parametrize("fam", FAMS)
@pytest.mark.parametrize("J", [1, 31, 32, 33, 1000, (1 << 15) - 1, 1 << 15, 10**6 + 7, 2**40 + 5, 2**63 + 1])
def test_family_skip_matches_oracle(fam, J):
    """xg_skip on the further members: stepping below 2^15 words, jump-ahead
    (z^J mod P evaluated on the device in 32-word Horner steps) above; streams
    1 .. 5 of 7, so an odd count and untouched neighbours are covered."""
    gs = XorgensStreams(7, seed=21, family=fam)
    gs.skip(J, first=1, count=5)
    idx = [1, 2, 3, 4, 5]
    want = _oracle_after_skip(fam, 21, 7, J, idx)
    torch.cuda.synchronize()
    _assert_state(gs, want, idx=idx)
    if J > 2_000_000:
        # also the oracle's matrix form (stored digests; no jump polynomial)
        digests = huge_skip_digests()
        name = "r64_w64" if PARAMS[fam].w == 64 else "r64_w32"
        ring, _, _ = gs.host_state()
        for i in idx:
            assert ring_digest(ring[i]) == digests[(name, 21, i, J)], i
    _assert_state(gs, _sub(_oracle(fam, 21, 7), 6, 7), idx=[6])
    got = _bits(_words(gs, fam, 1000, first=1, count=5))
    assert (got == _ref_words(want, fam, 1000)).all()


@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 63, 64, 65, 127, 128, 1000, 4133])
def test_r64w32_normals_match_oracle(n):
    """Box-Muller normals of the 32-bit member on consecutive output pairs:
    within 4 FP32 ulp of the FP64 oracle; odd n consumes 2 ceil(n / 2) words.
    Streams 3 .. 35 of 37 (the last wavefront holds one stream)."""
    gs = XorgensStreams(37, seed=11, family=R64W32)
    ref = _sub(_oracle(R64W32, 11, 37), 3, 36)
    z = gs.normal(n, first=3, count=33).cpu().numpy()
    zr = ref.normal(n)
    assert ulp32_error(z, zr).max() <= 4.0
    torch.cuda.synchronize()
    _assert_state(gs, ref, idx=list(range(3, 36)))
    # the words after the normals continue the stream
    assert (_bits(gs.u32(100, first=3, count=33)) == ref.u32(100)).all()


@pytest.mark.parametrize("n", [1, 64, 65, 1000, 4133, 1 << 16])
def test_r64w32_moments_within_bound(n):
    """Fused sums of z and z^2 within tau = 27 u of the FP64 oracle's (relative
    to sum |z| and sum z^2), as for Section 2's member."""
    gs = XorgensStreams(21, seed=5, family=R64W32)
    ref = _oracle(R64W32, 5, 21)
    m = gs.moments(n).cpu().numpy().astype(np.float64)
    mr = ref.moments(n)
    tau = 27 * 2.0**-24
    assert (np.abs(m[:, 0] - mr[:, 0]) <= tau * mr[:, 2]).all()
    assert (np.abs(m[:, 1] - mr[:, 1]) <= tau * mr[:, 1]).all()
    torch.cuda.synchronize()
    _assert_state(gs, ref)


@pytest.mark.parametrize("n", [1, 2, 31, 32, 33, 63, 64, 65, 127, 128, 1000, 4133])
def test_w64_normals_f64_match_oracle(n):
    """FP64 Box-Muller normals of the 64-bit member (53-bit uniforms):
    within 4 FP64 ulp of the oracle's long-double values rounded to double;
    odd n consumes 2 ceil(n / 2) words.  Streams 3 .. 35 of 37 (the last
    wavefront holds one stream)."""
    gs = XorgensStreams(37, seed=13, family=R64W64)
    ref = _sub(_oracle(R64W64, 13, 37), 3, 36)
    z = gs.normal_f64(n, first=3, count=33).cpu().numpy()
    zr = ref.normal(n)
    err = ulp64_error(z, zr)
    assert err.max() <= 4.0, err.max()
    torch.cuda.synchronize()
    _assert_state(gs, ref, idx=list(range(3, 36)))
    assert (_bits(gs.u64(100, first=3, count=33)) == ref.u64(100)).all()


@pytest.mark.parametrize("misalign", [False, True])
def test_w64_normals_f64_output_alignment(misalign):
    """Pairs go out as 16-byte stores only from a 16-byte-aligned buffer; an
    8-byte-aligned one takes single stores with the same values."""
    count, n = 5, 258
    gs = XorgensStreams(count, seed=2, family=R64W64)
    buf = torch.full((count * n + 1,), -7.0, dtype=torch.float64, device="cuda")
    out = (buf[1:] if misalign else buf[:-1]).view(count, n)
    gs.normal_f64(n, out=out)
    zr = _oracle(R64W64, 2, count).normal(n)
    assert ulp64_error(out.cpu().numpy(), zr).max() <= 4.0
    assert buf[0 if misalign else -1].item() == -7.0


def test_w64_normals_f64_large_sample():
    """2048 streams x 2^13 normals (the launch shape of a full wave of pairs
    per SIMD): every value within 4 FP64 ulp; the worst is printed."""
    count, n = 2048, 1 << 13
    gs = XorgensStreams(count, seed=42, family=R64W64)
    z = gs.normal_f64(n).cpu().numpy()
    zr = _oracle(R64W64, 42, count).normal(n)
    err = ulp64_error(z, zr)
    print("FP64 normals: max error %.3f ulp over %d values" % (err.max(), err.size))
    assert err.max() <= 4.0


@pytest.mark.parametrize("n", [1, 2, 64, 65, 1000, 4133, 1 << 16])
def test_w64_moments_f64_within_bound(n):
    """Fused FP64 sums of z and z^2 of the 64-bit member within tau = 27 u
    (u = 2^-53) of the oracle's long-double sums, relative to sum |z| and
    sum z^2: variates within 4 ulp (8 u), the pair add or square-and-FMA
    (1 u / 2 u), the lane's compensated sum (2 u), its fold (1 u) and a
    5-level tree over the stream's 32 lanes (5 u) give at most 17 u and
    26 u.  The streams then continue as the oracle's."""
    gs = XorgensStreams(21, seed=5, family=R64W64)
    ref = _oracle(R64W64, 5, 21)
    m = gs.moments_f64(n).cpu().numpy()
    mr = ref.moments(n)
    tau = 27 * 2.0**-53
    e1 = np.abs(m[:, 0] - mr[:, 0]) / mr[:, 2]
    e2 = np.abs(m[:, 1] - mr[:, 1]) / mr[:, 1]
    print("FP64 moments n=%d: max rel err %.3g, %.3g (bound %.3g)" % (n, e1.max(), e2.max(), tau))
    assert (e1 <= tau).all() and (e2 <= tau).all()
    torch.cuda.synchronize()
    _assert_state(gs, ref)
    assert (_bits(gs.u64(70)) == ref.u64(70)).all()


def test_w64_normals_f64_exact_special_values():
    """The FP64 map's exact cases, forced through attached states.  With an
    all-zero x-part ring the outputs are the tempered Weyl values alone,
    out = W xor (W >> 32) (Section 1.5, Eq. (1)), so a chosen W_0 fixes the
    words: out = 0xFFFFFFFF_FFFFF800 gives u1 = 1 (both normals exactly 0);
    out = k 2^62 gives u2 = k / 4 (a quarter turn: one normal exactly 0, the
    other +-rho).  Each stream's W_{-1} = W_0 - omega; the GPU must equal the
    oracle from the same states, with the exact zeros and signs."""
    omega = O.W64.omega
    m64 = (1 << 64) - 1
    # stream 0: word 0 gives u1 = 1; streams 1..4: word 1 gives u2 = k / 4
    w0s = [0xFFFFFFFF000007FF]
    for k in range(4):
        w1 = (k << 62) | (k << 30)                       # out_1 = W ^ (W >> 32) = k 2^62
        w0s.append((w1 - omega) & m64)
    S = len(w0s)
    words = np.zeros((S, 66), dtype=np.uint64)             # ring u64[64] | W | pos
    words[:, 64] = [(w - omega) & m64 for w in w0s]
    state = torch.from_numpy(words.view(np.int64).ravel().copy()).cuda()
    gs = XorgensStreams.attach(state, S, family=R64W64)
    ref = O.OracleStreams64.from_state(np.zeros((S, 64), dtype=np.uint64), words[:, 64].copy(),
                                       np.zeros(S, dtype=np.uint64), O.W64)
    z = gs.normal_f64(4).cpu().numpy()
    zr = ref.normal(4)
    assert z[0, 0] == 0.0 and z[0, 1] == 0.0 and zr[0, 0] == 0.0 and zr[0, 1] == 0.0
    for k in range(4):
        c, s = [(1, 0), (0, 1), (-1, 0), (0, -1)][k]
        z0, z1 = z[1 + k, 0], z[1 + k, 1]
        assert (z0 == 0.0) == (c == 0) and (z1 == 0.0) == (s == 0), (k, z0, z1)
        assert np.sign(z0) == c or c == 0, k
        assert np.sign(z1) == s or s == 0, k
    assert ulp64_error(z, zr).max() <= 4.0


@pytest.mark.parametrize("fp", [False, True])
def test_r64w32_automatic_shape_every_simd(fp):
    """With a wavefront on every SIMD (8 x CUs + 3 streams of the 32-bit r = 64
    member; the last wavefront holds one stream) the automatic shape takes
    unroll 2 for stream-major and 8 for the fill: both layouts equal the
    oracle at a ragged length (13 steps and 5 words), and so do the states."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    count, n = 8 * cus + 3, 32 * 13 + 5
    gs = XorgensStreams(count, seed=19, family=R64W32)
    ref = _oracle(R64W32, 19, count)
    sm = _bits(gs.f32(n)) if fp else _bits(gs.u32(n))
    want = _ref_words(ref, R64W32, n, fp=fp)
    assert (sm == (want.view(np.uint32) if fp else want)).all()
    fill = _bits(gs.fill_f32(n) if fp else gs.fill_u32(n))
    want = _ref_words(ref, R64W32, n, fp=fp)
    idx = xg.fill_index(count, n, chunk=32)
    assert (fill[idx] == (want.view(np.uint32) if fp else want)).all()
    torch.cuda.synchronize()
    _assert_state(gs, ref)
