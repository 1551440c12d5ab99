"""A small statistical battery (a regression guard, not TestU01) and the
paper's linearity claim.

Section 1.5: an xorgens x-part alone is GF(2)-linear, and adding a Weyl
sequence with an integer add (Eq. (1)) removes that linearity.  The linear
complexity of one output bit shows it directly: 4096 for the x-part (its
minimal polynomial is the degree-4096 characteristic polynomial), about N/2
for N bits of the combined output, as for a random sequence.

The other checks use thresholds with false-alarm probabilities far below
1e-6, so they flag gross defects (a stuck bit, a broken lag, correlated
streams) without flaking.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _bits(words: np.ndarray, bit: int) -> np.ndarray:
    return ((words >> np.uint32(bit)) & np.uint32(1)).astype(np.uint8)


def test_weyl_combination_removes_linearity():
    N = 20000
    st = O.OracleStreams(42, 1)
    ring = st.ring[0].copy()
    out = st.u32(N)[0]
    _, xbits = O.xpart_run(O.PAPER, ring, N, bit=0, want_bits=True)
    lc_x = O.berlekamp_massey(xbits).bit_length() - 1
    assert lc_x == 4096
    for bit in (0, 15, 31):
        lc = O.berlekamp_massey(_bits(out, bit)).bit_length() - 1
        assert abs(lc - N / 2) <= 12, (bit, lc)   # random sequences: N/2 +- a few


def battery(words: np.ndarray) -> dict:
    """Monobit, byte chi-square, runs, lag-1 serial correlation, uniform moments."""
    words = np.ascontiguousarray(words, dtype=np.uint32).ravel()
    n = words.size
    res = {}
    ones = int(np.unpackbits(words.view(np.uint8)).sum())
    nbits = 32 * n
    res["monobit_z"] = (ones - nbits / 2) / math.sqrt(nbits / 4)
    counts = np.bincount(words.view(np.uint8), minlength=256).astype(np.float64)
    e = counts.sum() / 256
    res["byte_chi2"] = float(((counts - e) ** 2 / e).sum())            # 255 dof
    b0 = _bits(words, 0).astype(np.int8)
    runs = 1 + int(np.count_nonzero(b0[1:] != b0[:-1]))
    pi = b0.mean()
    res["runs_z"] = (runs - 2 * n * pi * (1 - pi)) / (2 * math.sqrt(n) * pi * (1 - pi))
    u = words.astype(np.float64) / 2**32
    res["serial_r"] = float(np.corrcoef(u[:-1], u[1:])[0, 1]) * math.sqrt(n - 1)
    res["mean_z"] = (u.mean() - 0.5) / math.sqrt(1 / 12 / n)
    res["var_z"] = (u.var() - 1 / 12) / math.sqrt(1 / 180 / n)
    return res


def assert_battery(res: dict):
    assert abs(res["monobit_z"]) < 6, res
    assert 150 < res["byte_chi2"] < 400, res          # 255 dof: both tails beyond 1e-6
    assert abs(res["runs_z"]) < 6, res
    assert abs(res["serial_r"]) < 6, res
    assert abs(res["mean_z"]) < 6, res
    assert abs(res["var_z"]) < 6, res


def test_battery_on_oracle_stream():
    assert_battery(battery(O.OracleStreams(42, 1).u32(1 << 22)[0]))


def test_battery_catches_a_stuck_bit():
    w = O.OracleStreams(42, 1).u32(1 << 20)[0] | np.uint32(1 << 7)
    with pytest.raises(AssertionError):
        assert_battery(battery(w))


def test_consecutive_seeds_are_uncorrelated():
    """Section 4: blocks are seeded with consecutive values; the seeding must
    keep neighbouring streams apart."""
    u = O.OracleStreams(42, 64).u32(1 << 14).astype(np.float64) / 2**32
    r = np.corrcoef(u)                      # 64 x 64 stream correlations
    off = r[~np.eye(64, dtype=bool)]
    assert np.abs(off).max() * math.sqrt(u.shape[1]) < 6
    # the xor of neighbouring streams is still balanced bit by bit
    x = (O.OracleStreams(42, 2).u32(1 << 18))
    assert_battery(battery(x[0] ^ x[1]))


@pytest.mark.gpu
def test_battery_on_gpu_bulk_fill():
    torch = pytest.importorskip("torch")
    from gpu_helpers import HAVE_GPU
    if not HAVE_GPU:
        pytest.skip("no GPU visible")
    from paper_1108_0486_amd.streams import XorgensStreams, as_u32
    gs = XorgensStreams(1024, seed=42)
    flat = as_u32(gs.fill_u32(1 << 16))
    assert_battery(battery(flat))
    del torch


@pytest.mark.parametrize("member", ["r64_w32", "r64_w64"])
def test_further_members_linearity_and_battery(member):
    """The same claims for the further family members: the x-part alone has
    linear complexity n (2048 or 4096), the Weyl-combined output about N/2
    (Section 1.5), and the outputs pass the battery."""
    p = O.R64 if member == "r64_w32" else O.W64
    N = 2 * p.n + 4000
    if p.w == 64:
        st = O.OracleStreams64(42, 1, p)
        ring = st.ring[0].copy()
        out = st.u64(N)[0]
        words = out.view(np.uint32)                       # both halves of every 64-bit output
        bits = [((out >> np.uint64(b)) & np.uint64(1)).astype(np.uint8) for b in (0, 31, 63)]
    else:
        st = O.OracleStreams(42, 1, params=p)
        ring = st.ring[0].copy()
        words = st.u32(N)[0]
        bits = [_bits(words, b) for b in (0, 15, 31)]
    _, xbits = O.xpart_run(p, ring, N, bit=0, want_bits=True)
    assert O.berlekamp_massey(xbits).bit_length() - 1 == p.n
    for b in bits:
        lc = O.berlekamp_massey(b).bit_length() - 1
        assert abs(lc - N / 2) <= 12, (member, lc)
    more = O.OracleStreams64(7, 1, p).u64(1 << 21)[0].view(np.uint32) if p.w == 64 else \
        O.OracleStreams(7, 1, params=p).u32(1 << 22)[0]
    assert_battery(battery(more))


@pytest.mark.gpu
@pytest.mark.parametrize("member", ["r64_w32", "r64_w64"])
def test_battery_on_gpu_further_members(member):
    pytest.importorskip("torch")
    from gpu_helpers import HAVE_GPU
    if not HAVE_GPU:
        pytest.skip("no GPU visible")
    from paper_1108_0486_amd import xg
    from paper_1108_0486_amd.streams import XorgensStreams
    if member == "r64_w32":
        gs = XorgensStreams(2048, seed=42, family=xg.XG_FAMILY_R64_W32)
        flat = gs.fill_u32(1 << 12).cpu().numpy().view(np.uint32)
    else:
        gs = XorgensStreams(2048, seed=42, family=xg.XG_FAMILY_R64_W64)
        flat = gs.fill_u64(1 << 11).cpu().numpy().view(np.uint32)
    assert_battery(battery(flat))


def birthday_spacings_collisions(words: np.ndarray, m: int = 512, k_bits: int = 24, rounds: int = 400) -> float:
    """Birthday spacings (Marsaglia): draw m birthdays in a year of 2^k_bits
    days (the top k_bits of each word), sort, take the spacings and count the
    values that occur more than once.  The count is approximately Poisson
    with mean m^3 / (4 2^k_bits); returns the z-score of the total over
    `rounds` independent groups."""
    d = (words[: m * rounds] >> np.uint32(32 - k_bits)).reshape(rounds, m).astype(np.int64)
    d.sort(axis=1)
    sp = np.diff(d, axis=1, prepend=0)
    sp.sort(axis=1)
    coll = int((np.diff(sp, axis=1) == 0).sum())
    lam = rounds * m**3 / (4 * 2**k_bits)
    return (coll - lam) / math.sqrt(lam)


def gap_test_chi2(words: np.ndarray, lo: float = 0.0, hi: float = 0.5, classes: int = 12) -> float:
    """Knuth's gap test: lengths of runs between successive uniforms falling
    in [lo, hi); a gap of length g has probability p (1 - p)^g, the last
    class collecting g >= classes - 1.  Returns the chi-square statistic
    (classes - 1 degrees of freedom)."""
    u = words.astype(np.float64) / 2**32
    hits = np.flatnonzero((u >= lo) & (u < hi))
    gaps = np.diff(hits) - 1
    p = hi - lo
    counts = np.bincount(np.minimum(gaps, classes - 1), minlength=classes).astype(np.float64)
    probs = np.array([p * (1 - p) ** g for g in range(classes - 1)] + [(1 - p) ** (classes - 1)])
    e = probs * gaps.size
    return float(((counts - e) ** 2 / e).sum())


def test_birthday_spacings_and_gap_on_oracle_streams():
    """Two more classical tests on the paper's member and the further members;
    thresholds far in the tails (false alarm << 1e-6)."""
    for words in (O.OracleStreams(42, 1).u32(1 << 21)[0],
                  O.OracleStreams(42, 1, params=O.R64).u32(1 << 21)[0],
                  O.OracleStreams64(42, 1, O.W64).u64(1 << 20)[0].view(np.uint32)):
        assert abs(birthday_spacings_collisions(words)) < 6
        assert gap_test_chi2(words) < 60                       # 11 dof: P(chi2 > 60) ~ 1e-8


def test_birthday_spacings_and_gap_catch_defects():
    """The two tests reject sequences with known defects: a lattice
    (k 69069 + 1 mod 2^32, whose spacings repeat) for birthday spacings, and
    a sequence whose uniforms avoid long gaps for the gap test."""
    lattice = ((np.arange(1 << 18, dtype=np.uint64) * np.uint64(69069) + np.uint64(1)) & np.uint64(0xFFFFFFFF))
    assert abs(birthday_spacings_collisions(lattice.astype(np.uint32))) > 6
    u = O.OracleStreams(42, 1).u32(1 << 20)[0]
    alternating = u.copy()
    alternating[::2] = alternating[::2] >> np.uint32(1)        # every other uniform < 1/2: gaps stay short
    assert gap_test_chi2(alternating) > 100
