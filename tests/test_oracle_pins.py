"""Pins of the CPU oracle to what the paper and the mathematics fix.

The paper (arXiv:1108.0486) prints no generated values, so the oracle is pinned
by: the GF(2) primitivity of the characteristic polynomial that its period
claim needs (Section 1.5, Table 1: period 2^4128 = (2^4096 - 1) 2^32), brute
force periods on tiny members of the family, jump-ahead in two independent
forms against stepping, linearity, the Weyl closed form, the published
SplitMix64 vector, and closed forms of the output mappings.  A plausible
mistake in the oracle (a swapped shift pair, a shift applied in the wrong
order, a lag off by one, a dropped Weyl term) fails at least one of them.
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from oracle import fermat as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def paper_poly():
    P = O.charpoly(O.PAPER)
    assert P.bit_length() - 1 == 4096
    return P


# ---------------------------------------------------------------------------
# building blocks of the GF(2) toolkit
# ---------------------------------------------------------------------------

def _clmul_ref(a, b):
    r = 0
    for i in range(64):
        if (a >> i) & 1:
            r ^= b << i
    return r


def _polymod_ref(a, P):
    dp = P.bit_length() - 1
    while a and a.bit_length() - 1 >= dp:
        a ^= P << (a.bit_length() - 1 - dp)
    return a


def test_clmul_matches_definition():
    rng = np.random.default_rng(1)
    for _ in range(200):
        a, b = (int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64))
        a |= int(rng.integers(0, 2)) << 63
        assert O.clmul64(a, b) == _clmul_ref(a, b)
        assert O.clmul64(a, b, portable=True) == _clmul_ref(a, b)


def test_mulmod_matches_long_division():
    rng = np.random.default_rng(2)
    for n in (5, 17, 64, 65, 130, 4096):
        P = (1 << n) | int(rng.integers(0, 2**62)) | 1
        if n > 62:
            P |= int.from_bytes(rng.bytes(n // 8), "little") & ((1 << n) - 1)
        for _ in range(3):
            a = int.from_bytes(rng.bytes(n // 8 + 1), "little") % (1 << n)
            b = int.from_bytes(rng.bytes(n // 8 + 1), "little") % (1 << n)
            prod = 0
            x = a
            i = 0
            while x:
                if x & 1:
                    prod ^= b << i
                x >>= 1
                i += 1
            assert O.mulmod(a, b, P) == _polymod_ref(prod, P)


def test_gcd_degree():
    # (z+1)(z^2+z+1) and (z+1)(z^3+z+1) share exactly z + 1
    a = 0b11 * 0  # placeholder to keep names short
    z1, q2, q3 = 0b11, 0b111, 0b1011

    def pm(x, y):
        r = 0
        i = 0
        while y:
            if y & 1:
                r ^= x << i
            y >>= 1
            i += 1
        return r
    assert O.gcd_degree(pm(z1, q2), pm(z1, q3)) == 1
    assert O.gcd_degree(q2, q3) == 0
    assert O.gcd_degree(pm(q2, q3), pm(q3, z1)) == 3
    del a


def test_berlekamp_massey_known_lfsr():
    # z^4 + z + 1 (primitive): s_k = s_{k-3} ^ s_{k-4}
    s = [1, 0, 0, 0]
    for k in range(4, 40):
        s.append(s[k - 3] ^ s[k - 4])
    assert O.berlekamp_massey(np.array(s, dtype=np.uint8)) == 0b10011
    assert O.is_primitive(0b10011) == 0
    # z^4 + z^3 + z^2 + z + 1 is irreducible but has order 5, not 15
    assert O.is_primitive(0b11111) != 0
    # z^4 + z^2 + 1 = (z^2 + z + 1)^2 is reducible
    assert O.is_primitive(0b10101) != 0


def test_primitivity_matches_known_degree_8_count():
    # There are phi(255) / 8 = 16 primitive polynomials of degree 8 over GF(2).
    count = sum(1 for low in range(0, 256) if O.is_primitive((1 << 8) | low) == 0)
    assert count == 16


# ---------------------------------------------------------------------------
# the factorisation of 2^4096 - 1
# ---------------------------------------------------------------------------

def test_fermat_factorisation_of_mersenne_4096():
    qs = F.mersenne_2pow_prime_factors(12)
    assert len(qs) == 25
    prod = 1
    for q in qs:
        prod *= q
    assert prod == 2**4096 - 1
    assert all(F.miller_rabin(q) for q in qs)
    assert not F.miller_rabin(F.fermat(5))          # composite F_5 is caught
    assert F.miller_rabin(F.fermat(4))


# ---------------------------------------------------------------------------
# the paper's member: period claim <=> primitive characteristic polynomial
# ---------------------------------------------------------------------------

def test_paper_parameters_are_primitive(paper_poly):
    """Section 2's (128,65,15,14,12,17), w = 32, with (I + L^a) acting before
    (I + R^b): the characteristic polynomial of the x-part has degree 4096 and
    is primitive, so its period is 2^4096 - 1 as the paper claims."""
    assert O.is_primitive(paper_poly, F.mersenne_2pow_prime_factors(12)) == 0
    # The same polynomial from another output bit and another start state.
    ring = np.random.default_rng(5).integers(0, 2**32, size=128, dtype=np.uint64).astype(np.uint32)
    assert O.charpoly(O.PAPER, ring=ring, bit=31) == paper_poly


def _variant_bits(order_right_first=False, swap=False, nbits=2 * 4096 + 64, s=65, shifts=(15, 14, 12, 17)):
    """Bit 0 of the x-part of a variant of the recurrence (pure Python)."""
    a, b, c, d = shifts
    if swap:
        a, b, c, d = c, d, a, b
    M = 0xFFFFFFFF

    def op(v, left, right):
        if order_right_first:
            v ^= v >> right
            v ^= (v << left) & M
        else:
            v ^= (v << left) & M
            v ^= v >> right
        return v
    x = [(i * 2654435761 + 12345) & M for i in range(128)]
    out = []
    for k in range(nbits):
        xk = op(x[k], a, b) ^ op(x[k + 128 - s], c, d)
        x.append(xk)
        out.append(xk & 1)
    return np.array(out, dtype=np.uint8)


def test_pure_python_variant_matches_oracle(paper_poly):
    assert O.berlekamp_massey(_variant_bits()) == paper_poly


@pytest.mark.parametrize("kw", [dict(swap=True), dict(swap=True, order_right_first=True),
                                dict(s=64), dict(s=66), dict(shifts=(14, 15, 12, 17)),
                                dict(shifts=(15, 14, 17, 12)), dict(shifts=(15, 14, 12, 16))])
def test_misread_parameters_are_not_primitive(kw):
    """Plausible misreadings of Section 2 (lags swapped between the shift
    pairs, s off by one, a shift pair transposed or off by one) fail the
    primitivity test, so the paper's period claim pins them."""
    P = O.berlekamp_massey(_variant_bits(**kw))
    if P.bit_length() - 1 == 4096:
        assert O.is_primitive(P, F.mersenne_2pow_prime_factors(12)) != 0


def test_shift_order_within_a_factor_is_not_pinned_by_primitivity(paper_poly):
    """Applying (I + R^b) before (I + L^a) gives the same characteristic
    polynomial, so primitivity cannot choose the order; the oracle follows the
    row-vector notation x (I + L^a)(I + R^b), where (I + L^a) acts first.  The
    two orders do give different outputs."""
    assert O.berlekamp_massey(_variant_bits(order_right_first=True)) == paper_poly
    assert not (_variant_bits(order_right_first=True, nbits=256) == _variant_bits(nbits=256)).all()


# ---------------------------------------------------------------------------
# tiny members: brute-force period <=> primitivity
# ---------------------------------------------------------------------------

TINY = [(4, 2, 1), (4, 4, 1), (4, 4, 3), (8, 2, 1), (4, 3, 1), (4, 3, 2)]


@pytest.mark.parametrize("w,r,s", TINY)
def test_tiny_members_brute_force_period(w, r, s):
    n = r * w
    full = 2**n - 1
    seen = {True: 0, False: 0}
    shifts = range(1, w)
    combos = list(itertools.product(shifts, repeat=4))
    for a, b, c, d in combos:
        p = O.Params(w=w, r=r, s=s, a=a, b=b, c=c, d=d, gamma=w // 2, omega=1)
        ring = np.zeros(r, dtype=np.uint32)
        ring[-1] = 1
        period = O.xpart_period(p, ring, full)
        P = O.charpoly(p, ring=ring)
        prim = (P.bit_length() - 1 == n) and O.is_primitive(P) == 0
        assert (period == full) == prim, (w, r, s, a, b, c, d, period)
        seen[prim] += 1
    assert seen[True] > 0 and seen[False] > 0


def test_tiny_full_period_with_weyl():
    """Section 1.5: the Weyl term multiplies the period by 2^w."""
    w, r, s = 4, 2, 1
    for a, b, c, d in itertools.product(range(1, w), repeat=4):
        p = O.Params(w=w, r=r, s=s, a=a, b=b, c=c, d=d, gamma=2, omega=0b1011)
        ring = np.array([0, 1], dtype=np.uint32)
        if O.xpart_period(p, ring, 2**8) == 255:
            assert O.full_period(p, ring, 3, 2**20) == 255 * 16
            return
    pytest.fail("no primitive member found")


def test_weyl_constant_from_golden_ratio():
    """omega is the odd integer nearest 2^31 (sqrt 5 - 1) (Section 1.5)."""
    exact = 2**31 * (math.sqrt(5) - 1)
    assert O.weyl_omega(32) == 0x9E3779B9 == O.PAPER.omega
    assert abs(O.PAPER.omega - exact) < 1 and O.PAPER.omega % 2 == 1
    assert O.PAPER.gamma == 16


# ---------------------------------------------------------------------------
# jump-ahead: matrix power == polynomial == stepping
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("J", [1, 63, 64, 4096])
def test_paper_jump_matrix_poly_step(paper_poly, J):
    st = O.OracleStreams(42, 1)
    ring = st.ring[0].copy()
    stepped, _ = O.xpart_run(O.PAPER, ring.copy(), J)
    g = O.z_pow_mod(J, paper_poly)
    by_poly = O.xpart_jump_poly(O.PAPER, ring, O.poly_to_words(g, 64))
    assert (by_poly == stepped).all()
    M = O.xpart_matrix(O.PAPER)
    by_mat = O.bits_to_ring(O.PAPER, O.mat_pow_apply(M, 4096, J, O.ring_to_bits(O.PAPER, ring)))
    assert (by_mat == stepped).all()


def test_paper_jump_poly_large(paper_poly):
    ring = O.OracleStreams(7, 1).ring[0].copy()
    J = 10**5
    stepped, _ = O.xpart_run(O.PAPER, ring.copy(), J)
    g = O.z_pow_mod(J, paper_poly)
    assert (O.xpart_jump_poly(O.PAPER, ring, O.poly_to_words(g, 64)) == stepped).all()
    # the full period returns to the start: z^(2^4096 - 1) == 1
    assert O.z_pow_mod(2**4096 - 1, paper_poly) == 1


def test_tiny_jump_matrix_vs_poly_huge_J():
    w, r, s = 8, 2, 1
    for a, b, c, d in itertools.product(range(1, w), repeat=4):
        p = O.Params(w=w, r=r, s=s, a=a, b=b, c=c, d=d, gamma=4, omega=1)
        ring = np.array([3, 200], dtype=np.uint32)
        P = O.charpoly(p, ring=ring)
        if P.bit_length() - 1 == 16 and O.is_primitive(P) == 0:
            break
    for J in (5, 65534, 2**40 + 12345, 3**50):
        stepped, _ = O.xpart_run(p, ring.copy(), J % (2**16 - 1))
        g = O.z_pow_mod(J, P)
        assert (O.xpart_jump_poly(p, ring, O.poly_to_words(g, 1)) == stepped).all()
        M = O.xpart_matrix(p)
        v = O.mat_pow_apply(M, 16, J, O.ring_to_bits(p, ring))
        assert (O.bits_to_ring(p, v) == stepped).all()


# ---------------------------------------------------------------------------
# linearity, Weyl closed form, seeding
# ---------------------------------------------------------------------------

def test_xpart_linearity():
    rng = np.random.default_rng(9)
    s1 = rng.integers(0, 2**32, size=128, dtype=np.uint64).astype(np.uint32)
    s2 = rng.integers(0, 2**32, size=128, dtype=np.uint64).astype(np.uint32)
    a, _ = O.xpart_run(O.PAPER, s1.copy(), 1000)
    b, _ = O.xpart_run(O.PAPER, s2.copy(), 1000)
    c, _ = O.xpart_run(O.PAPER, s1 ^ s2, 1000)
    assert (c == (a ^ b)).all()


def test_weyl_closed_form_and_combination():
    """out_k = x_k + (W_k xor (W_k >> 16)) mod 2^32 with W_k = W_{-1} + (k+1) omega."""
    st = O.OracleStreams(42, 1)
    ring0, w0 = st.ring[0].copy(), int(st.weyl[0])
    n = 5000
    out = st.u32(n)[0].astype(np.int64)
    x = []
    ring = ring0.copy()
    for _ in range(n):
        ring, _ = O.xpart_run(O.PAPER, ring, 1)
        x.append(int(ring[-1]))
    x = np.array(x, dtype=np.int64)
    k = np.arange(n, dtype=np.int64)
    W = (w0 + (k + 1) * O.PAPER.omega) % 2**32
    assert (((out - x) % 2**32) == (W ^ (W >> 16))).all()
    assert int(st.weyl[0]) == (w0 + n * O.PAPER.omega) % 2**32
    assert int(st.pos[0]) == n


def test_splitmix64_published_vector():
    want = [int(l, 16) for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if l.startswith("0x")]
    assert O.splitmix64_sequence(0, 3) == want


def test_seeding_reading():
    """INIT-v1: ring from the high halves of SplitMix64, then 4r discarded
    steps; stream i uses seed + i."""
    seed = 42
    vals = O.splitmix64_sequence(seed, 129)
    p = O.PAPER
    # rebuild the pre-warm-up state and run 512 discarded outputs
    pre = O.OracleStreams.from_state(np.array([v >> 32 for v in vals[:128]], dtype=np.uint32),
                                     np.array([vals[128] >> 32], dtype=np.uint32),
                                     np.array([0], dtype=np.uint64))
    pre.skip(4 * p.r)
    st = O.OracleStreams(seed, 3)
    assert (st.ring[0] == pre.ring[0]).all() and st.weyl[0] == pre.weyl[0] and st.pos[0] == 0
    one = O.OracleStreams(seed + 2, 1)
    assert (one.ring[0] == st.ring[2]).all()
    assert (O.OracleStreams(seed, 1, first=2).ring[0] == st.ring[2]).all()


def test_split_call_invariance():
    a = O.OracleStreams(42, 4)
    b = a.copy()
    whole = a.u32(3000)
    parts = np.concatenate([b.u32(1000), b.u32(999), b.u32(1001)], axis=1)
    assert (whole == parts).all()
    assert (a.ring == b.ring).all() and (a.weyl == b.weyl).all() and (a.pos == b.pos).all()


def test_threads_do_not_change_results():
    a = O.OracleStreams(100, 9).u32(777, threads=1)
    b = O.OracleStreams(100, 9).u32(777, threads=4)
    assert (a == b).all()


# ---------------------------------------------------------------------------
# the section 2 dependency analysis (chunked evaluation of the ring)
# ---------------------------------------------------------------------------

def _chunked(ring, nwords, C, mode):
    """Evaluates x_k for k >= 0 in chunks of C terms on a circular buffer of
    r = 128 words.  mode "phased": every term of a chunk reads its operands,
    then every term writes (one wavefront step).  mode "adversarial": terms run
    from the last to the first, each writing right after its own reads."""
    M = 0xFFFFFFFF
    buf = [int(v) for v in ring]
    out = []

    def A(v):
        v ^= (v << 15) & M
        return v ^ (v >> 14)

    def B(v):
        v ^= (v << 12) & M
        return v ^ (v >> 17)
    k = 0
    while k < nwords:
        lanes = range(min(C, nwords - k))
        if mode == "phased":
            vals = [A(buf[(k + j) % 128]) ^ B(buf[(k + j + 128 - 65) % 128]) for j in lanes]
            for j in lanes:
                buf[(k + j) % 128] = vals[j]
        else:
            vals = [0] * len(lanes)
            for j in reversed(lanes):
                vals[j] = A(buf[(k + j) % 128]) ^ B(buf[(k + j + 128 - 65) % 128])
                buf[(k + j) % 128] = vals[j]
        out.extend(vals)
        k += len(lanes)
    return out


def test_parallel_chunk_bound():
    """Section 2: terms x_k .. x_{k+C-1} are independent for C <= s when all
    reads precede all writes; with arbitrary interleaving of reads and writes
    on the shared r-word buffer the safe bound is r - s = 63, the paper's
    min(s, r - s)."""
    ring = O.OracleStreams(42, 1).ring[0].copy()
    ref, _ = O.xpart_run(O.PAPER, ring.copy(), 1000, bit=0)
    seq = []
    rr = ring.copy()
    for _ in range(1000):
        rr, _ = O.xpart_run(O.PAPER, rr, 1)
        seq.append(int(rr[-1]))
    for C in (1, 16, 63, 64, 65):
        assert _chunked(ring, 1000, C, "phased") == seq
    assert _chunked(ring, 1000, 66, "phased") != seq
    assert _chunked(ring, 1000, 63, "adversarial") == seq
    assert _chunked(ring, 1000, 64, "adversarial") != seq
    del ref


# ---------------------------------------------------------------------------
# output mappings
# ---------------------------------------------------------------------------

def test_f32_mapping_exact():
    st = O.OracleStreams(42, 1)
    ref = st.copy().u32(100000)[0]
    f = st.f32(100000)[0]
    assert (f.astype(np.float64) * 2**24 == (ref >> 8).astype(np.float64)).all()
    assert f.min() >= 0.0 and f.max() < 1.0


def test_box_muller_special_cases_and_invariants():
    top = (2**24 - 1) << 8
    z0, z1 = O.box_muller64(top, 0)          # u1 = 1 -> rho = 0
    assert z0 == 0.0 and z1 == 0.0
    z0, z1 = O.box_muller64(0, 0)            # u1 = 2^-24, u2 = 0
    rho = math.sqrt(-2 * math.log(2.0**-24))
    assert z0 == pytest.approx(rho, rel=1e-15) and z1 == 0.0
    for quarter, (c, s) in {1: (0, 1), 2: (-1, 0), 3: (0, -1)}.items():
        z0, z1 = O.box_muller64(0, (quarter << 22) << 8)   # u2 = quarter / 4
        assert z0 == pytest.approx(c * rho, abs=0) and z1 == pytest.approx(s * rho, abs=0)
    rng = np.random.default_rng(3)
    for _ in range(2000):
        e, o = (int(v) for v in rng.integers(0, 2**32, size=2, dtype=np.uint64))
        u1 = ((e >> 8) + 1) * 2.0**-24
        u2 = (o >> 8) * 2.0**-24
        z0, z1 = O.box_muller64(e, o)
        assert z0 * z0 + z1 * z1 == pytest.approx(-2 * math.log(u1), rel=1e-13, abs=1e-300)
        if u1 < 1:
            ang = math.atan2(z1, z0) % (2 * math.pi)
            d = abs(ang - 2 * math.pi * u2)
            assert min(d, 2 * math.pi - d) < 1e-12


def test_box_muller_many_is_the_pairwise_map():
    """The oracle's vectorised map (used for the exhaustive GPU sweeps) is the
    pair map itself, pair by pair, in every thread slice."""
    rng = np.random.default_rng(4)
    words = rng.integers(0, 2**32, size=2 * 3001, dtype=np.uint64).astype(np.uint32)
    words[:2] = [(2**24 - 1) << 8, 0]                     # u1 = 1
    z = O.box_muller_many(words, threads=3)
    assert z.shape == (3001, 2)
    for m in range(3001):
        assert tuple(z[m]) == O.box_muller64(int(words[2 * m]), int(words[2 * m + 1])), m


def test_normals_pairing_and_moments():
    st = O.OracleStreams(42, 2)
    u = st.copy().u32(1002)
    z = st.copy().normal(1001)
    for i in range(2):
        for m in range(0, 1001, 2):
            z0, z1 = O.box_muller64(int(u[i, m]), int(u[i, m + 1]))
            assert z[i, m] == z0
            if m + 1 < 1001:
                assert z[i, m + 1] == z1
    # odd n consumes 2 ceil(n/2) words
    s2 = st.copy()
    s2.normal(1001)
    assert (s2.pos == 1002).all()
    mom = st.copy().moments(1001)
    assert np.allclose(mom[:, 0], z.sum(axis=1), rtol=0, atol=1e-9)
    assert np.allclose(mom[:, 1], (z * z).sum(axis=1), rtol=1e-14)
    assert np.allclose(mom[:, 2], np.abs(z).sum(axis=1), rtol=1e-14)


def test_normals_are_standard():
    z = O.OracleStreams(11, 16).normal(1 << 16).ravel()
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 0.01


def test_stored_digests_match_oracle():
    """The stored digests (written by tests/golden/make_golden.py from the
    oracle) still describe the oracle."""
    import hashlib
    lines = dict(l.split(" ", 1) for l in open(os.path.join(GOLDEN, "single_stream_seed42_2p20.txt"))
                 if not l.startswith("#"))
    st = O.OracleStreams(42, 1)
    u = st.u32(1 << 20)[0]
    assert hashlib.sha256(u.tobytes()).hexdigest() == lines["sha256_le_u32"].strip()
    assert int(lines["final_weyl"], 16) == int(st.weyl[0])
