"""Jump-ahead at large J, pinned by methods that share nothing.

The x-part of xorgens is GF(2)-linear (Section 1.5): its n-bit state moves by
a matrix T, so the state after J steps is T^J applied to the start state.
Three routes reach it here:

  * the oracle's matrix form: T built column by column from single steps of
    the recurrence, T^J by binary powering of bit matrices (no polynomial);
  * libxg's jump polynomial z^J mod P (P from Krylov vectors, powers through
    the Frobenius map), applied to the state by the oracle's g(T) evaluation;
  * the oracle's own jump polynomial (P by Berlekamp-Massey, products with a
    Barrett reduction), and a plain pure-Python square-and-multiply with
    long division modulo that P.

All of them must give the same state for every family member at J far
beyond what stepping can check.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1108_0486_amd import xg

MEMBERS = [(xg.XG_FAMILY_R128_W32, O.PAPER), (xg.XG_FAMILY_R64_W32, O.R64), (xg.XG_FAMILY_R64_W64, O.W64)]
BIG_J = [2**20 + 7, 2**32 + 5, 2**50 + 3, 2**63 + 1]


def _start_ring(p):
    if p.w == 64:
        return O.OracleStreams64(7, 1, p).ring[0]
    return O.OracleStreams(7, 1, params=p).ring[0]


def _pymulmod(a: int, b: int, P: int, n: int) -> int:
    """a b mod P on Python ints (bit i = coefficient of z^i): shift-and-XOR
    product, then long division from the top bit down."""
    r = 0
    while b:
        low = b & -b
        r ^= a << (low.bit_length() - 1)
        b ^= low
    for i in range(r.bit_length() - 1, n - 1, -1):
        if (r >> i) & 1:
            r ^= P << (i - n)
    return r


def _py_z_pow(J: int, P: int, n: int) -> int:
    acc, base = 1, 2
    while J:
        if J & 1:
            acc = _pymulmod(acc, base, P, n)
        J >>= 1
        if J:
            base = _pymulmod(base, base, P, n)
    return acc


@pytest.mark.slow
@pytest.mark.parametrize("fam,p", MEMBERS, ids=["r128_w32", "r64_w32", "r64_w64"])
def test_large_jumps_agree_with_the_matrix_form(fam, p):
    n = p.n
    ring = _start_ring(p)
    M = O.xpart_matrix(p)
    v0 = O.ring_to_bits(p, ring)
    want = O.mat_pow_apply_many(M, n, BIG_J, np.stack([v0] * len(BIG_J)))
    P = O.charpoly(p)
    for j, J in enumerate(BIG_J):
        expect = O.bits_to_ring(p, want[j])
        g_lib = xg.xg_family_jump_polynomial(fam, J)
        assert (O.xpart_jump_poly(p, ring, O.poly_to_words(g_lib, n // 64)) == expect).all(), J
        g_orc = O.z_pow_mod(J, P)
        assert g_orc == g_lib, J
        assert (O.xpart_jump_poly(p, ring, O.poly_to_words(g_orc, n // 64)) == expect).all(), J


@pytest.mark.parametrize("fam,p", MEMBERS, ids=["r128_w32", "r64_w32", "r64_w64"])
def test_jump_polynomials_equal_plain_python_powering(fam, p):
    P = O.charpoly(p)
    assert P.bit_length() - 1 == p.n
    for J in (2**32 + 5, 2**63 + 1, 2**64 - 1):
        assert xg.xg_family_jump_polynomial(fam, J) == _py_z_pow(J, P, p.n), J


def test_matrix_form_agrees_with_stepping():
    """The matrix route itself, against plain stepping, at small J."""
    for p in (O.PAPER, O.W64):
        ring = _start_ring(p)
        M = O.xpart_matrix(p)
        Js = [1, 65, 1000, 4099]
        got = O.mat_pow_apply_many(M, p.n, Js, np.stack([O.ring_to_bits(p, ring)] * len(Js)))
        for j, J in enumerate(Js):
            if p.w == 64:
                ref = O.OracleStreams64.from_state(ring[None, :], np.zeros(1, np.uint64), np.zeros(1, np.uint64), p)
            else:
                ref = O.OracleStreams.from_state(ring[None, :], np.zeros(1, np.uint32), np.zeros(1, np.uint64), p)
            ref.skip(J)
            assert (O.bits_to_ring(p, got[j]) == ref.ring[0]).all(), (p.w, J)


def test_family_jump_polynomial_arguments():
    with pytest.raises(xg.XgError) as e:
        xg.xg_family_jump_polynomial(3, 5)
    assert e.value.status == xg.XG_EINVAL
    assert xg.xg_family_jump_polynomial(xg.XG_FAMILY_R64_W32, 0) == 1
    assert xg.xg_family_jump_polynomial(xg.XG_FAMILY_R64_W64, 1) == 2


def test_stored_matrix_form_digests_agree_with_the_oracle_polynomial_jump():
    """The stored large-skip rings (matrix form, written by
    tests/golden/make_golden.py) against the oracle's polynomial route."""
    import hashlib
    from gpu_helpers import huge_skip_digests
    params = {"r128_w32": O.PAPER, "r64_w32": O.R64, "r64_w64": O.W64}
    for (name, seed, stream, J), digest in huge_skip_digests().items():
        p = params[name]
        ref = O.OracleStreams64(seed, stream + 1, p) if p.w == 64 else O.OracleStreams(seed, stream + 1, params=p)
        g = O.poly_to_words(O.z_pow_mod(J, O.charpoly(p)), p.n // 64)
        ring = O.xpart_jump_poly(p, ref.ring[stream], g)
        assert hashlib.sha256(ring.tobytes()).hexdigest() == digest, (name, stream, J)
