"""Python face of the CPU oracle (plain C in xorgens_oracle.c, xorgens64_oracle.c
and gf2.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and
by the CPU-baseline leg of bench.py.  The product package never imports it,
and it imports nothing from the product package.

The oracle is the plain definition of xorgens as used by xorgensGP
(arXiv:1108.0486): the recurrence of Section 2, the Weyl generator and the
output combination of Section 1.5, Eq. (1), the parameter set of Section 2, run
one word at a time.  Readings where the paper is silent (Weyl constant, gamma,
seeding, the uniform / normal mappings) are listed in the header of
xorgens_oracle.c.

Stream state is held as three numpy arrays (ring[count, r] with
ring[i, t] = x_{pos-r+t}, weyl[count] = W_{pos-1}, pos[count]).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ("xorgens_oracle.c", "xorgens64_oracle.c", "gf2.c")

U32, F32, NORMAL, MOMENTS, SKIP = 0, 1, 2, 3, 4


def build(force: bool = True) -> str:
    """Compiles liboracle.so with gcc (plain -O2, no hand SIMD in the generator)."""
    if not force and os.path.exists(_LIB_PATH):
        built = os.path.getmtime(_LIB_PATH)
        if all(os.path.getmtime(os.path.join(_HERE, s)) <= built for s in _SOURCES):
            return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-std=gnu11", "-O2", "-fPIC", "-shared", "-mpclmul", "-msse4.1",
           *[os.path.join(_HERE, s) for s in _SOURCES], "-o", tmp, "-lpthread", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("w", "r", "s", "a", "b", "c", "d", "gamma", "omega")]


class _Params64(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint32) for n in ("w", "r", "s", "a", "b", "c", "d", "gamma")] + \
        [("omega", ctypes.c_uint64)]


@dataclass(frozen=True)
class Params:
    """A member of the xorgens family: word size w, lags r > s, shifts a..d,
    Weyl constant omega and output shift gamma."""
    w: int
    r: int
    s: int
    a: int
    b: int
    c: int
    d: int
    gamma: int
    omega: int

    @property
    def n(self) -> int:
        return self.r * self.w

    def c_struct(self):
        if self.w == 64:
            return _Params64(self.w, self.r, self.s, self.a, self.b, self.c, self.d, self.gamma, self.omega)
        return _Params(self.w, self.r, self.s, self.a, self.b, self.c, self.d, self.gamma,
                       self.omega & 0xFFFFFFFF)


# Section 2: (r,s,a,b,c,d) = (128,65,15,14,12,17) for w = 32.  omega is the odd
# integer nearest 2^31 (sqrt(5) - 1) (Section 1.5); gamma = w / 2 (Section 1.5
# asks for a value close to w / 2).
PAPER = Params(w=32, r=128, s=65, a=15, b=14, c=12, d=17, gamma=16, omega=0x9E3779B9)

# Further members (Section 1.5: n = r w any power of two up to 4096; Section 2:
# s = r/2 +- 1 for the GPU).  The paper gives no shifts for them: these are
# the choices of family_search.py (shifts in [w/4, 3w/4], seeded order, the
# primitive candidate whose characteristic polynomial weight is nearest n/2),
# and the tests pin each by primitivity.
R64 = Params(w=32, r=64, s=33, a=19, b=19, c=9, d=18, gamma=16, omega=0x9E3779B9)
W64 = Params(w=64, r=64, s=33, a=24, b=22, c=37, d=45, gamma=32, omega=0x9E3779B97F4A7C15)

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        build(force=False)  # builds when missing or older than its sources
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER
        u32p, u64p, u8p = P(ctypes.c_uint32), P(ctypes.c_uint64), P(ctypes.c_uint8)
        L.xgo_params_valid.argtypes = [P(_Params)]
        L.xgo_splitmix64.argtypes = [u64p]
        L.xgo_splitmix64.restype = ctypes.c_uint64
        L.xgo_box_muller.argtypes = [ctypes.c_uint32, ctypes.c_uint32, P(ctypes.c_double), P(ctypes.c_double)]
        L.xgo_box_muller_many.argtypes = [u32p, ctypes.c_uint64, P(ctypes.c_double)]
        L.xgo_box_muller_many.restype = None
        L.xgo_seed_streams.argtypes = [P(_Params), ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                       u32p, u32p, u64p]
        L.xgo_run_streams.argtypes = [P(_Params), u32p, u32p, u64p, ctypes.c_uint64, ctypes.c_int,
                                      ctypes.c_uint64, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int]
        L.xgo_xpart_run.argtypes = [P(_Params), u32p, ctypes.c_uint64, ctypes.c_uint32, u8p]
        L.xgo_xpart_period.argtypes = [P(_Params), u32p, ctypes.c_uint64]
        L.xgo_xpart_period.restype = ctypes.c_uint64
        L.xgo_full_period.argtypes = [P(_Params), u32p, ctypes.c_uint32, ctypes.c_uint64]
        L.xgo_full_period.restype = ctypes.c_uint64
        L.xgo_xpart_matrix.argtypes = [P(_Params), u64p]
        L.xgo_xpart_jump_poly.argtypes = [P(_Params), u32p, u64p]
        P64 = P(_Params64)
        L.xgo64_params_valid.argtypes = [P64]
        L.xgo64_seed_streams.argtypes = [P64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, u64p, u64p, u64p]
        L.xgo64_run_streams.argtypes = [P64, u64p, u64p, u64p, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int]
        L.xgo64_xpart_run.argtypes = [P64, u64p, ctypes.c_uint64, ctypes.c_uint32, u8p]
        L.xgo64_xpart_jump_poly.argtypes = [P64, u64p, u64p]
        L.xgo64_box_muller.argtypes = [ctypes.c_uint64, ctypes.c_uint64, P(ctypes.c_double), P(ctypes.c_double)]
        L.xgo64_box_muller.restype = None
        L.gf2_clmul64.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u64p, u64p]
        L.gf2_clmul64_portable.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u64p, u64p]
        L.gf2_degree.argtypes = [u64p, ctypes.c_int]
        L.gf2_mulmod.argtypes = [u64p, ctypes.c_int, u64p, u64p, u64p]
        L.gf2_gcd_degree.argtypes = [u64p, u64p, ctypes.c_int]
        L.gf2_berlekamp_massey.argtypes = [u8p, ctypes.c_int, u64p, ctypes.c_int]
        L.gf2_is_primitive.argtypes = [u64p, ctypes.c_int, P(ctypes.c_int), ctypes.c_int, u64p,
                                       ctypes.c_int, ctypes.c_int]
        L.gf2_z_pow_mod.argtypes = [u64p, ctypes.c_int, u8p, ctypes.c_int, u64p]
        L.gf2_mat_pow_apply.argtypes = [u64p, ctypes.c_int, u8p, ctypes.c_int, u64p]
        L.gf2_mat_pow_apply_many.argtypes = [u64p, ctypes.c_int, u8p, ctypes.c_int, ctypes.c_int, u64p]
        L.xgo64_xpart_matrix.argtypes = [P64, u64p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ctype):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def default_threads() -> int:
    """Host cores this process may run on (the oracle's streams are independent,
    so each thread takes a share of them)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except (AttributeError, OSError):
        return max(1, os.cpu_count() or 1)


# ---------------------------------------------------------------------------
# streams
# ---------------------------------------------------------------------------

class OracleStreams:
    """`count` xorgens streams; stream i is seeded with seed + first + i."""

    def __init__(self, seed: int, count: int, first: int = 0, params: Params = PAPER):
        self.params = params
        self.count = count
        self.ring = np.zeros((count, params.r), dtype=np.uint32)
        self.weyl = np.zeros(count, dtype=np.uint32)
        self.pos = np.zeros(count, dtype=np.uint64)
        cp = params.c_struct()
        rc = lib().xgo_seed_streams(ctypes.byref(cp), seed & (2**64 - 1), first, count,
                                    _ptr(self.ring, ctypes.c_uint32), _ptr(self.weyl, ctypes.c_uint32),
                                    _ptr(self.pos, ctypes.c_uint64))
        if rc != 0:
            raise ValueError("invalid xorgens parameters")

    @classmethod
    def from_state(cls, ring, weyl, pos, params: Params = PAPER) -> "OracleStreams":
        self = cls.__new__(cls)
        self.params = params
        self.ring = np.ascontiguousarray(ring, dtype=np.uint32).reshape(-1, params.r).copy()
        self.count = self.ring.shape[0]
        self.weyl = np.ascontiguousarray(weyl, dtype=np.uint32).reshape(-1).copy()
        self.pos = np.ascontiguousarray(pos, dtype=np.uint64).reshape(-1).copy()
        return self

    def copy(self) -> "OracleStreams":
        return OracleStreams.from_state(self.ring, self.weyl, self.pos, self.params)

    def subset(self, idx) -> "OracleStreams":
        return OracleStreams.from_state(self.ring[idx], self.weyl[idx], self.pos[idx], self.params)

    def _run(self, kind: int, n: int, out: np.ndarray | None, threads: int | None):
        cp = self.params.c_struct()
        stride = out.strides[0] if out is not None and out.ndim == 2 else 0
        rc = lib().xgo_run_streams(
            ctypes.byref(cp), _ptr(self.ring, ctypes.c_uint32), _ptr(self.weyl, ctypes.c_uint32),
            _ptr(self.pos, ctypes.c_uint64), self.count, kind, n,
            None if out is None else out.ctypes.data_as(ctypes.c_void_p), stride,
            threads or default_threads())
        if rc != 0:
            raise RuntimeError("oracle run failed (%d)" % rc)

    def u32(self, n: int, threads: int | None = None) -> np.ndarray:
        out = np.empty((self.count, n), dtype=np.uint32)
        self._run(U32, n, out, threads)
        return out

    def f32(self, n: int, threads: int | None = None) -> np.ndarray:
        out = np.empty((self.count, n), dtype=np.float32)
        self._run(F32, n, out, threads)
        return out

    def normal(self, n: int, threads: int | None = None) -> np.ndarray:
        """FP64 Box-Muller normals; consumes 2 * ceil(n / 2) words per stream."""
        out = np.empty((self.count, n), dtype=np.float64)
        self._run(NORMAL, n, out, threads)
        return out

    def moments(self, n: int, threads: int | None = None) -> np.ndarray:
        """[count, 3] FP64 sums of z, z^2 and |z| over n normals (the last one
        scales the error bound of an FP32 sum of z)."""
        out = np.empty((self.count, 3), dtype=np.float64)
        self._run(MOMENTS, n, out, threads)
        return out

    def skip(self, n: int, threads: int | None = None) -> None:
        """Advances every stream by n words, producing nothing."""
        self._run(SKIP, n, None, threads)


class OracleStreams64:
    """`count` streams of a 64-bit-word member (xorgens64_oracle.c); stream i
    is seeded with seed + first + i.  ring[count, r] uint64, weyl, pos."""

    def __init__(self, seed: int, count: int, params: "Params", first: int = 0):
        if params.w != 64:
            raise ValueError("OracleStreams64 needs w = 64")
        self.params, self.count = params, count
        self.ring = np.zeros((count, params.r), dtype=np.uint64)
        self.weyl = np.zeros(count, dtype=np.uint64)
        self.pos = np.zeros(count, dtype=np.uint64)
        rc = lib().xgo64_seed_streams(ctypes.byref(params.c_struct()), seed & (2**64 - 1), first, count,
                                      _ptr(self.ring, ctypes.c_uint64), _ptr(self.weyl, ctypes.c_uint64),
                                      _ptr(self.pos, ctypes.c_uint64))
        if rc != 0:
            raise ValueError("invalid xorgens parameters")

    @classmethod
    def from_state(cls, ring, weyl, pos, params: "Params") -> "OracleStreams64":
        self = cls.__new__(cls)
        self.params = params
        self.ring = np.ascontiguousarray(ring, dtype=np.uint64).reshape(-1, params.r).copy()
        self.count = self.ring.shape[0]
        self.weyl = np.ascontiguousarray(weyl, dtype=np.uint64).reshape(-1).copy()
        self.pos = np.ascontiguousarray(pos, dtype=np.uint64).reshape(-1).copy()
        return self

    def copy(self) -> "OracleStreams64":
        return OracleStreams64.from_state(self.ring, self.weyl, self.pos, self.params)

    def _run(self, kind: int, n: int, out, threads):
        stride = out.strides[0] if out is not None else 0
        rc = lib().xgo64_run_streams(
            ctypes.byref(self.params.c_struct()), _ptr(self.ring, ctypes.c_uint64),
            _ptr(self.weyl, ctypes.c_uint64), _ptr(self.pos, ctypes.c_uint64), self.count, kind, n,
            None if out is None else out.ctypes.data_as(ctypes.c_void_p), stride, threads or default_threads())
        if rc != 0:
            raise RuntimeError("oracle run failed (%d)" % rc)

    def u64(self, n: int, threads: int | None = None) -> np.ndarray:
        out = np.empty((self.count, n), dtype=np.uint64)
        self._run(0, n, out, threads)
        return out

    def f64(self, n: int, threads: int | None = None) -> np.ndarray:
        """(out >> 11) 2^-53 per word."""
        out = np.empty((self.count, n), dtype=np.float64)
        self._run(1, n, out, threads)
        return out

    def normal(self, n: int, threads: int | None = None) -> np.ndarray:
        """n FP64 Box-Muller normals per stream (long double, rounded once);
        consumes 2 ceil(n / 2) words."""
        out = np.empty((self.count, n), dtype=np.float64)
        self._run(2, n, out, threads)
        return out

    def moments(self, n: int, threads: int | None = None) -> np.ndarray:
        """[count, 3]: sums of z, z^2 and |z| over the n normals normal(n)
        would give, accumulated in long double; the same words consumed."""
        out = np.empty((self.count, 3), dtype=np.float64)
        self._run(3, n, out, threads)
        return out

    def skip(self, n: int, threads: int | None = None) -> None:
        self._run(SKIP, n, None, threads)


def splitmix64_sequence(seed: int, k: int) -> list[int]:
    z = ctypes.c_uint64(seed & (2**64 - 1))
    return [int(lib().xgo_splitmix64(ctypes.byref(z))) for _ in range(k)]


def box_muller_w64(o_even: int, o_odd: int) -> tuple[float, float]:
    """The 64-bit member's pair map: 53-bit uniforms, long double, rounded once."""
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    lib().xgo64_box_muller(o_even & (2**64 - 1), o_odd & (2**64 - 1), ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


def box_muller_many(words: np.ndarray, threads: int | None = None) -> np.ndarray:
    """The FP64 Box-Muller map of the oracle (xgo_box_muller) on consecutive
    word pairs: returns an array of shape (pairs, 2).  Slices run in threads
    (the C call releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    words = np.ascontiguousarray(words, dtype=np.uint32)
    pairs = words.size // 2
    out = np.empty((pairs, 2), dtype=np.float64)
    nt = max(1, threads or default_threads())
    step = -(-pairs // nt) if pairs else 1
    fn = lib().xgo_box_muller_many

    def run(a):
        b = min(pairs, a + step)
        if b > a:
            fn(_ptr(words[2 * a:2 * b], ctypes.c_uint32), b - a, _ptr(out[a:b], ctypes.c_double))

    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(run, range(0, pairs, step)))
    return out


def box_muller64(o_even: int, o_odd: int) -> tuple[float, float]:
    z0, z1 = ctypes.c_double(), ctypes.c_double()
    lib().xgo_box_muller(o_even, o_odd, ctypes.byref(z0), ctypes.byref(z1))
    return z0.value, z1.value


# ---------------------------------------------------------------------------
# x-part (GF(2)-linear) helpers
# ---------------------------------------------------------------------------

def xpart_run(params: Params, ring: np.ndarray, steps: int, bit: int = 0, want_bits: bool = False):
    """Steps one linear ring `steps` times (in place); optionally returns bit
    `bit` of every x_k produced."""
    if params.w == 64:
        ring = np.ascontiguousarray(ring, dtype=np.uint64)
        bits = np.zeros(steps, dtype=np.uint8) if want_bits else None
        rc = lib().xgo64_xpart_run(ctypes.byref(params.c_struct()), _ptr(ring, ctypes.c_uint64), steps, bit,
                                   None if bits is None else _ptr(bits, ctypes.c_uint8))
        if rc != 0:
            raise ValueError("bad xpart_run arguments")
        return ring, bits
    ring = np.ascontiguousarray(ring, dtype=np.uint32)
    cp = params.c_struct()
    bits = np.zeros(steps, dtype=np.uint8) if want_bits else None
    rc = lib().xgo_xpart_run(ctypes.byref(cp), _ptr(ring, ctypes.c_uint32), steps, bit,
                             None if bits is None else _ptr(bits, ctypes.c_uint8))
    if rc != 0:
        raise ValueError("bad xpart_run arguments")
    return ring, bits


def xpart_period(params: Params, ring, max_steps: int) -> int:
    ring = np.ascontiguousarray(ring, dtype=np.uint32)
    return int(lib().xgo_xpart_period(ctypes.byref(params.c_struct()), _ptr(ring, ctypes.c_uint32), max_steps))


def full_period(params: Params, ring, weyl: int, max_steps: int) -> int:
    ring = np.ascontiguousarray(ring, dtype=np.uint32)
    return int(lib().xgo_full_period(ctypes.byref(params.c_struct()), _ptr(ring, ctypes.c_uint32),
                                     weyl, max_steps))


def xpart_matrix(params: Params) -> np.ndarray:
    """The x-part's one-step matrix (n rows of bits; next = M state)."""
    n = params.n
    rw = (n - 1) // 64 + 1
    rows = np.zeros((n, rw), dtype=np.uint64)
    if params.w == 64:
        rc = lib().xgo64_xpart_matrix(ctypes.byref(params.c_struct()), _ptr(rows, ctypes.c_uint64))
    else:
        rc = lib().xgo_xpart_matrix(ctypes.byref(params.c_struct()), _ptr(rows, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("bad params")
    return rows


def ring_to_bits(params: Params, ring) -> np.ndarray:
    """Packs a linear ring into the column bit vector used by xpart_matrix
    (state bit w t + b is bit b of ring word t)."""
    n = params.n
    v = np.zeros((n - 1) // 64 + 1, dtype=np.uint64)
    for t, word in enumerate(np.asarray(ring, dtype=np.uint64 if params.w == 64 else np.uint32)):
        for b in range(params.w):
            if (int(word) >> b) & 1:
                i = t * params.w + b
                v[i // 64] |= np.uint64(1 << (i % 64))
    return v


def bits_to_ring(params: Params, v: np.ndarray) -> np.ndarray:
    wt = np.uint64 if params.w == 64 else np.uint32
    ring = np.zeros(params.r, dtype=wt)
    for i in range(params.n):
        if (int(v[i // 64]) >> (i % 64)) & 1:
            ring[i // params.w] |= wt(1 << (i % params.w))
    return ring


def mat_pow_apply(M: np.ndarray, n: int, J: int, v: np.ndarray) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.uint64).copy()
    jb = _int_bits(J)
    rc = lib().gf2_mat_pow_apply(_ptr(np.ascontiguousarray(M), ctypes.c_uint64), n,
                                 _ptr(jb, ctypes.c_uint8), len(jb), _ptr(v, ctypes.c_uint64))
    if rc != 0:
        raise RuntimeError("mat_pow_apply failed")
    return v


def mat_pow_apply_many(M: np.ndarray, n: int, Js, vs: np.ndarray) -> np.ndarray:
    """Row j of the result is M^(Js[j]) vs[j] (the binary powers of M formed
    once for all j)."""
    Js = [int(J) for J in Js]
    nb = max(1, max(J.bit_length() for J in Js))
    jb = np.array([[(J >> i) & 1 for i in range(nb)] for J in Js], dtype=np.uint8)
    vs = np.ascontiguousarray(vs, dtype=np.uint64).copy()
    rc = lib().gf2_mat_pow_apply_many(_ptr(np.ascontiguousarray(M), ctypes.c_uint64), n,
                                      _ptr(jb, ctypes.c_uint8), nb, len(Js), _ptr(vs, ctypes.c_uint64))
    if rc != 0:
        raise RuntimeError("mat_pow_apply_many failed")
    return vs


def xpart_jump_poly(params: Params, ring, g: np.ndarray) -> np.ndarray:
    g = np.ascontiguousarray(g, dtype=np.uint64)
    if params.w == 64:
        ring = np.ascontiguousarray(ring, dtype=np.uint64).copy()
        if lib().xgo64_xpart_jump_poly(ctypes.byref(params.c_struct()), _ptr(ring, ctypes.c_uint64),
                                       _ptr(g, ctypes.c_uint64)) != 0:
            raise ValueError("bad params")
        return ring
    ring = np.ascontiguousarray(ring, dtype=np.uint32).copy()
    rc = lib().xgo_xpart_jump_poly(ctypes.byref(params.c_struct()), _ptr(ring, ctypes.c_uint32),
                                   _ptr(g, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("bad params")
    return ring


# ---------------------------------------------------------------------------
# GF(2) polynomials (Python ints as coefficient bit strings: bit i <-> z^i)
# ---------------------------------------------------------------------------

def _int_bits(J: int) -> np.ndarray:
    nb = max(1, J.bit_length())
    return np.array([(J >> i) & 1 for i in range(nb)], dtype=np.uint8)


def poly_to_words(P: int, words: int) -> np.ndarray:
    return np.array([(P >> (64 * i)) & (2**64 - 1) for i in range(words)], dtype=np.uint64)


def words_to_poly(a: np.ndarray) -> int:
    v = 0
    for i, w in enumerate(np.asarray(a, dtype=np.uint64)):
        v |= int(w) << (64 * i)
    return v


def berlekamp_massey(bits: np.ndarray) -> int:
    """Characteristic polynomial (as an int) of the shortest LFSR for `bits`."""
    bits = np.ascontiguousarray(bits, dtype=np.uint8)
    words = len(bits) // 64 + 2
    poly = np.zeros(words, dtype=np.uint64)
    lib().gf2_berlekamp_massey(_ptr(bits, ctypes.c_uint8), len(bits), _ptr(poly, ctypes.c_uint64), words)
    return words_to_poly(poly)


def clmul64(a: int, b: int, portable: bool = False) -> int:
    lo, hi = ctypes.c_uint64(), ctypes.c_uint64()
    f = lib().gf2_clmul64_portable if portable else lib().gf2_clmul64
    f(a, b, ctypes.byref(lo), ctypes.byref(hi))
    return lo.value | (hi.value << 64)


def mulmod(a: int, b: int, P: int) -> int:
    n = P.bit_length() - 1
    w = (n - 1) // 64 + 1
    pw = n // 64 + 1
    out = np.zeros(w, dtype=np.uint64)
    rc = lib().gf2_mulmod(_ptr(poly_to_words(P, pw), ctypes.c_uint64), n,
                          _ptr(poly_to_words(a, w), ctypes.c_uint64),
                          _ptr(poly_to_words(b, w), ctypes.c_uint64), _ptr(out, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("bad modulus")
    return words_to_poly(out)


def gcd_degree(a: int, b: int) -> int:
    words = max(a.bit_length(), b.bit_length()) // 64 + 1
    return int(lib().gf2_gcd_degree(_ptr(poly_to_words(a, words), ctypes.c_uint64),
                                    _ptr(poly_to_words(b, words), ctypes.c_uint64), words))


def z_pow_mod(J: int, P: int) -> int:
    n = P.bit_length() - 1
    w = (n - 1) // 64 + 1
    g = np.zeros(w, dtype=np.uint64)
    jb = _int_bits(J)
    rc = lib().gf2_z_pow_mod(_ptr(poly_to_words(P, n // 64 + 1), ctypes.c_uint64), n,
                             _ptr(jb, ctypes.c_uint8), len(jb), _ptr(g, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("bad modulus")
    return words_to_poly(g)


def distinct_prime_factors_small(m: int) -> list[int]:
    """Trial division (for the small moduli 2^n - 1, n <= 64, of the tiny sets)."""
    out, p = [], 2
    while p * p <= m:
        if m % p == 0:
            out.append(p)
            while m % p == 0:
                m //= p
        p += 1 if p == 2 else 2
    if m > 1:
        out.append(m)
    return out


def is_primitive(P: int, mersenne_primes: list[int] | None = None) -> int:
    """0 if P (degree n) is primitive over GF(2), else the failing check code
    (see gf2_is_primitive).  `mersenne_primes` are the distinct primes dividing
    2^n - 1; found by trial division when n is small."""
    n = P.bit_length() - 1
    if mersenne_primes is None:
        mersenne_primes = distinct_prime_factors_small(2**n - 1)
    N = 2**n - 1
    for q in mersenne_primes:
        if N % q:
            raise ValueError("%d does not divide 2^%d - 1" % (q, n))
    sub = [n // p for p in distinct_prime_factors_small(n)]
    ew = (n - 1) // 64 + 1
    exps = np.concatenate([poly_to_words(N // q, ew) for q in mersenne_primes]) if mersenne_primes \
        else np.zeros(ew, dtype=np.uint64)
    sub_a = (ctypes.c_int * max(1, len(sub)))(*sub)
    return int(lib().gf2_is_primitive(_ptr(poly_to_words(P, n // 64 + 1), ctypes.c_uint64), n, sub_a, len(sub),
                                      _ptr(np.ascontiguousarray(exps), ctypes.c_uint64), len(mersenne_primes), ew))


def charpoly(params: Params, ring=None, bit: int = 0, extra: int = 64) -> int:
    """Minimal polynomial of bit `bit` of the x-part sequence, from 2n + extra
    terms by Berlekamp-Massey.  For a nonzero start ring and a primitive
    characteristic polynomial it equals that polynomial."""
    wt = np.uint64 if params.w == 64 else np.uint32
    if ring is None:
        ring = np.arange(1, params.r + 1, dtype=np.uint64) & np.uint64((1 << min(params.w, 64)) - 1)
    _, bits = xpart_run(params, np.array(ring, dtype=wt), 2 * params.n + extra, bit, want_bits=True)
    return berlekamp_massey(bits)


def weyl_omega(w: int) -> int:
    """Odd integer nearest 2^{w-1} (sqrt 5 - 1) (Section 1.5), computed with
    exact integer square roots."""
    # 2^{w-1} sqrt 5 = sqrt(5 * 4^{w-1}); take it to 8 extra bits to round.
    scaled = math.isqrt(5 * 4 ** (w - 1) * 4 ** 8)   # floor(2^8 * 2^{w-1} sqrt 5)
    val_x256 = scaled - (2 ** (w - 1)) * 2 ** 8      # 2^8 * 2^{w-1}(sqrt 5 - 1), floored
    nearest = (val_x256 + 128) >> 8
    if nearest % 2 == 1:
        return nearest
    # nearest odd neighbour
    lo, hi = nearest - 1, nearest + 1
    return lo if (val_x256 - lo * 256) <= (hi * 256 - val_x256) else hi
