"""Exhaustive accuracy of the FP32 Box-Muller map against FP64.

u1 and u2 each take 2^24 values.  With u2 = 0 (cos = 1, sin = 0) the first
output is rho(u1) = sqrt(-2 ln u1) itself, so every u1 is checked; with
fixed u1 every u2 is checked for both outputs.  Every value must be within
4 FP32 ulp of the FP64 oracle's value for that very pair (its C map applied
to all 2^24 pairs of each sweep; its maximum is reported); z_1 must be
exactly zero where the FP64 value is."""
import numpy as np
import pytest

from gpu_helpers import needs_gpu, ulp32_error
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402

M = 1 << 24


def _gpu_box_muller(e: np.ndarray, o: np.ndarray) -> np.ndarray:
    words = np.empty(2 * e.size, dtype=np.uint32)
    words[0::2], words[1::2] = e, o
    d = torch.from_numpy(words.view(np.int32)).cuda()
    out = torch.empty(2 * e.size, dtype=torch.float32, device="cuda")
    xg.xg_box_muller(d.data_ptr(), e.size, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    return out.cpu().numpy().reshape(-1, 2)


def _fp64_numpy(e: np.ndarray, o: np.ndarray) -> np.ndarray:
    """A second FP64 form of the same map, in numpy (same pairing, exact
    quarter-turn reduction of the dyadic angle), used only as a cross-check
    of the oracle."""
    u1 = ((e >> 8).astype(np.float64) + 1.0) * 2.0**-24
    u2 = (o >> 8).astype(np.float64) * 2.0**-24
    rho = np.sqrt(-2.0 * np.log(u1))
    y = 4.0 * u2                       # 2 v with v = 2 u2; reduce v = q / 2 + f exactly
    q = np.rint(y)
    f = 0.5 * (y - q)
    sf, cf = np.sin(np.pi * f), np.cos(np.pi * f)
    qi = (q.astype(np.int64) % 4)
    s = np.choose(qi, [sf, cf, -sf, -cf])
    c = np.choose(qi, [cf, -sf, -cf, sf])
    s[f == 0] = np.choose(qi[f == 0], [0.0, 1.0, 0.0, -1.0])
    c[f == 0] = np.choose(qi[f == 0], [1.0, 0.0, -1.0, 0.0])
    return np.stack([rho * c, rho * s], axis=1)


def _fp64(e: np.ndarray, o: np.ndarray) -> np.ndarray:
    """The oracle's FP64 Box-Muller (its C function, xgo_box_muller) on every
    pair; the numpy form must agree with it to within FP64 rounding."""
    words = np.empty(2 * e.size, dtype=np.uint32)
    words[0::2], words[1::2] = e, o
    z = O.box_muller_many(words)
    zn = _fp64_numpy(e, o)
    assert (np.abs(zn - z) <= 1e-15 * np.maximum(1.0, np.abs(z))).all()
    return z


def test_every_u1():
    e = (np.arange(M, dtype=np.uint32) << np.uint32(8))
    o = np.zeros(M, dtype=np.uint32)
    z = _gpu_box_muller(e, o)
    zr = _fp64(e, o)
    err = ulp32_error(z[:, 0], zr[:, 0])
    print("rho: max %.3f ulp" % err.max())
    assert err.max() <= 4.0
    assert (z[:, 1] == 0).all()


@pytest.mark.parametrize("k1", [0, 1, 1 << 12, (1 << 23) + 5, M - 2])
def test_every_u2(k1):
    o = (np.arange(M, dtype=np.uint32) << np.uint32(8)) | np.uint32(0x5A)
    e = np.full(M, (k1 << 8) | 0xC3, dtype=np.uint32)
    z = _gpu_box_muller(e, o)
    zr = _fp64(e, o)
    err0, err1 = ulp32_error(z[:, 0], zr[:, 0]), ulp32_error(z[:, 1], zr[:, 1])
    print("u1 index %d: max %.3f / %.3f ulp" % (k1, err0.max(), err1.max()))
    assert err0.max() <= 4.0 and err1.max() <= 4.0
