"""Guard bands and determinism for every generating call.

Each call writes into the middle of a buffer whose leading and trailing
guard words hold a sentinel; after the call the guards must be intact (no
write outside [out, out + elements)), and running the same call twice from
the same state must give identical bytes.  Lengths are ragged and stream
ranges offset, so tails, odd stream counts and partial wavefronts are
exercised.
"""
import hashlib

import numpy as np
import pytest

from gpu_helpers import needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import xg  # noqa: E402
from paper_1108_0486_amd.batch import Batch  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams  # noqa: E402

GUARD = 4096                     # 32-bit words on each side (16 KB)
SENTINEL = np.int32(0x5A5A5A5A)


def _guarded(words: int):
    buf = torch.full((GUARD + words + GUARD,), int(SENTINEL), dtype=torch.int32, device="cuda")
    return buf, buf[GUARD:GUARD + words]


def _check_guards(buf, words):
    a = buf.cpu().numpy()
    assert (a[:GUARD] == SENTINEL).all(), "write before the output"
    assert (a[GUARD + words:] == SENTINEL).all(), "write after the output"
    return hashlib.sha256(a[GUARD:GUARD + words].tobytes()).hexdigest()


# (family, call, elements per stream-value, per-stream elements(n), extra)
CASES = []
for n in (1, 31, 33, 63, 65, 129, 1001):
    CASES += [(xg.XG_FAMILY_R128_W32, name, n) for name in ("u32", "f32", "normal", "moments", "fill_u32", "fill_f32")]
    CASES += [(xg.XG_FAMILY_R64_W32, name, n) for name in ("u32", "f32", "normal", "moments", "fill_u32", "fill_f32")]
    CASES += [(xg.XG_FAMILY_R64_W64, name, n) for name in ("u64", "f64", "fill_u64", "fill_f64", "normal_f64",
                                                           "moments_f64")]


def _words_of(name, n, count):
    per = 2 if name.startswith("moments") else n
    wide = name in ("u64", "f64", "fill_u64", "fill_f64", "normal_f64", "moments_f64")
    return count * per * (2 if wide else 1)


def _run(family, name, n, first, count, out_words):
    gs = XorgensStreams(first + count + 2, seed=31, family=family)
    saved = gs.checkpoint()
    hashes = []
    for _ in range(2):
        gs.restore(saved)
        buf, view = _guarded(out_words)
        if name in ("u64", "f64", "fill_u64", "fill_f64", "normal_f64", "moments_f64"):
            dt = torch.int64 if "u64" in name else torch.float64
            target = view.view(dt)
        elif name in ("f32", "normal", "moments", "fill_f32"):
            target = view.view(torch.float32)
        else:
            target = view
        if name.startswith("fill"):
            getattr(gs, name)(n, first=first, count=count, out=target)
        elif name.startswith("moments"):
            getattr(gs, name)(n, first=first, count=count, out=target.view(count, 2))
        else:
            getattr(gs, name)(n, first=first, count=count, out=target.view(count, -1))
        torch.cuda.synchronize()
        hashes.append(_check_guards(buf, out_words))
    assert hashes[0] == hashes[1], "two runs from one state differ"


@pytest.mark.parametrize("family,name,n", CASES)
def test_guard_bands_and_determinism(family, name, n):
    first, count = 3, 7
    _run(family, name, n, first, count, _words_of(name, n, count))


def test_batch_guard_bands_and_determinism():
    gs = XorgensStreams(9, seed=2)
    saved = gs.checkpoint()
    reqs = [(0, 1001, 0, 0), (3, 63, 1001, 2), (3, 65, 1064, 1), (8, 4133, 1129, 0), (5, 1, 5262, 2)]
    words = 5263
    hashes = []
    for _ in range(2):
        gs.restore(saved)
        buf, view = _guarded(words)
        b = Batch(gs, reqs, words, out=view)
        b.run()
        torch.cuda.synchronize()
        assert b.error_flag() == 0
        hashes.append(_check_guards(buf, words))
    assert hashes[0] == hashes[1]


@pytest.mark.gpu
def test_caller_output_checked_before_launch():
    # A caller's output tensor that the call would overrun, or that the
    # kernels cannot address linearly, is refused before anything is launched.
    gs = XorgensStreams(8, seed=5)
    dev = gs.device
    with pytest.raises(ValueError, match="holds"):
        gs.u32(64, first=0, count=4, out=torch.empty(4 * 64 - 1, dtype=torch.int32, device=dev))
    with pytest.raises(ValueError, match="contiguous"):
        gs.f32(64, first=0, count=4, out=torch.empty(64, 8, dtype=torch.float32, device=dev).t())
    with pytest.raises(ValueError, match="byte"):
        gs.normal(64, first=0, count=4, out=torch.empty(4, 64, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError, match="GPU"):
        gs.fill_u32(64, first=0, count=4, out=torch.empty(4 * 64, dtype=torch.int32))
    with pytest.raises(ValueError, match="out_elems"):
        Batch(gs, [(0, 100, 0, 0)], 100, out=torch.empty(99, dtype=torch.int32, device=dev))
    # Nothing ran: the states are those of a fresh generator.
    ref = XorgensStreams(8, seed=5)
    assert torch.equal(gs.u32(64), ref.u32(64))
