"""Shared helpers of the GPU parity tests: comparison metrics, and the
word-by-word check of a ragged batch output against the oracle."""
import numpy as np
import pytest

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    torch = None
    HAVE_GPU = False

needs_gpu = pytest.mark.skipif(not HAVE_GPU, reason="no GPU visible")


def ulp32_error(z32: np.ndarray, z64: np.ndarray) -> np.ndarray:
    """|z32 - z64| in units of the FP32 ulp of z64: ulp32(v) = 2^(max(e, -126) - 23)
    with e = floor(log2 |v|).  Where z64 == 0 exactly the error is 0 if z32 == 0
    and infinite otherwise."""
    z32 = np.asarray(z32, dtype=np.float32).astype(np.float64)
    z64 = np.asarray(z64, dtype=np.float64)
    a = np.abs(z64)
    _, e2 = np.frexp(np.where(a > 0, a, 1.0))      # a = m 2^e2, m in [0.5, 1)
    e = np.maximum(e2 - 1, -126)
    err = np.abs(z32 - z64) / np.exp2(e - 23.0)
    zero = a == 0
    err[zero] = np.where(z32[zero] == 0, 0.0, np.inf)
    return err


def ulp64_error(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """|got - ref| in units of the FP64 ulp of ref: 2^(max(e, -1022) - 52) with
    e = floor(log2 |ref|); where ref == 0 exactly the error is 0 if got == 0
    and infinite otherwise."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    a = np.abs(ref)
    _, e2 = np.frexp(np.where(a > 0, a, 1.0))
    e = np.maximum(e2 - 1, -1022)
    err = np.abs(got - ref) / np.exp2(e - 52.0)
    zero = a == 0
    err[zero] = np.where(got[zero] == 0, 0.0, np.inf)
    return err


def huge_skip_digests() -> dict:
    """Stored sha256 digests of rings after large skips, computed by the
    oracle's matrix form (tests/golden/huge_skips_matrix_form.txt), keyed by
    (member name, seed, stream, J)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "huge_skips_matrix_form.txt")
    out = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        out[(f[0], int(f[2]), int(f[4]), int(f[6]))] = f[8]
    return out


def ring_digest(ring: np.ndarray) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(ring).tobytes()).hexdigest()


def check_ragged_every_word(out, lengths, off, seed, params=None, window_words=1 << 28, chunk=16):
    """Every word of every stream of a ragged CSR output against the oracle:
    the output comes back in windows of consecutive streams (one copy each);
    inside a window the streams are taken in order of length, `chunk` at a
    time, and the oracle runs those streams in parallel up to the longest."""
    from oracle import oracle as O
    S = len(lengths)
    ref_all = O.OracleStreams(seed, S, params=params or O.PAPER)
    k0, checked = 0, 0
    while k0 < S:
        k1 = k0 + 1
        while k1 < S and int(off[k1 + 1] - off[k0]) <= window_words:
            k1 += 1
        host = out[int(off[k0]):int(off[k1])].cpu().numpy().view(np.uint32)
        order = k0 + np.argsort(lengths[k0:k1], kind="stable")
        for c in range(0, len(order), chunk):
            sel = order[c:c + chunk]
            want = ref_all.subset(sel).u32(int(lengths[sel].max()))
            for j, i in enumerate(sel):
                n, a = int(lengths[i]), int(off[i] - off[k0])
                assert np.array_equal(host[a:a + n], want[j, :n]), i
                checked += n
        k0 = k1
    assert checked == int(off[-1])
