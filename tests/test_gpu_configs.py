"""The workloads at their full sizes, in the launch configurations bench.py
and the batched path use, against the CPU oracle.

- one stream, seed 42, 2^20 uint32: every word, and the stored digest;
- 1024 streams (seed 42 + i) x 2^20, uint32 then FP32, bulk-fill layout (the
  benchmark's launches) and stream-major layout: every word of every stream;
- 65536 streams with log-uniform lengths in [2^10, 2^20] (seed 7), the
  one-call batch captured in a HIP graph with the autotuner's shape: every
  word of every stream, every stream's final position;
- 4096 streams x 2^18 normals reduced in-kernel to sums of z and z^2: every
  stream within the stated bound; and all 2^30 variates within 4 ulp through
  the unfused path.
"""
import hashlib
import os

import numpy as np
import pytest

from gpu_helpers import check_ragged_every_word, needs_gpu, ulp32_error
from oracle import oracle as O

pytestmark = [pytest.mark.gpu, needs_gpu]

torch = pytest.importorskip("torch")

from paper_1108_0486_amd import workloads as W  # noqa: E402
from paper_1108_0486_amd.batch import Batch  # noqa: E402
from paper_1108_0486_amd.streams import XorgensStreams, as_u32  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fill_view(flat: np.ndarray, count: int, n: int, k0: int, k1: int) -> np.ndarray:
    """[k1 - k0, n] per-stream view of a bulk-fill output (n a multiple of 64)."""
    assert n % 64 == 0
    return flat.reshape(n // 64, count, 64)[:, k0:k1, :].transpose(1, 0, 2).reshape(k1 - k0, n)


def test_single_stream_seed42():
    gs = XorgensStreams(1, seed=W.SEED)
    out = as_u32(gs.u32(W.SINGLE_N))[0]
    ref = O.OracleStreams(W.SEED, 1)
    assert (out == ref.u32(W.SINGLE_N)[0]).all()
    lines = dict(l.split(" ", 1) for l in open(os.path.join(GOLDEN, "single_stream_seed42_2p20.txt"))
                 if not l.startswith("#"))
    assert hashlib.sha256(out.tobytes()).hexdigest() == lines["sha256_le_u32"].strip()
    ring, weyl, pos = gs.host_state()
    assert int(weyl[0]) == int(lines["final_weyl"], 16) and int(pos[0]) == W.SINGLE_N


def test_bulk_fill_layout_every_stream():
    """The benchmark's two launches (xg_fill_u32, then xg_fill_f32, default
    launch shape) against the oracle, every word."""
    S, N = W.BULK_STREAMS, W.BULK_N
    gs = XorgensStreams(S, seed=W.SEED)
    u = as_u32(gs.fill_u32(N))
    f = gs.fill_f32(N).cpu().numpy()
    torch.cuda.synchronize()
    step = 128
    for k0 in range(0, S, step):
        ref = O.OracleStreams(W.SEED, step, first=k0)
        assert (_fill_view(u, S, N, k0, k0 + step) == ref.u32(N)).all(), k0
        assert (_fill_view(f, S, N, k0, k0 + step) == ref.f32(N)).all(), k0
        ring, weyl, pos = gs.host_state(list(range(k0, k0 + step)))
        assert (ring == ref.ring).all() and (weyl == ref.weyl).all() and (pos == ref.pos).all()


def test_bulk_stream_major_every_stream():
    S, N = W.BULK_STREAMS, W.BULK_N
    gs = XorgensStreams(S, seed=W.SEED)
    u = as_u32(gs.u32(N))
    digests = dict(l.split()[1:] for l in open(os.path.join(GOLDEN, "bulk_1024x2p20_samples.txt"))
                   if l.startswith("stream"))
    for i, d in digests.items():
        assert hashlib.sha256(u[int(i)].tobytes()).hexdigest() == d, i
    f = gs.f32(N).cpu().numpy()
    step = 128
    for k0 in range(0, S, step):
        ref = O.OracleStreams(W.SEED, step, first=k0)
        assert (u[k0:k0 + step] == ref.u32(N)).all(), k0
        assert (f[k0:k0 + step] == ref.f32(N)).all(), k0


def test_ragged_batch_full_size_graph():
    """The ragged workload (65 536 streams, 9.95 x 10^9 uint32 words) through
    the one-call batch with the autotuned shape, captured in a HIP graph, as
    the bench times it: every word of every stream against the oracle, every
    end position, and the end states of 512 streams against the oracle's own
    polynomial jump."""
    lengths = W.ragged_lengths()
    off = W.csr_offsets(lengths)
    total = int(off[-1])
    S = len(lengths)
    reqs = [(i, int(lengths[i]), int(off[i]), 0) for i in range(S)]
    gs = XorgensStreams(S, seed=W.SEED)
    b = Batch(gs, reqs, total)
    key = "test/ragged65536/u32"
    best, recs = b.autotune(reps=1, tune_key=key)
    g = b.capture_graph(tune_key=key)
    g.replay()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    _, _, pos = gs.host_state()
    assert (pos == lengths).all()
    check_ragged_every_word(b.out, lengths, off, W.SEED)
    # End states of 512 streams: each depends on every word the stream
    # generated.  The oracle reaches them by its own polynomial jump
    # (z^n mod P on the x-part, n omega on the Weyl word).
    rng = np.random.default_rng(0)
    P = O.charpoly(O.PAPER)
    more = sorted(rng.choice(S, size=512, replace=False).tolist())
    ring, weyl, _ = gs.host_state(more)
    for j, i in enumerate(more):
        n = int(lengths[i])
        start = O.OracleStreams(W.SEED + i, 1)
        gp = O.poly_to_words(O.z_pow_mod(n, P), 64)
        assert (ring[j] == O.xpart_jump_poly(O.PAPER, start.ring[0], gp)).all(), i
        assert int(weyl[j]) == (int(start.weyl[0]) + n * O.PAPER.omega) % 2**32, i
    del recs


def test_fused_moments_full_size():
    S, N = W.FUSED_STREAMS, W.FUSED_N
    gs = XorgensStreams(S, seed=W.SEED)
    saved = gs.checkpoint()
    m = gs.moments(N).cpu().numpy().astype(np.float64)
    ref = O.OracleStreams(W.SEED, S)
    mref = ref.moments(N)
    tau = 27 * 2.0**-24
    err1 = np.abs(m[:, 0] - mref[:, 0]) / mref[:, 2]
    err2 = np.abs(m[:, 1] - mref[:, 1]) / mref[:, 1]
    assert err1.max() <= tau, err1.max()
    assert err2.max() <= tau, err2.max()
    ring, weyl, pos = gs.host_state()
    assert (pos == ref.pos).all() and (ring == ref.ring).all()
    # the same variates through the unfused path, for a sample of streams
    gs.restore(saved)
    first, count = 1000, 64
    z = gs.normal(N, first=first, count=count).cpu().numpy()
    zr = O.OracleStreams(W.SEED, count, first=first).normal(N)
    assert ulp32_error(z, zr).max() <= 4.0
    print("moments: max rel err sum z %.3g, sum z^2 %.3g (bound %.3g)" % (err1.max(), err2.max(), tau))


def test_fused_config_every_variate_unfused():
    """Every one of the 2^30 variates of the fused workload (4096 streams x
    2^18), produced through the unfused path, is within 4 FP32 ulp of the
    FP64 oracle.  The fused kernel computes each pair's two values with the
    same device functions (rho, the reduced angle and its polynomials); for a
    whole pair it only skips the swap of odd quadrants, so it sums the same
    two floats, in an order immaterial to the sums.
    Checked 256 streams at a time to bound host memory."""
    S, N = W.FUSED_STREAMS, W.FUSED_N
    gs = XorgensStreams(S, seed=W.SEED)
    step, worst = 256, 0.0
    for first in range(0, S, step):
        z = gs.normal(N, first=first, count=step).cpu().numpy()
        zr = O.OracleStreams(W.SEED, step, first=first).normal(N)
        worst = max(worst, float(ulp32_error(z, zr).max()))
        assert worst <= 4.0, (first, worst)
        del z, zr
    print("normals: max error over all 2^30 variates %.3f ulp" % worst)
