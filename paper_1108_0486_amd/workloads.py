"""Seeded synthetic workloads (shapes and request traces only).

This module draws sizes, stream choices and arrival times with numpy's
default_rng; it holds none of the generator's arithmetic, so both the HIP
path's tests and the oracle side can use it.  There is no dataset: the
paper's own measurement is repeated bulk generation (Section 3).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED = 42                      # stream i is seeded from SEED + i
SINGLE_N = 1 << 20             # one stream, 2^20 outputs
BULK_STREAMS = 1024            # 1024 streams x 2^20 outputs, uint32 and FP32
BULK_N = 1 << 20
RAGGED_STREAMS = 65536         # lengths log-uniform in [2^10, 2^20]
RAGGED_LEN_SEED = 7
FUSED_STREAMS = 4096           # 4096 streams x 2^18 normals, reduced in-kernel
FUSED_N = 1 << 18
SERVE_STREAMS = 100_000        # device-resident streams of the request server
SERVE_RATE = 20_000.0          # Poisson arrivals per second
SERVE_SEED = 11


def ragged_lengths(num_streams: int = RAGGED_STREAMS, seed: int = RAGGED_LEN_SEED,
                   lo_exp: int = 10, hi_exp: int = 20) -> np.ndarray:
    """n_i = floor(2^(lo + (hi - lo) U_i)), U = default_rng(seed).random(num_streams),
    clipped to [2^lo, 2^hi]."""
    u = np.random.default_rng(seed).random(num_streams)
    n = np.floor(np.exp2(lo_exp + (hi_exp - lo_exp) * u)).astype(np.int64)
    return np.clip(n, 1 << lo_exp, 1 << hi_exp).astype(np.uint64)


def csr_offsets(lengths: np.ndarray) -> np.ndarray:
    off = np.zeros(len(lengths) + 1, dtype=np.uint64)
    np.cumsum(lengths, out=off[1:])
    return off


@dataclass
class Request:
    rid: int
    arrival_s: float
    stream: int
    n: int
    dtype: int  # 0 uint32, 1 FP32 uniform, 2 FP32 normal


def serving_trace(num_requests: int, num_streams: int = SERVE_STREAMS, rate: float = SERVE_RATE,
                  seed: int = SERVE_SEED, lo_exp: int = 8, hi_exp: int = 24) -> list[Request]:
    """Poisson arrivals (exponential inter-arrival times of mean 1 / rate); each
    request names a uniform random stream, N = floor(2^(lo + (hi - lo) U)) and a
    dtype uniform over {uint32, FP32 uniform, FP32 normal}."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=num_requests)
    arrivals = np.cumsum(gaps)
    streams = rng.integers(0, num_streams, size=num_requests)
    ns = np.floor(np.exp2(lo_exp + (hi_exp - lo_exp) * rng.random(num_requests))).astype(np.int64)
    ns = np.clip(ns, 1 << lo_exp, 1 << hi_exp)
    dtypes = rng.integers(0, 3, size=num_requests)
    return [Request(i, float(arrivals[i]), int(streams[i]), int(ns[i]), int(dtypes[i]))
            for i in range(num_requests)]
