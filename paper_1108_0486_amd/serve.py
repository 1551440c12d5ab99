"""Request serving over device-resident streams (the libxg server) and the
drivers that replay a timed request trace through it.

The scheduling (admission by memory and per-stream order, batching, lanes,
completion) is libxg's (xg_server_*); this module allocates the device pool
with torch, replays arrivals in real time, and turns completion records into
latency statistics.
"""
from __future__ import annotations

import ctypes
import gc
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import xg
from .streams import XorgensStreams, _stream_handle


@dataclass
class Completion:
    id: int
    stream: int
    n: int
    dtype: int
    out_offset: int
    start_pos: int
    t_submit_ns: int
    t_launch_ns: int
    t_done_ns: int
    lane: int


class Server:
    def __init__(self, streams: XorgensStreams, pool_elems: int, num_lanes: int = 4, max_batch: int = 1024,
                 tune=None, segment_words: int = 0, tune_key: str | None = None):
        self.streams = streams
        # Pool elements are the member's word width: 8 bytes for the 64-bit member.
        wide = streams.family == xg.XG_FAMILY_R64_W64
        self.pool = torch.empty(pool_elems, dtype=torch.int64 if wide else torch.int32, device=streams.device)
        nbytes = xg.xg_server_device_bytes(num_lanes, max_batch, segment_words)
        if nbytes == 0:
            raise ValueError("invalid server configuration")
        self.tables = torch.empty(nbytes, dtype=torch.uint8, device=streams.device)
        self.srv = xg.xg_server_create(streams.ctx, num_lanes, max_batch, tune, self.pool.data_ptr(), pool_elems,
                                       self.tables.data_ptr(), nbytes, segment_words, tune_key)
        self._cap = 4096
        self._buf = (xg.xg_completion * self._cap)()

    def submit(self, rid: int, stream: int, n: int, dtype: int) -> None:
        xg.xg_server_submit(self.srv, rid, stream, n, dtype)

    def poll(self) -> list[Completion]:
        out = []
        while True:
            k = xg.xg_server_poll(self.srv, self._buf, self._cap)
            for i in range(k):
                c = self._buf[i]
                out.append(Completion(c.id, c.stream, c.n, c.dtype, c.out_offset, c.start_pos, c.t_submit_ns,
                                      c.t_launch_ns, c.t_done_ns, c.lane))
            if k < self._cap:
                return out

    def output(self, c: Completion) -> torch.Tensor:
        v = self.pool[c.out_offset:c.out_offset + c.n]
        if c.dtype == xg.XG_U32:
            return v
        return v.view(torch.float64 if v.element_size() == 8 else torch.float32)

    def release(self, rid: int) -> None:
        xg.xg_server_release(self.srv, rid)

    @property
    def outstanding(self) -> int:
        return xg.xg_server_outstanding(self.srv)

    def stats(self) -> dict:
        return xg.xg_server_get_stats(self.srv)

    def close(self) -> None:
        if self.srv is not None:
            xg.xg_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def latency_summary(lat_s: np.ndarray, total_rn: int, span_s: float, arrival_s: np.ndarray | None = None) -> dict:
    out = {"requests": int(lat_s.size), "p50_ms": float(np.percentile(lat_s, 50) * 1e3),
           "p99_ms": float(np.percentile(lat_s, 99) * 1e3), "max_ms": float(lat_s.max() * 1e3),
           "mean_ms": float(lat_s.mean() * 1e3), "rn": int(total_rn), "span_s": span_s,
           "rn_per_s": total_rn / span_s if span_s > 0 else 0.0,
           "over_10ms": int((lat_s > 0.010).sum())}
    if arrival_s is not None and lat_s.size:
        out["worst_arrival_s"] = float(arrival_s[int(lat_s.argmax())])
    return out


class _NoCollector:
    """Keeps Python's cyclic garbage collector off for a timed replay: a full
    collection over the hundreds of thousands of completion records would
    stall the polling loop (and so every request in flight) for tens of ms."""

    def __enter__(self):
        self.was = gc.isenabled()
        gc.collect()
        gc.disable()

    def __exit__(self, *exc):
        if self.was:
            gc.enable()


def run_trace(server: Server, trace, keep_outputs: bool = False, timeout_s: float = 120.0):
    """Replays `trace` (workloads.Request, arrival times in seconds from the
    start) in real time through the server.  Latency of a request: the host
    time its completion was seen minus its scheduled arrival.  Returns
    (summary, completions, outputs by id if keep_outputs)."""
    reqs = sorted(trace, key=lambda r: r.arrival_s)
    idx = 0
    done: list[Completion] = []
    outputs = {}
    arrival_ns = {}
    with _NoCollector():   # its collection runs before the clock starts
        t0 = time.monotonic_ns()
        deadline = t0 + int(timeout_s * 1e9)
        while len(done) < len(reqs):
            now = time.monotonic_ns()
            if now > deadline:
                raise TimeoutError("serving trace did not finish in %.0f s" % timeout_s)
            while idx < len(reqs) and t0 + int(reqs[idx].arrival_s * 1e9) <= now:
                r = reqs[idx]
                arrival_ns[r.rid] = t0 + int(r.arrival_s * 1e9)
                server.submit(r.rid, r.stream, r.n, r.dtype)
                idx += 1
            for c in server.poll():
                if keep_outputs:
                    outputs[c.id] = server.output(c).clone()
                server.release(c.id)
                done.append(c)
    lat = np.array([(c.t_done_ns - arrival_ns[c.id]) * 1e-9 for c in done])
    arr = np.array([(arrival_ns[c.id] - t0) * 1e-9 for c in done])
    span = (max(c.t_done_ns for c in done) - t0) * 1e-9
    summary = latency_summary(lat, sum(c.n for c in done), span, arr)
    summary["server"] = server.stats()
    return summary, done, outputs


def run_trace_plain_fifo(streams: XorgensStreams, trace, max_n: int, timeout_s: float = 120.0):
    """Baseline: each request is one plain launch (one stream, one wavefront)
    issued at its arrival, first in first out on a single HIP stream."""
    reqs = sorted(trace, key=lambda r: r.arrival_s)
    out = torch.empty(max_n, dtype=torch.int32, device=streams.device)
    stream = torch.cuda.current_stream()
    h = _stream_handle(stream)
    launch = {xg.XG_U32: xg.xg_generate_u32, xg.XG_F32: xg.xg_generate_f32, xg.XG_NORMAL: xg.xg_generate_normal}
    torch.cuda.synchronize()
    idx = 0
    inflight = []  # (event, request, arrival_ns)
    lat = []
    with _NoCollector():
        t0 = time.monotonic_ns()
        deadline = t0 + int(timeout_s * 1e9)
        while len(lat) < len(reqs):
            now = time.monotonic_ns()
            if now > deadline:
                raise TimeoutError("plain FIFO trace did not finish in %.0f s" % timeout_s)
            while idx < len(reqs) and t0 + int(reqs[idx].arrival_s * 1e9) <= now:
                r = reqs[idx]
                launch[r.dtype](streams.ctx, r.stream, 1, r.n, out.data_ptr(), h)
                ev = torch.cuda.Event()
                ev.record(stream)
                inflight.append((ev, r, t0 + int(r.arrival_s * 1e9)))
                idx += 1
            while inflight and inflight[0][0].query():
                _, r, a = inflight.pop(0)
                lat.append((time.monotonic_ns() - a) * 1e-9)
    span = (time.monotonic_ns() - t0) * 1e-9
    return latency_summary(np.array(lat), sum(r.n for r in reqs), span)


del ctypes
