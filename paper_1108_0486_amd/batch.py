"""Batched requests served by one persistent launch.

Batch: the one-call path (xg_generate_batch).  The request table goes to the
device in the caller's order; libxg groups it by stream, orders it and serves
it on the device, so a call (or a captured HIP graph of it) needs no host
round trip.  The launch shape comes from libxg's tuning cache by key.

PlannedBatch: the host-planned path (xg_plan_batch, then
xg_generate_batch_planned with an explicit shape).

torch provides the device buffers and the graph object; planning, the queue
and generation are libxg's.
"""
from __future__ import annotations

import numpy as np
import torch

from . import xg
from .streams import XorgensStreams, _stream_handle


def _table(requests) -> np.ndarray:
    """(stream, n, out_offset, dtype) tuples as xg_request records (flags 0)."""
    arr = np.zeros(max(1, len(requests)), dtype=[("stream", "<u8"), ("n", "<u8"), ("out_offset", "<u8"),
                                                 ("dtype", "<u4"), ("flags", "<u4")])
    if len(requests):
        cols = np.array(requests, dtype=np.uint64).reshape(len(requests), 4)
        arr["stream"][: len(requests)] = cols[:, 0]
        arr["n"][: len(requests)] = cols[:, 1]
        arr["out_offset"][: len(requests)] = cols[:, 2]
        arr["dtype"][: len(requests)] = cols[:, 3]
    return arr


def _out_buffer(streams: XorgensStreams, out_elems: int, out: torch.Tensor | None) -> torch.Tensor:
    # Elements are the member's word width: 8 bytes for the 64-bit member, else 4.
    width = 8 if streams.family == xg.XG_FAMILY_R64_W64 else 4
    if out is not None and (not out.is_cuda or not out.is_contiguous() or out.element_size() != width
                            or out.numel() < out_elems):
        raise ValueError("out must be a contiguous GPU tensor of at least out_elems %d-byte elements" % width)
    if out is None:
        out = torch.empty(max(1, out_elems), dtype=torch.int64 if width == 8 else torch.int32,
                          device=streams.device)
    return out


def shape_key(tune) -> str:
    """Tuning-cache key under which Batch.run(tune=...) stores an explicit shape."""
    t = tuple(tune) + (0,) * (4 - len(tuple(tune)))
    return "shape/%d/%d/%d/%d" % t


class Batch:
    """requests: (stream, n, out_offset, dtype) in the order they are to be
    served on each stream.  tile_words / max_tiles: split long single
    requests of a stream into tiles (xg_set_batch_scratch)."""

    def __init__(self, streams: XorgensStreams, requests, out_elems: int, out: torch.Tensor | None = None,
                 tile_words: int = 0, max_tiles: int = 0, table: torch.Tensor | None = None):
        self.streams = streams
        self.requests = [tuple(int(v) for v in r) for r in requests]
        self.num_reqs = len(self.requests)
        self.out_elems = int(out_elems)
        self.tile_words, self.max_tiles = int(tile_words), int(max_tiles) if tile_words else 0
        raw = _table(self.requests).view(np.int32)
        self.d_reqs = torch.from_numpy(raw.copy()).to(streams.device) if table is None else table
        self.out = _out_buffer(streams, self.out_elems, out)
        self.scratch = streams.batch_scratch(self.num_reqs, self.max_tiles, self.tile_words)

    def requests_in_order(self):
        """(stream, n, out_offset, dtype) in the order each stream serves them."""
        return list(self.requests)

    def _key(self, tune, tune_key):
        if tune is None:
            return tune_key
        arch, cus = xg.xg_tune_identity(self.streams.ctx)
        key = shape_key(tune)
        xg.xg_tune_cache_put(arch, cus, self.streams.family, key, tune)
        return key

    def run(self, tune=None, tune_key: str | None = None, stream: torch.cuda.Stream | None = None) -> None:
        """tune: an explicit shape (stored in the tuning cache under shape_key(tune)); else tune_key."""
        key = self._key(tune, tune_key)
        self.scratch = self.streams.batch_scratch(self.num_reqs, self.max_tiles, self.tile_words, stream)
        xg.xg_generate_batch(self.streams.ctx, self.d_reqs.data_ptr(), self.num_reqs, self.out.data_ptr(), key,
                             _stream_handle(stream))

    def capture_graph(self, tune=None, tune_key: str | None = None) -> torch.cuda.CUDAGraph:
        """Captures the whole call (planning kernels and batched launch) once;
        each replay serves the table again from the streams' current positions."""
        key = self._key(tune, tune_key)
        self.scratch = self.streams.batch_scratch(self.num_reqs, self.max_tiles, self.tile_words)
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            self.run(tune_key=key)
        return g

    def error_flag(self) -> int:
        return int(self.scratch[1].item())

    def served_counts(self):
        """(queue items, table entries) of the last planned call."""
        return int(self.scratch[2].item()), int(self.scratch[3].item())

    def served_plan(self):
        """The last planned table: ([(stream, n, out_offset, dtype, flags)], [item offsets])."""
        return xg.xg_batch_read_plan(self.streams.ctx, self.num_reqs + self.max_tiles, self.num_reqs + self.max_tiles,
                                     _stream_handle(None))

    def autotune(self, reps: int = 3, tune_key: str | None = None, stream: torch.cuda.Stream | None = None):
        """Times every launch shape on a scratch copy of the state (storing the
        best under tune_key); returns (best (wpb, unroll, bpc, store_words),
        [(wpb, unroll, bpc, store_words, ms)])."""
        self.scratch = self.streams.batch_scratch(self.num_reqs, self.max_tiles, self.tile_words, stream)
        scratch_state = torch.empty_like(self.streams.state)
        scratch_out = torch.empty_like(self.out)
        return xg.xg_autotune_batch(self.streams.ctx, self.d_reqs.data_ptr(), self.num_reqs, scratch_out.data_ptr(),
                                    scratch_state.data_ptr(), tune_key, reps, _stream_handle(stream))


class PlannedBatch:
    """The host-planned path: xg_plan_batch on the host, then
    xg_generate_batch_planned with an explicit launch shape."""

    def __init__(self, streams: XorgensStreams, requests, out_elems: int, out: torch.Tensor | None = None):
        self.streams = streams
        self.num_reqs = len(requests)
        self.out_elems = int(out_elems)
        arr, groups = xg.xg_plan_batch(list(requests), streams.num_streams, self.out_elems)
        self.num_groups = len(groups) - 1
        self._order = [(arr[i].stream, arr[i].n, arr[i].out_offset, arr[i].dtype) for i in range(self.num_reqs)]
        raw = np.frombuffer(bytes(memoryview(arr))[: 32 * max(1, self.num_reqs)], dtype=np.int32).copy()
        dev = streams.device
        self.d_reqs = torch.from_numpy(raw).to(dev)
        self.d_groups = torch.from_numpy(np.array(groups, dtype=np.uint32).view(np.int32)).to(dev)
        self.out = _out_buffer(streams, self.out_elems, out)
        self.work = torch.zeros(xg.xg_batch_workspace_bytes() // 4, dtype=torch.int32, device=dev)

    def requests_in_order(self):
        """(stream, n, out_offset, dtype) in the planned (served) order."""
        return list(self._order)

    def run(self, tune=None, stream: torch.cuda.Stream | None = None) -> None:
        xg.xg_generate_batch_planned(self.streams.ctx, self.d_reqs.data_ptr(), self.num_reqs,
                                     self.d_groups.data_ptr(), self.num_groups, self.out.data_ptr(), self.out_elems,
                                     tune, self.work.data_ptr(), _stream_handle(stream))

    def capture_graph(self, tune=None) -> torch.cuda.CUDAGraph:
        """Captures (workspace fill, batched kernel) once; each replay serves
        the table again from the streams' current positions."""
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            self.run(tune=tune)
        return g

    def error_flag(self) -> int:
        return int(self.work[1].item())
