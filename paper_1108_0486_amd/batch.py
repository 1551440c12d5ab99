"""Batched requests served by one persistent launch (xg_generate_batch).

The host plans the table once (xg_plan_batch: same-stream requests grouped in
order, groups largest first), copies it to the device, and then launches, or
captures the launch in a HIP graph and replays it.  torch provides the device
buffers and the graph object; the planning, the queue and the generation are
libxg's.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import xg
from .streams import XorgensStreams, _stream_handle


class Batch:
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
        # Elements are the member's word width: 8 bytes for the 64-bit member, else 4.
        width = 8 if streams.family == xg.XG_FAMILY_R64_W64 else 4
        if out is not None and (not out.is_cuda or not out.is_contiguous() or out.element_size() != width
                                or out.numel() < self.out_elems):
            raise ValueError("out must be a contiguous GPU tensor of at least out_elems %d-byte elements" % width)
        if out is None:
            out = torch.empty(max(1, self.out_elems), dtype=torch.int64 if width == 8 else torch.int32, device=dev)
        self.out = out
        self.work = torch.zeros(xg.xg_batch_workspace_bytes() // 4, dtype=torch.int32, device=dev)

    def requests_in_order(self):
        """(stream, n, out_offset, dtype) in the planned (served) order."""
        return list(self._order)

    def run(self, tune=None, stream: torch.cuda.Stream | None = None) -> None:
        xg.xg_generate_batch(self.streams.ctx, self.d_reqs.data_ptr(), self.num_reqs, self.d_groups.data_ptr(),
                             self.num_groups, self.out.data_ptr(), self.out_elems, tune, self.work.data_ptr(),
                             _stream_handle(stream))

    def capture_graph(self, tune=None) -> torch.cuda.CUDAGraph:
        """Captures (clear workspace, batched kernel) once; each replay serves
        the table again from the streams' current positions."""
        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            self.run(tune=tune)
        return g

    def error_flag(self) -> int:
        return int(self.work[1].item())

    def autotune(self, reps: int = 3, stream: torch.cuda.Stream | None = None):
        """Times every launch shape on a scratch copy of the state; returns
        (best (waves_per_block, unroll, blocks_per_cu, store_words),
         [(wpb, unroll, bpc, store_words, ms)])."""
        scratch_state = torch.empty_like(self.streams.state)
        scratch_out = torch.empty_like(self.out)
        return xg.xg_autotune_batch(self.streams.ctx, self.d_reqs.data_ptr(), self.num_reqs,
                                    self.d_groups.data_ptr(), self.num_groups, scratch_out.data_ptr(),
                                    self.out_elems, scratch_state.data_ptr(), self.work.data_ptr(),
                                    reps, _stream_handle(stream))


del ctypes
