"""Device-resident xorgens streams: torch owns the memory, libxg does the work.

PyTorch is used here only to allocate device buffers and to name the HIP
stream; each method is one call through the C ABI (paper_1108_0486_amd.xg).
"""
from __future__ import annotations

import numpy as np
import torch

from . import xg


def _stream_handle(stream: torch.cuda.Stream | None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class XorgensStreams:
    """num_streams streams of one family member (xg.XG_FAMILY_*, default
    Section 2's); stream i is seeded from seed + i."""

    def __init__(self, num_streams: int, seed: int, device: str | torch.device = "cuda",
                 stream: torch.cuda.Stream | None = None, state: torch.Tensor | None = None,
                 family: int = xg.XG_FAMILY_R128_W32):
        self.device = torch.device(device)
        self.num_streams = int(num_streams)
        self.family = int(family)
        nbytes = xg.xg_family_state_bytes(self.family, self.num_streams)
        if nbytes == 0:
            raise ValueError("unknown family %r" % family)
        if state is None:
            self.state = torch.empty(nbytes // 4, dtype=torch.int32, device=self.device)
            with torch.cuda.device(self.device):
                self.ctx = xg.xg_init_family(self.family, self.state.data_ptr(), nbytes, self.num_streams, seed,
                                             _stream_handle(stream))
        else:
            if state.numel() * state.element_size() < nbytes or not state.is_cuda:
                raise ValueError("state buffer too small or not on a GPU")
            self.state = state
            with torch.cuda.device(self.device):
                self.ctx = xg.xg_attach_family(self.family, self.state.data_ptr(), nbytes, self.num_streams)

    @classmethod
    def attach(cls, state: torch.Tensor, num_streams: int, family: int = xg.XG_FAMILY_R128_W32) -> "XorgensStreams":
        return cls(num_streams, 0, device=state.device, state=state, family=family)

    def close(self) -> None:
        if getattr(self, "ctx", None) is not None:
            xg.xg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- batch scratch ---------------------------------------------------------
    def batch_scratch(self, max_reqs: int, max_tiles: int = 0, tile_words: int = 0,
                      stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """Device scratch of xg_generate_batch on these streams, attached to the
        handle: reused while it holds max_reqs requests with the same tile
        setting, else replaced by a new one."""
        cfg = getattr(self, "_batch_cfg", None)
        max_reqs = max(1, int(max_reqs))
        if cfg is not None and cfg[0] >= max_reqs and cfg[1:] == (max_tiles, tile_words):
            return self._batch_scratch
        nbytes = xg.xg_batch_scratch_bytes(self.ctx, max_reqs, max_tiles)
        if nbytes == 0:
            raise ValueError("no batch scratch for %d requests and %d tiles" % (max_reqs, max_tiles))
        buf = torch.empty((nbytes + 3) // 4, dtype=torch.int32, device=self.device)
        if buf.data_ptr() % 256:
            raise RuntimeError("batch scratch is not 256-byte aligned")
        with torch.cuda.device(self.device):
            xg.xg_set_batch_scratch(self.ctx, buf.data_ptr(), nbytes, max_reqs, max_tiles, tile_words,
                                    _stream_handle(stream))
        self._batch_scratch, self._batch_cfg = buf, (max_reqs, max_tiles, tile_words)
        return buf

    # ---- tuning -----------------------------------------------------------
    def set_plain_tune(self, waves_per_block: int, unroll: int, store_words: int = 0) -> None:
        xg.xg_set_plain_tune(self.ctx, waves_per_block, unroll, store_words)

    def plain_tune(self) -> tuple:
        return xg.xg_get_plain_tune(self.ctx)

    # ---- plain launches -------------------------------------------------------
    def _range(self, first: int, count: int | None) -> tuple[int, int]:
        return first, (self.num_streams - first if count is None else count)

    def _out(self, out, shape, dtype):
        """A new output tensor, or the caller's after checks that keep every
        kernel write inside it: on a GPU, contiguous, elements of the dtype's
        width, and at least as many as the call writes."""
        if out is None:
            return torch.empty(shape, dtype=dtype, device=self.device)
        need = 1
        for d in shape:
            need *= int(d)
        width = dtype.itemsize
        if not out.is_cuda:
            raise ValueError("out must be a GPU tensor")
        if not out.is_contiguous():
            raise ValueError("out must be contiguous")
        if out.element_size() != width:
            raise ValueError("out has %d-byte elements; this call writes %d-byte values" % (out.element_size(), width))
        if out.numel() < need:
            raise ValueError("out holds %d elements; this call writes %d" % (out.numel(), need))
        return out

    def u32(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
            stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """[count, n] int32 tensor holding the uint32 outputs' bits."""
        first, count = self._range(first, count)
        out = self._out(out, (count, n), torch.int32)
        xg.xg_generate_u32(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def f32(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
            stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        first, count = self._range(first, count)
        out = self._out(out, (count, n), torch.float32)
        xg.xg_generate_f32(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def fill_u32(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
                 stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """count * n int32 (uint32 bits) in the bulk-fill layout (xg.fill_index)."""
        first, count = self._range(first, count)
        out = self._out(out, (count * n,), torch.int32)
        xg.xg_fill_u32(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def fill_f32(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
                 stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        first, count = self._range(first, count)
        out = self._out(out, (count * n,), torch.float32)
        xg.xg_fill_f32(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def u64(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
            stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """[count, n] int64 tensor holding the uint64 outputs' bits (64-bit member)."""
        first, count = self._range(first, count)
        out = self._out(out, (count, n), torch.int64)
        xg.xg_generate_u64(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def f64(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
            stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        first, count = self._range(first, count)
        out = self._out(out, (count, n), torch.float64)
        xg.xg_generate_f64(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def fill_u64(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
                 stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """count * n int64 (uint64 bits) in the bulk-fill layout (xg.fill_index, chunk 32)."""
        first, count = self._range(first, count)
        out = self._out(out, (count * n,), torch.int64)
        xg.xg_fill_u64(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def fill_f64(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
                 stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        first, count = self._range(first, count)
        out = self._out(out, (count * n,), torch.float64)
        xg.xg_fill_f64(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def normal_f64(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
                   stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """FP64 Box-Muller normals (64-bit member only); consumes 2 ceil(n / 2) words."""
        first, count = self._range(first, count)
        out = self._out(out, (count, n), torch.float64)
        xg.xg_generate_normal_f64(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def moments_f64(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
                    stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """[count, 2] FP64 sums of z and z^2 over n fused normals (64-bit member)."""
        first, count = self._range(first, count)
        out = self._out(out, (count, 2), torch.float64)
        xg.xg_normal_moments_f64(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def normal(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
               stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        first, count = self._range(first, count)
        out = self._out(out, (count, n), torch.float32)
        xg.xg_generate_normal(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def moments(self, n: int, first: int = 0, count: int | None = None, out: torch.Tensor | None = None,
                stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """[count, 2] float32: sum of z and sum of z^2 over n normals."""
        first, count = self._range(first, count)
        out = self._out(out, (count, 2), torch.float32)
        xg.xg_normal_moments(self.ctx, first, count, n, out.data_ptr(), _stream_handle(stream))
        return out

    def skip(self, J: int, first: int = 0, count: int | None = None,
             stream: torch.cuda.Stream | None = None) -> None:
        """Advances the selected streams by J words without producing them."""
        first, count = self._range(first, count)
        xg.xg_skip(self.ctx, first, count, J, _stream_handle(stream))

    # ---- state --------------------------------------------------------------
    def host_state(self, idx=None):
        """(ring[k, r], weyl[k], pos[k] uint64) of the selected streams: ring
        and weyl uint32 for the 32-bit members (r = 128 or 64), uint64 for
        the 64-bit member (r = 64)."""
        if self.family != xg.XG_FAMILY_R128_W32:
            per = xg.xg_family_state_bytes(self.family, 1) // 4
            words = self.state[: self.num_streams * per].view(self.num_streams, per)
            if idx is not None:
                words = words[torch.as_tensor(idx, device=self.device)]
            a = words.cpu().numpy().view(np.uint32)
            if self.family == xg.XG_FAMILY_R64_W64:
                q = a.view(np.uint64)
                return q[:, :64].copy(), q[:, 64].copy(), q[:, 65].copy()
            return a[:, :64].copy(), a[:, 64].copy(), a.view(np.uint64)[:, 33].copy()
        words = self.state.view(self.num_streams, xg.XG_STATE_WORDS)
        if idx is not None:
            words = words[torch.as_tensor(idx, device=self.device)]
        a = words.cpu().numpy().view(np.uint32)
        ring = a[:, :128].copy()
        weyl = a[:, 128].copy()
        pos = a[:, 130].astype(np.uint64) | (a[:, 131].astype(np.uint64) << np.uint64(32))
        return ring, weyl, pos

    def checkpoint(self) -> torch.Tensor:
        return self.state.clone()

    def restore(self, saved: torch.Tensor) -> None:
        self.state.copy_(saved)


def as_u32(t: torch.Tensor) -> np.ndarray:
    """Host uint32 view of an int32 device tensor of generator outputs."""
    return t.cpu().numpy().view(np.uint32)
