"""ctypes binding of libxg (include/xg.h), with the same function names.

Argument marshalling only: every step of generation runs in the HIP kernels
of libxg.so.  Pointers are passed as integers (device addresses from
torch tensors' data_ptr()), HIP streams as integers (torch's cuda_stream).
If libxg.so has not been built this module raises on first use; there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libxg.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "xg.h")

XG_OK = 0
XG_EINVAL = -1
XG_ERANGE = -2
XG_EALIGN = -3
XG_EHIP = -4
XG_ENOTSUP = -5
XG_ENOMEM = -6
XG_EBUSY = -7

XG_STATE_WORDS = 132
XG_U32, XG_F32, XG_NORMAL = 0, 1, 2
XG_U64, XG_F64 = 4, 5
XG_FAMILY_R128_W32, XG_FAMILY_R64_W32, XG_FAMILY_R64_W64 = 0, 1, 2


class XgError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, strerror(status), status))


class xg_request(ctypes.Structure):
    _fields_ = [("stream", ctypes.c_uint64), ("n", ctypes.c_uint64), ("out_offset", ctypes.c_uint64),
                ("dtype", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class xg_tune(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_uint32), ("unroll", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32), ("store_words", ctypes.c_uint32)]

    @classmethod
    def of(cls, shape) -> "xg_tune":
        """(waves_per_block, unroll, blocks_per_cu[, store_words]); store_words 0 = default."""
        shape = tuple(shape) + (0,) * (4 - len(shape))
        return cls(*shape)

    def as_tuple(self):
        return (self.waves_per_block, self.unroll, self.blocks_per_cu, self.store_words)


class xg_server_config(ctypes.Structure):
    _fields_ = [("num_lanes", ctypes.c_uint32), ("max_batch", ctypes.c_uint32), ("tune", xg_tune),
                ("segment_words", ctypes.c_uint64), ("tune_key", ctypes.c_char_p)]


class xg_completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("stream", ctypes.c_uint64), ("n", ctypes.c_uint64),
                ("out_offset", ctypes.c_uint64), ("start_pos", ctypes.c_uint64),
                ("t_submit_ns", ctypes.c_uint64), ("t_launch_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("dtype", ctypes.c_uint32), ("lane", ctypes.c_uint32)]


class xg_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("submitted", "completed", "batches", "admitted", "max_lanes_busy",
                                              "max_batch_seen", "pool_high_water", "admission_waits")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libxg.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libxg.so is not built (%s); run `python -m paper_1108_0486_amd.build`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    st = ctypes.c_int32
    P = ctypes.POINTER
    sig = {
        "xg_state_bytes": (ctypes.c_size_t, [u64]),
        "xg_init_streams": (st, [P(vp), vp, ctypes.c_size_t, u64, u64, vp]),
        "xg_attach_streams": (st, [P(vp), vp, ctypes.c_size_t, u64]),
        "xg_destroy": (None, [vp]),
        "xg_num_streams": (u64, [vp]),
        "xg_state_ptr": (vp, [vp]),
        "xg_set_plain_tune": (st, [vp, P(xg_tune)]),
        "xg_get_plain_tune": (st, [vp, P(xg_tune)]),
        "xg_generate_u32": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_generate_f32": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_generate_normal": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_normal_moments": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_fill_u32": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_skip": (st, [vp, u64, u64, u64, vp]),
        "xg_box_muller": (st, [vp, u64, vp, vp]),
        "xg_jump_polynomial": (st, [u64, P(u64)]),
        "xg_family_jump_polynomial": (st, [u32, u64, P(u64)]),
        "xg_fill_f32": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_fill_value": (st, [vp, u64, u32, vp]),
        "xg_family_state_bytes": (ctypes.c_size_t, [u32, u64]),
        "xg_init_family": (st, [P(vp), u32, vp, ctypes.c_size_t, u64, u64, vp]),
        "xg_attach_family": (st, [P(vp), u32, vp, ctypes.c_size_t, u64]),
        "xg_family": (u32, [vp]),
        "xg_generate_u64": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_generate_f64": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_fill_u64": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_fill_f64": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_generate_normal_f64": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_normal_moments_f64": (st, [vp, u64, u64, u64, vp, vp]),
        "xg_batch_workspace_bytes": (ctypes.c_size_t, []),
        "xg_plan_batch": (st, [P(xg_request), u32, u64, u64, P(xg_request), P(u32), P(u32)]),
        "xg_generate_batch_planned": (st, [vp, vp, u32, vp, u32, vp, u64, P(xg_tune), vp, vp]),
        "xg_batch_scratch_bytes": (ctypes.c_size_t, [vp, u32, u32]),
        "xg_set_batch_scratch": (st, [vp, vp, ctypes.c_size_t, u32, u32, u64, vp]),
        "xg_generate_batch": (st, [vp, vp, u32, vp, ctypes.c_char_p, vp]),
        "xg_autotune_batch": (st, [vp, vp, u32, vp, vp, ctypes.c_char_p, i32, P(xg_tune),
                                   P(ctypes.c_float), u32, P(u32), vp]),
        "xg_tune_cache_load": (st, [ctypes.c_char_p]),
        "xg_tune_cache_save": (st, [ctypes.c_char_p]),
        "xg_tune_cache_put": (st, [ctypes.c_char_p, u32, u32, ctypes.c_char_p, P(xg_tune), ctypes.c_float]),
        "xg_tune_cache_get": (st, [ctypes.c_char_p, u32, u32, ctypes.c_char_p, P(xg_tune),
                                   P(ctypes.c_float)]),
        "xg_tune_cache_size": (u32, []),
        "xg_tune_cache_clear": (None, []),
        "xg_tune_identity": (st, [vp, ctypes.c_char_p, ctypes.c_size_t, P(u32)]),
        "xg_batch_read_plan": (st, [vp, P(xg_request), u32, P(u32), u32, P(u32), P(u32), vp]),
        "xg_generate_batch_static": (st, [vp, vp, u32, vp, ctypes.c_char_p, vp, vp]),
        "xg_strerror": (ctypes.c_char_p, [st]),
        "xg_server_device_bytes": (ctypes.c_size_t, [P(xg_server_config)]),
        "xg_server_create": (st, [P(vp), vp, P(xg_server_config), vp, u64, vp, ctypes.c_size_t]),
        "xg_server_submit": (st, [vp, u64, u64, u64, u32]),
        "xg_server_poll": (st, [vp, P(xg_completion), u32, P(u32)]),
        "xg_server_release": (st, [vp, u64]),
        "xg_server_outstanding": (u64, [vp]),
        "xg_server_get_stats": (st, [vp, P(xg_server_stats)]),
        "xg_server_destroy": (None, [vp]),
        "xg_server_get_tune": (st, [vp, P(xg_tune)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions include/xg.h declares."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xg_[a-z0-9_]+)\s*\(", text)))


def strerror(status: int) -> str:
    return lib().xg_strerror(status).decode()


def _check(status: int, where: str) -> None:
    if status != XG_OK:
        raise XgError(status, where)


# ---- thin wrappers with the C names ------------------------------------------

def xg_state_bytes(num_streams: int) -> int:
    return int(lib().xg_state_bytes(num_streams))


def xg_init_streams(d_state: int, state_bytes: int, num_streams: int, seed: int, stream: int = 0):
    ctx = ctypes.c_void_p()
    _check(lib().xg_init_streams(ctypes.byref(ctx), d_state, state_bytes, num_streams,
                                 seed & (2**64 - 1), stream), "xg_init_streams")
    return ctx


def xg_attach_streams(d_state: int, state_bytes: int, num_streams: int):
    ctx = ctypes.c_void_p()
    _check(lib().xg_attach_streams(ctypes.byref(ctx), d_state, state_bytes, num_streams),
           "xg_attach_streams")
    return ctx


def xg_destroy(ctx) -> None:
    lib().xg_destroy(ctx)


def xg_set_plain_tune(ctx, waves_per_block: int, unroll: int, store_words: int = 0) -> None:
    t = xg_tune(waves_per_block, unroll, 1, store_words)
    _check(lib().xg_set_plain_tune(ctx, ctypes.byref(t)), "xg_set_plain_tune")


def xg_get_plain_tune(ctx) -> tuple:
    """(waves_per_block, unroll, store_words) of the plain launches."""
    t = xg_tune()
    _check(lib().xg_get_plain_tune(ctx, ctypes.byref(t)), "xg_get_plain_tune")
    return (t.waves_per_block, t.unroll, t.store_words)


def xg_generate_u32(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_generate_u32(ctx, first, count, n, d_out, stream), "xg_generate_u32")


def xg_generate_f32(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_generate_f32(ctx, first, count, n, d_out, stream), "xg_generate_f32")


def xg_generate_normal(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_generate_normal(ctx, first, count, n, d_out, stream), "xg_generate_normal")


def xg_normal_moments(ctx, first: int, count: int, n: int, d_sums: int, stream: int = 0) -> None:
    _check(lib().xg_normal_moments(ctx, first, count, n, d_sums, stream), "xg_normal_moments")


def xg_fill_u32(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_fill_u32(ctx, first, count, n, d_out, stream), "xg_fill_u32")


def xg_fill_f32(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_fill_f32(ctx, first, count, n, d_out, stream), "xg_fill_f32")


def fill_index(count: int, n: int, chunk: int = 64):
    """numpy index array idx[k, t]: where xg_fill_* put value t of the k-th
    stream (chunk = 64 words for Section 2's member, 32 for the others)."""
    import numpy as np
    full, rem = n // chunk, n % chunk
    t = np.arange(n, dtype=np.int64)
    k = np.arange(count, dtype=np.int64)[:, None]
    head = (t // chunk) * chunk * count + k * chunk + t % chunk
    tail = chunk * full * count + k * rem + (t - chunk * full)
    return np.where(t < chunk * full, head, tail)


def xg_fill_value(d_out: int, words: int, value: int, stream: int = 0) -> None:
    _check(lib().xg_fill_value(d_out, words, value & 0xFFFFFFFF, stream), "xg_fill_value")


def xg_family_state_bytes(family: int, num_streams: int) -> int:
    return int(lib().xg_family_state_bytes(family, num_streams))


def xg_init_family(family: int, d_state: int, state_bytes: int, num_streams: int, seed: int, stream: int = 0):
    ctx = ctypes.c_void_p()
    _check(lib().xg_init_family(ctypes.byref(ctx), family, d_state, state_bytes, num_streams,
                                seed & (2**64 - 1), stream), "xg_init_family")
    return ctx


def xg_attach_family(family: int, d_state: int, state_bytes: int, num_streams: int):
    ctx = ctypes.c_void_p()
    _check(lib().xg_attach_family(ctypes.byref(ctx), family, d_state, state_bytes, num_streams),
           "xg_attach_family")
    return ctx


def xg_family(ctx) -> int:
    return int(lib().xg_family(ctx))


def xg_generate_u64(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_generate_u64(ctx, first, count, n, d_out, stream), "xg_generate_u64")


def xg_generate_f64(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_generate_f64(ctx, first, count, n, d_out, stream), "xg_generate_f64")


def xg_fill_u64(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_fill_u64(ctx, first, count, n, d_out, stream), "xg_fill_u64")


def xg_fill_f64(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_fill_f64(ctx, first, count, n, d_out, stream), "xg_fill_f64")


def xg_generate_normal_f64(ctx, first: int, count: int, n: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_generate_normal_f64(ctx, first, count, n, d_out, stream), "xg_generate_normal_f64")


def xg_normal_moments_f64(ctx, first: int, count: int, n: int, d_sums: int, stream: int = 0) -> None:
    _check(lib().xg_normal_moments_f64(ctx, first, count, n, d_sums, stream), "xg_normal_moments_f64")


def xg_box_muller(d_words: int, pairs: int, d_out: int, stream: int = 0) -> None:
    _check(lib().xg_box_muller(d_words, pairs, d_out, stream), "xg_box_muller")


def xg_skip(ctx, first: int, count: int, J: int, stream: int = 0) -> None:
    _check(lib().xg_skip(ctx, first, count, J, stream), "xg_skip")


def xg_jump_polynomial(J: int) -> int:
    """z^J mod P as a Python int (bit i = coefficient of z^i)."""
    g = (ctypes.c_uint64 * 64)()
    _check(lib().xg_jump_polynomial(J, g), "xg_jump_polynomial")
    return sum(int(g[k]) << (64 * k) for k in range(64))


def xg_family_jump_polynomial(family: int, J: int) -> int:
    """z^J mod P of a family member's x-part, as a Python int."""
    g = (ctypes.c_uint64 * 64)()
    _check(lib().xg_family_jump_polynomial(family, J, g), "xg_family_jump_polynomial")
    return sum(int(g[k]) << (64 * k) for k in range(64))


def xg_batch_workspace_bytes() -> int:
    return int(lib().xg_batch_workspace_bytes())


def xg_plan_batch(requests, num_streams: int, out_elems: int):
    """requests: sequence of (stream, n, out_offset, dtype).  Returns
    (sorted ctypes array of xg_request, list of group offsets)."""
    nr = len(requests)
    arr = (xg_request * max(1, nr))()
    for i, (s, n, off, dt) in enumerate(requests):
        arr[i] = xg_request(s, n, off, dt, 0)
    out = (xg_request * max(1, nr))()
    groups = (ctypes.c_uint32 * (nr + 1))()
    ng = ctypes.c_uint32()
    _check(lib().xg_plan_batch(arr, nr, num_streams, out_elems, out, groups, ctypes.byref(ng)),
           "xg_plan_batch")
    return out, list(groups[: ng.value + 1])


def xg_generate_batch_planned(ctx, d_reqs: int, num_reqs: int, d_groups: int, num_groups: int, d_out: int,
                              out_elems: int, tune: tuple | None, d_work: int, stream: int = 0) -> None:
    t = None if tune is None else ctypes.byref(xg_tune.of(tune))
    _check(lib().xg_generate_batch_planned(ctx, d_reqs, num_reqs, d_groups, num_groups, d_out, out_elems, t,
                                           d_work, stream), "xg_generate_batch_planned")


def _key(tune_key: str | None):
    return None if tune_key is None else tune_key.encode()


def xg_batch_scratch_bytes(ctx, max_reqs: int, max_tiles: int = 0) -> int:
    return int(lib().xg_batch_scratch_bytes(ctx, max_reqs, max_tiles))


def xg_set_batch_scratch(ctx, d_scratch: int | None, scratch_bytes: int, max_reqs: int, max_tiles: int = 0,
                         tile_words: int = 0, stream: int = 0) -> None:
    _check(lib().xg_set_batch_scratch(ctx, d_scratch, scratch_bytes, max_reqs, max_tiles, tile_words, stream),
           "xg_set_batch_scratch")


def xg_generate_batch(ctx, d_reqs: int, num_reqs: int, d_out: int, tune_key: str | None = None,
                      stream: int = 0) -> None:
    _check(lib().xg_generate_batch(ctx, d_reqs, num_reqs, d_out, _key(tune_key), stream), "xg_generate_batch")


XG_STATIC_MAX_REQS = 65536


def xg_generate_batch_static(ctx, d_reqs: int, num_reqs: int, d_out: int, tune_key: str | None = None,
                             d_error: int | None = None, stream: int = 0) -> None:
    _check(lib().xg_generate_batch_static(ctx, d_reqs, num_reqs, d_out, _key(tune_key), d_error, stream),
           "xg_generate_batch_static")


def xg_autotune_batch(ctx, d_reqs: int, num_reqs: int, d_scratch_out: int, d_scratch_state: int,
                      tune_key: str | None = None, reps: int = 3, stream: int = 0):
    """Returns (best (wpb, unroll, bpc, store_words), [(wpb, unroll, bpc, store_words, ms), ...])."""
    best = xg_tune()
    maxt = 256
    times = (ctypes.c_float * (5 * maxt))()
    nt = ctypes.c_uint32()
    _check(lib().xg_autotune_batch(ctx, d_reqs, num_reqs, d_scratch_out, d_scratch_state, _key(tune_key), reps,
                                   ctypes.byref(best), times, maxt, ctypes.byref(nt), stream), "xg_autotune_batch")
    recs = [(int(times[5 * i]), int(times[5 * i + 1]), int(times[5 * i + 2]), int(times[5 * i + 4]),
             float(times[5 * i + 3])) for i in range(nt.value)]
    return best.as_tuple(), recs


def xg_batch_read_plan(ctx, max_entries: int, max_groups: int, stream: int = 0):
    """The last planned table: ([(stream, n, out_offset, dtype, flags)], [group offsets])."""
    table = (xg_request * max(1, max_entries))()
    groups = (ctypes.c_uint32 * (max_groups + 1))()
    ne, ng = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().xg_batch_read_plan(ctx, table, max_entries, groups, max_groups, ctypes.byref(ne), ctypes.byref(ng),
                                    stream), "xg_batch_read_plan")
    rows = [(table[i].stream, table[i].n, table[i].out_offset, table[i].dtype, table[i].flags) for i in range(ne.value)]
    return rows, list(groups[: ng.value + 1])


def xg_tune_cache_load(path: str) -> None:
    _check(lib().xg_tune_cache_load(path.encode()), "xg_tune_cache_load")


def xg_tune_cache_save(path: str) -> None:
    _check(lib().xg_tune_cache_save(path.encode()), "xg_tune_cache_save")


def xg_tune_cache_put(arch: str, cus: int, family: int, tune_key: str, tune, ms: float = float("nan")) -> None:
    _check(lib().xg_tune_cache_put(arch.encode(), cus, family, tune_key.encode(), ctypes.byref(xg_tune.of(tune)),
                                   ms), "xg_tune_cache_put")


def xg_tune_cache_get(arch: str, cus: int, family: int, tune_key: str):
    """(shape tuple, ms) of an entry, or None when the cache has no such key."""
    t = xg_tune()
    ms = ctypes.c_float()
    st = lib().xg_tune_cache_get(arch.encode(), cus, family, tune_key.encode(), ctypes.byref(t), ctypes.byref(ms))
    if st == XG_ERANGE:
        return None
    _check(st, "xg_tune_cache_get")
    return t.as_tuple(), float(ms.value)


def xg_tune_cache_size() -> int:
    return int(lib().xg_tune_cache_size())


def xg_tune_cache_clear() -> None:
    lib().xg_tune_cache_clear()


def xg_tune_identity(ctx):
    """(arch, compute units) under which calls on ctx look shapes up."""
    buf = ctypes.create_string_buffer(64)
    cus = ctypes.c_uint32()
    _check(lib().xg_tune_identity(ctx, buf, 64, ctypes.byref(cus)), "xg_tune_identity")
    return buf.value.decode(), int(cus.value)


# ---- serving -----------------------------------------------------------------

def xg_server_device_bytes(num_lanes: int, max_batch: int, segment_words: int = 0) -> int:
    cfg = xg_server_config(num_lanes, max_batch, xg_tune(), segment_words, None)
    return int(lib().xg_server_device_bytes(ctypes.byref(cfg)))


def xg_server_create(ctx, num_lanes: int, max_batch: int, tune, d_pool: int, pool_elems: int,
                     d_tables: int, tables_bytes: int, segment_words: int = 0, tune_key: str | None = None):
    cfg = xg_server_config(num_lanes, max_batch, xg_tune() if tune is None else xg_tune.of(tune), segment_words,
                           _key(tune_key))
    srv = ctypes.c_void_p()
    _check(lib().xg_server_create(ctypes.byref(srv), ctx, ctypes.byref(cfg), d_pool, pool_elems, d_tables,
                                  tables_bytes), "xg_server_create")
    return srv


def xg_server_submit(srv, rid: int, stream: int, n: int, dtype: int) -> None:
    _check(lib().xg_server_submit(srv, rid, stream, n, dtype), "xg_server_submit")


def xg_server_poll(srv, buf, max_out: int) -> int:
    """Fills the ctypes array `buf` (xg_completion * max_out); returns the count."""
    k = ctypes.c_uint32()
    _check(lib().xg_server_poll(srv, buf, max_out, ctypes.byref(k)), "xg_server_poll")
    return k.value


def xg_server_release(srv, rid: int) -> None:
    _check(lib().xg_server_release(srv, rid), "xg_server_release")


def xg_server_outstanding(srv) -> int:
    return int(lib().xg_server_outstanding(srv))


def xg_server_get_stats(srv) -> dict:
    st = xg_server_stats()
    _check(lib().xg_server_get_stats(srv, ctypes.byref(st)), "xg_server_get_stats")
    return st.as_dict()


def xg_server_get_tune(srv) -> tuple:
    t = xg_tune()
    _check(lib().xg_server_get_tune(srv, ctypes.byref(t)), "xg_server_get_tune")
    return t.as_tuple()


def xg_server_destroy(srv) -> None:
    lib().xg_server_destroy(srv)
