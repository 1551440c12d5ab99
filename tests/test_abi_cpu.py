"""The C-ABI library without a GPU: it loads, exports every function the
header declares, rejects bad arguments synchronously, and plans batches."""
import ctypes
import subprocess

import pytest

from paper_1108_0486_amd import xg


def test_library_exports_every_declared_symbol():
    names = xg.header_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", xg.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = xg.lib()
    for n in names:
        assert hasattr(L, n)


def test_state_bytes_and_strerror():
    assert xg.xg_state_bytes(1) == 528
    assert xg.xg_state_bytes(100_000) == 52_800_000
    assert xg.xg_state_bytes(2**33) == 0
    for st in (0, -1, -2, -3, -4, -5, -6, -7):
        assert xg.strerror(st) != "unknown status"
    assert xg.strerror(-99) == "unknown status"
    assert xg.xg_batch_workspace_bytes() == 256


def test_null_arguments_rejected_without_gpu():
    L = xg.lib()
    assert L.xg_generate_u32(None, 0, 1, 16, None, None) == xg.XG_EINVAL
    assert L.xg_generate_f32(None, 0, 1, 16, None, None) == xg.XG_EINVAL
    assert L.xg_generate_normal(None, 0, 1, 16, None, None) == xg.XG_EINVAL
    assert L.xg_normal_moments(None, 0, 1, 16, None, None) == xg.XG_EINVAL
    assert L.xg_init_streams(None, None, 0, 1, 0, None) == xg.XG_EINVAL
    ctx = ctypes.c_void_p()
    assert L.xg_init_streams(ctypes.byref(ctx), None, 528, 1, 0, None) == xg.XG_EINVAL
    assert ctx.value is None
    assert L.xg_init_streams(ctypes.byref(ctx), 0x1000, 527, 1, 0, None) == xg.XG_ERANGE
    assert L.xg_init_streams(ctypes.byref(ctx), 0x1004, 528, 1, 0, None) == xg.XG_EALIGN
    assert L.xg_init_streams(ctypes.byref(ctx), 0x1000, 528, 0, 0, None) == xg.XG_EINVAL
    assert L.xg_generate_batch_planned(None, None, 0, None, 0, None, 0, None, None, None) == xg.XG_EINVAL
    assert L.xg_generate_batch(None, None, 0, None, None, None) == xg.XG_EINVAL
    assert L.xg_generate_batch(None, None, 0, None, b"k", None) == xg.XG_EINVAL
    assert L.xg_autotune_batch(None, None, 0, None, None, None, 1, None, None, 0, None, None) == xg.XG_EINVAL
    assert L.xg_set_batch_scratch(None, None, 0, 1, 0, 0, None) == xg.XG_EINVAL
    assert L.xg_batch_scratch_bytes(None, 1, 0) == 0
    assert L.xg_tune_identity(None, None, 0, None) == xg.XG_EINVAL
    assert L.xg_set_plain_tune(None, None) == xg.XG_EINVAL
    L.xg_destroy(None)
    assert L.xg_num_streams(None) == 0


def test_plan_batch_groups_and_orders():
    reqs = [(5, 100, 0, 0), (2, 1000, 100, 1), (5, 50, 1100, 2), (9, 10, 1150, 0), (2, 7, 1160, 0)]
    out, groups = xg.xg_plan_batch(reqs, num_streams=10, out_elems=2000)
    assert groups[0] == 0 and groups[-1] == len(reqs)
    seq = [(out[i].stream, out[i].n) for i in range(len(reqs))]
    # stream 2 (cost 1007) first, then stream 5 (100 + 4 * 50), then stream 9
    assert seq == [(2, 1000), (2, 7), (5, 100), (5, 50), (9, 10)]
    assert groups == [0, 2, 4, 5]


def test_plan_batch_rejects_bad_requests():
    with pytest.raises(xg.XgError) as e:
        xg.xg_plan_batch([(10, 1, 0, 0)], num_streams=10, out_elems=10)
    assert e.value.status == xg.XG_ERANGE
    with pytest.raises(xg.XgError) as e:
        xg.xg_plan_batch([(1, 11, 0, 0)], num_streams=10, out_elems=10)
    assert e.value.status == xg.XG_ERANGE
    with pytest.raises(xg.XgError) as e:
        xg.xg_plan_batch([(1, 2, 2**64 - 1, 0)], num_streams=10, out_elems=10)
    assert e.value.status == xg.XG_ERANGE
    with pytest.raises(xg.XgError) as e:
        xg.xg_plan_batch([(1, 1, 0, 3)], num_streams=10, out_elems=10)
    assert e.value.status == xg.XG_EINVAL
    out, groups = xg.xg_plan_batch([], num_streams=10, out_elems=0)
    assert groups == [0]


def test_plan_batch_large_is_balanced_order():
    import numpy as np
    from paper_1108_0486_amd import workloads as W
    n = W.ragged_lengths(4096)
    off = W.csr_offsets(n)
    reqs = [(i, int(n[i]), int(off[i]), 0) for i in range(len(n))]
    out, groups = xg.xg_plan_batch(reqs, num_streams=4096, out_elems=int(off[-1]))
    lens = [out[i].n for i in range(len(reqs))]
    assert lens == sorted(lens, reverse=True)
    assert sorted((out[i].stream for i in range(len(reqs)))) == list(range(4096))
    assert len(groups) == 4097
    del np


@pytest.mark.parametrize("count,n", [(1, 1), (3, 64), (5, 65), (7, 1000), (64, 4096 + 13), (2, 0)])
def test_fill_index_is_a_permutation(count, n):
    import numpy as np
    idx = xg.fill_index(count, n)
    assert idx.shape == (count, n)
    assert np.array_equal(np.sort(idx.ravel()), np.arange(count * n))
    # a 64-word chunk of one stream stays contiguous; chunk c of stream k at (c count + k) 64
    for k in range(count):
        for c in range(n // 64):
            assert idx[k, 64 * c] == (c * count + k) * 64
            assert (np.diff(idx[k, 64 * c:64 * c + 64]) == 1).all()


def test_server_abi_without_gpu():
    L = xg.lib()
    assert xg.xg_server_device_bytes(4, 1024) > 4 * 1024 * 32
    assert xg.xg_server_device_bytes(0, 1024) == 0
    assert xg.xg_server_device_bytes(9, 1024) == 0
    assert L.xg_server_submit(None, 0, 0, 1, 0) == xg.XG_EINVAL
    k = ctypes.c_uint32()
    assert L.xg_server_poll(None, None, 0, ctypes.byref(k)) == xg.XG_EINVAL
    assert L.xg_server_release(None, 0) == xg.XG_EINVAL
    assert L.xg_server_outstanding(None) == 0
    srv = ctypes.c_void_p()
    assert L.xg_server_create(ctypes.byref(srv), None, None, None, 0, None, 0) == xg.XG_EINVAL
    L.xg_server_destroy(None)


@pytest.mark.parametrize("J", [0, 1, 64, 4095, 4096, 10**5, 2**32 + 5, 2**63 + 12345, 2**64 - 1])
def test_jump_polynomial_matches_oracle(J):
    """The library's own z^J mod P (host, no GPU) equals the oracle's."""
    from oracle import oracle as O
    P = O.charpoly(O.PAPER)
    assert xg.xg_jump_polynomial(J) == O.z_pow_mod(J, P)


def test_family_entry_points_without_gpu():
    """Family state sizes, the family of a NULL handle, and argument errors
    that are caught before any device call."""
    assert xg.xg_family_state_bytes(xg.XG_FAMILY_R128_W32, 3) == 3 * 528
    assert xg.xg_family_state_bytes(xg.XG_FAMILY_R64_W32, 3) == 3 * 272
    assert xg.xg_family_state_bytes(xg.XG_FAMILY_R64_W64, 3) == 3 * 528
    assert xg.xg_family_state_bytes(7, 3) == 0
    assert xg.xg_family_state_bytes(xg.XG_FAMILY_R64_W32, 2**33) == 0
    L = xg.lib()
    assert L.xg_family(None) == 0xFFFFFFFF
    ctx = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(4096 + 16)
    aligned = (ctypes.addressof(buf) + 15) // 16 * 16
    assert L.xg_init_family(ctypes.byref(ctx), 7, aligned, 4096, 1, 0, None) == xg.XG_EINVAL
    assert L.xg_attach_family(ctypes.byref(ctx), 7, aligned, 4096, 1) == xg.XG_EINVAL
    assert L.xg_attach_family(ctypes.byref(ctx), xg.XG_FAMILY_R64_W32, aligned, 271, 1) == xg.XG_ERANGE
    assert L.xg_attach_family(ctypes.byref(ctx), xg.XG_FAMILY_R64_W64, aligned, 528 * 8 - 1, 8) == xg.XG_ERANGE
    assert L.xg_attach_family(None, xg.XG_FAMILY_R64_W32, aligned, 4096, 1) == xg.XG_EINVAL
    for f in (L.xg_generate_u64, L.xg_generate_f64, L.xg_fill_u64, L.xg_fill_f64):
        assert f(None, 0, 1, 16, None, None) == xg.XG_EINVAL


def test_fill_index_chunk32_is_a_permutation():
    import numpy as np
    for count, n in [(1, 1), (3, 31), (5, 32), (7, 33), (4, 1000)]:
        idx = xg.fill_index(count, n, chunk=32)
        assert np.array_equal(np.sort(idx.ravel()), np.arange(count * n))
        full = n // 32
        if full:   # chunk c of stream k is contiguous at (c count + k) 32
            assert idx[count - 1, 32 * full - 1] == (full - 1) * 32 * count + (count - 1) * 32 + 31


def test_fill_value_arguments_without_gpu():
    L = xg.lib()
    assert L.xg_fill_value(None, 0, 7, None) == xg.XG_OK          # nothing to do
    assert L.xg_fill_value(None, 16, 7, None) == xg.XG_EINVAL
    buf = ctypes.create_string_buffer(64 + 16)
    aligned = (ctypes.addressof(buf) + 15) // 16 * 16
    assert L.xg_fill_value(aligned + 4, 4, 7, None) == xg.XG_EALIGN
    assert L.xg_fill_value(aligned, 2**63, 7, None) == xg.XG_ERANGE


# ---- tuning cache (host only) -------------------------------------------------

def _fresh_cache():
    xg.xg_tune_cache_clear()
    assert xg.xg_tune_cache_size() == 0


def test_tune_cache_round_trip(tmp_path):
    _fresh_cache()
    xg.xg_tune_cache_put("gfx950", 256, xg.XG_FAMILY_R128_W32, "ragged65536/u32", (1, 1, 8, 1), 7.31)
    xg.xg_tune_cache_put("gfx950", 256, xg.XG_FAMILY_R64_W32, "ragged65536/u32", (8, 2, 1, 0), 7.26)
    xg.xg_tune_cache_put("gfx950", 304, xg.XG_FAMILY_R128_W32, "ragged65536/u32", (4, 8, 4, 4), 9.0)
    xg.xg_tune_cache_put("gfx950", 256, xg.XG_FAMILY_R128_W32, "serve/mixed", (2, 4, 16, 1))
    assert xg.xg_tune_cache_size() == 4
    # the key has four parts: each one tells entries apart
    assert xg.xg_tune_cache_get("gfx950", 256, 0, "ragged65536/u32")[0] == (1, 1, 8, 1)
    assert xg.xg_tune_cache_get("gfx950", 256, 1, "ragged65536/u32")[0] == (8, 2, 1, 0)
    assert xg.xg_tune_cache_get("gfx950", 304, 0, "ragged65536/u32")[0] == (4, 8, 4, 4)
    assert xg.xg_tune_cache_get("gfx942", 256, 0, "ragged65536/u32") is None
    assert xg.xg_tune_cache_get("gfx950", 256, 0, "ragged65536/f32") is None
    path = str(tmp_path / "tune.json")
    xg.xg_tune_cache_save(path)
    _fresh_cache()
    xg.xg_tune_cache_load(path)
    assert xg.xg_tune_cache_size() == 4
    shape, ms = xg.xg_tune_cache_get("gfx950", 256, 0, "ragged65536/u32")
    assert shape == (1, 1, 8, 1) and abs(ms - 7.31) < 1e-4
    assert xg.xg_tune_cache_get("gfx950", 256, 0, "serve/mixed")[1] == -1.0  # stored without a time
    # loading merges: a later file replaces equal keys and keeps the others
    _fresh_cache()
    xg.xg_tune_cache_put("gfx950", 256, 0, "ragged65536/u32", (16, 8, 2, 4), 1.0)
    xg.xg_tune_cache_put("gfx950", 256, 0, "only-here", (1, 2, 1, 1), 2.0)
    xg.xg_tune_cache_load(path)
    assert xg.xg_tune_cache_size() == 5
    assert xg.xg_tune_cache_get("gfx950", 256, 0, "ragged65536/u32")[0] == (1, 1, 8, 1)
    assert xg.xg_tune_cache_get("gfx950", 256, 0, "only-here")[0] == (1, 2, 1, 1)
    _fresh_cache()


def test_tune_cache_rejects_bad_arguments_and_files(tmp_path):
    _fresh_cache()
    bad_shapes = [(3, 1, 1, 1), (1, 3, 1, 1), (1, 1, 0, 1), (1, 1, 33, 1), (1, 2, 1, 4), (1, 1, 1, 2)]
    for t in bad_shapes:
        with pytest.raises(xg.XgError) as e:
            xg.xg_tune_cache_put("gfx950", 256, 0, "k", t)
        assert e.value.status == xg.XG_EINVAL
    for arch, cus, fam, key in [("", 256, 0, "k"), ("gfx950", 0, 0, "k"), ("gfx950", 256, 3, "k"),
                                ("gfx950", 256, 0, ""), ("gfx950", 256, 0, 'a"b'), ("gfx950", 256, 0, "a\\b"),
                                ("gfx950", 256, 0, "x" * 257), ("gfx950", 256, 0, "tab\tkey")]:
        with pytest.raises(xg.XgError) as e:
            xg.xg_tune_cache_put(arch, cus, fam, key, (1, 1, 1, 1))
        assert e.value.status == xg.XG_EINVAL
    xg.xg_tune_cache_put("gfx950", 256, 0, "x" * 256, (1, 1, 1, 1))
    assert xg.xg_tune_cache_size() == 1
    # malformed files are refused whole
    good = ('{"xg_tune_cache": 1, "entries": [{"arch": "gfx950", "key": "k", "cus": 256, "family": 0, '
            '"waves_per_block": 1, "unroll": 1, "blocks_per_cu": 8, "store_words": 1, "ms": 7.0}]}')
    broken = [
        "", "{", "[]", good.replace('"xg_tune_cache": 1', '"xg_tune_cache": 2'),
        good.replace('"unroll": 1', '"unroll": 3'), good.replace('"cus": 256', '"cus": -1'),
        good.replace('"cus": 256', '"cus": 2.5'), good.replace('"arch": "gfx950", ', ''),
        good.replace('"key": "k"', '"key": 5'), good[:-1], good + "x",
        good.replace('"family": 0', '"family": 7'), good.replace('"key": "k"', '"key": "\\u00e9"'),
    ]
    path = str(tmp_path / "bad.json")
    for text in broken:
        with open(path, "w") as f:
            f.write(text)
        with pytest.raises(xg.XgError) as e:
            xg.xg_tune_cache_load(path)
        assert e.value.status == xg.XG_EINVAL, text
        assert xg.xg_tune_cache_size() == 1  # nothing merged
    with open(path, "w") as f:
        f.write(good)
    xg.xg_tune_cache_load(path)
    assert xg.xg_tune_cache_get("gfx950", 256, 0, "k")[0] == (1, 1, 8, 1)
    with pytest.raises(xg.XgError):
        xg.xg_tune_cache_load(str(tmp_path / "missing.json"))
    with pytest.raises(xg.XgError):
        xg.xg_tune_cache_save(str(tmp_path / "no-such-dir" / "t.json"))
    _fresh_cache()


def test_tune_cache_env_file_loaded_before_first_lookup(tmp_path):
    """XG_TUNE_CACHE names a file merged in before the first lookup (in a fresh process)."""
    import sys
    path = tmp_path / "env.json"
    path.write_text('{"xg_tune_cache": 1, "entries": [{"arch": "gfx950", "key": "env", "cus": 8, "family": 1, '
                    '"waves_per_block": 2, "unroll": 4, "blocks_per_cu": 3, "store_words": 0, "ms": 1.5}]}')
    code = ("from paper_1108_0486_amd import xg; r = xg.xg_tune_cache_get('gfx950', 8, 1, 'env'); "
            "print(r[0], xg.xg_tune_cache_size())")
    import os
    env = dict(os.environ, XG_TUNE_CACHE=str(path))
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=root,
                         check=True).stdout
    assert out.split() == ["(2,", "4,", "3,", "0)", "1"]


def test_jump_polynomial_cache_keeps_results():
    """The library keeps its 16 most recent jump polynomials: 24 distinct J
    (more than it keeps, for two members), then the same J again in another
    order (hits and recomputations after eviction) all equal the oracle's."""
    from oracle import oracle as O
    P = {xg.XG_FAMILY_R128_W32: O.charpoly(O.PAPER), xg.XG_FAMILY_R64_W64: O.charpoly(O.W64)}
    Js = [(2**40 + 977 * k) for k in range(24)]
    want = {(f, J): O.z_pow_mod(J, P[f]) for f in P for J in Js[::5]}
    first = {(f, J): xg.xg_family_jump_polynomial(f, J) for J in Js for f in P}
    for f, J in reversed(list(first)):
        assert xg.xg_family_jump_polynomial(f, J) == first[(f, J)], (f, J)
    for key, g in want.items():
        assert first[key] == g, key
