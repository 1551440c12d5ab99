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
    assert L.xg_generate_batch(None, None, 0, None, 0, None, 0, None, None, None) == xg.XG_EINVAL
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
