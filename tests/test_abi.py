"""The C-ABI library loads, exports what include/mt.h declares, and rejects bad
arguments on the host (no GPU work is enqueued by these calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mt.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mt_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    import paper_2301_10838_amd.mt as mt

    if not os.path.exists(mt.LIB_PATH):
        from paper_2301_10838_amd import build

        build.build()
    return mt.load_library()


def test_exports_match_header(lib):
    import paper_2301_10838_amd.mt as mt

    names = _declared()
    assert names == sorted(mt.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for code, name in [(0, b"MT_OK"), (-1, b"MT_ERR_INVALID_ARG"), (-3, b"MT_ERR_NAN"), (-8, b"MT_ERR_INTERNAL")]:
        assert lib.mt_status_string(code) == name


def test_workspace_sizes(lib):
    assert lib.mt_workspace_bytes(0, 1, 1) == 0
    assert lib.mt_workspace_bytes(1 << 31, 1, 1) == 0  # one dimension of 2^31
    assert lib.mt_workspace_bytes(4096, 1024, 1024) == 0  # 2^32 vertices
    assert lib.mt_workspace_bytes(65536, 65535, 1) > 0  # 2^32 - 65536 vertices: ids up to 2^32 - 2
    assert lib.mt_workspace_bytes(2048, 1024, 1024) > 0  # 2^31 vertices
    w = lib.mt_workspace_bytes(64, 64, 64)
    assert w >= 4 * 64 ** 3 and w % 256 == 0
    dims = (ctypes.c_int64 * 6)(64, 64, 64, 100, 90, 1)
    wb = lib.mt_batch_workspace_bytes(dims, 2)
    assert wb >= 4 * (64 ** 3 + 9000)
    assert lib.mt_batch_workspace_bytes(dims, 0) == 0


def test_host_argument_checks(lib):
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: checks fail first
    ws = lib.mt_workspace_bytes(8, 8, 8)
    # bad dims
    assert lib.mt_build(fake, 0, 8, 8, fake, fake, ws, None) == -1
    assert lib.mt_build(fake, -3, 8, 8, fake, fake, ws, None) == -1
    # too many vertices for 32-bit ids
    assert lib.mt_build(fake, 1 << 16, 1 << 16, 1, fake, fake, ws, None) == -2
    # the 64-bit output variant wants 16-byte aligned triplets
    n = ctypes.c_int64(0)
    assert lib.mt_build_pairs64(fake, 8, 8, 8, 0, ctypes.c_void_p(0x10008), fake, fake, fake, fake, 10,
                                ctypes.byref(n), None, fake, ws, None) == -1
    assert lib.mt_build_pairs64(fake, 1 << 16, 1 << 16, 1, 0, fake, fake, fake, fake, fake, 10, ctypes.byref(n),
                                None, fake, ws, None) == -2
    # null / misaligned triplets
    assert lib.mt_build(fake, 8, 8, 8, None, fake, ws, None) == -1
    assert lib.mt_build(fake, 8, 8, 8, ctypes.c_void_p(0x10004), fake, ws, None) == -1
    # workspace missing, misaligned or too small
    assert lib.mt_build(fake, 8, 8, 8, fake, None, ws, None) == -6
    assert lib.mt_build(fake, 8, 8, 8, fake, ctypes.c_void_p(0x10010), ws, None) == -6
    assert lib.mt_build(fake, 8, 8, 8, fake, fake, ws - 1, None) == -6
    # pairs: n_pairs required, negative capacity
    n = ctypes.c_int64(0)
    assert lib.mt_persistence_pairs(fake, fake, 8, 8, 8, fake, fake, fake, fake, 10, None, None, fake, ws,
                                    None) == -1
    assert lib.mt_persistence_pairs(fake, fake, 8, 8, 8, fake, fake, fake, fake, -1, ctypes.byref(n), None,
                                    fake, ws, None) == -1
    # fused tree + pairs: kind, n_pairs, capacity, workspace
    assert lib.mt_build_pairs(fake, 8, 8, 8, 2, fake, fake, fake, fake, fake, 10, ctypes.byref(n), None, fake, ws,
                              None) == -1
    assert lib.mt_build_pairs(fake, 8, 8, 8, 0, fake, fake, fake, fake, fake, 10, None, None, fake, ws, None) == -1
    assert lib.mt_build_pairs(fake, 8, 8, 8, 0, fake, fake, fake, fake, fake, -1, ctypes.byref(n), None, fake, ws,
                              None) == -1
    assert lib.mt_build_pairs(fake, 8, 8, 8, 0, fake, None, None, None, None, 10, ctypes.byref(n), None, fake, ws,
                              None) == -1
    assert lib.mt_build_pairs(fake, 8, 8, 8, 1, fake, fake, fake, fake, fake, 10, ctypes.byref(n), None, fake,
                              ws - 1, None) == -6
    # vertex ranks: kind, dims, null ranks, workspace
    rws = lib.mt_rank_workspace_bytes(8, 8, 8)
    assert rws > 16 * 512 and lib.mt_rank_workspace_bytes(0, 8, 8) == 0
    assert lib.mt_rank_workspace_bytes(1 << 16, 1 << 16, 1) == 0
    assert lib.mt_vertex_ranks(fake, 8, 8, 8, 2, fake, fake, rws, None) == -1
    assert lib.mt_vertex_ranks(fake, 8, 0, 8, 0, fake, fake, rws, None) == -1
    assert lib.mt_vertex_ranks(fake, 1 << 16, 1 << 16, 1, 0, fake, fake, rws, None) == -2
    assert lib.mt_vertex_ranks(fake, 8, 8, 8, 0, None, fake, rws, None) == -1
    assert lib.mt_vertex_ranks(fake, 8, 8, 8, 1, fake, fake, rws - 1, None) == -6
    assert lib.mt_vertex_ranks(fake, 8, 8, 8, 1, fake, ctypes.c_void_p(0x10010), rws, None) == -6
    # batch: no fields, bad dims
    dims = (ctypes.c_int64 * 3)(8, 0, 8)
    assert lib.mt_batch_build(fake, dims, 1, fake, fake, fake, fake, fake, 10, fake, fake, 1 << 20, None) == -1
    assert lib.mt_batch_build(fake, dims, 0, fake, fake, fake, fake, fake, 10, fake, fake, 1 << 20, None) == -1
    big = (ctypes.c_int64 * 6)(1 << 16, 1 << 15, 1, 1 << 16, 1 << 15, 1)  # 2^32 vertices in all
    assert lib.mt_batch_build(fake, big, 2, fake, fake, fake, fake, fake, 10, fake, fake, 1 << 20, None) == -2
    # tree kind: only merge (0) and split (1)
    good = (ctypes.c_int64 * 3)(8, 8, 8)
    assert lib.mt_build_tree(fake, 8, 8, 8, 2, fake, fake, ws, None) == -1
    assert lib.mt_build_tree(fake, 8, 8, 8, -1, fake, fake, ws, None) == -1
    assert lib.mt_build_tree(fake, 0, 8, 8, 1, fake, fake, ws, None) == -1
    assert lib.mt_batch_build_tree(fake, good, 1, 7, fake, fake, fake, fake, fake, 10, fake, fake, 1 << 20,
                                   None) == -1
    # backward
    assert lib.mt_pairs_backward(dims, 1, fake, 0, None, None, None, None, fake, 0, None) == -1
    assert lib.mt_sync_status(None, None, None, None) == -6


def test_setter_bounds(lib):
    """Loop bounds: out-of-range settings are refused on the host; the
    defaults are restored by 0 / -1.  (No GPU work is enqueued.)"""
    assert lib.mt_get_max_steps() == 1 << 24
    assert lib.mt_set_max_steps(-1) == -1
    assert lib.mt_set_max_steps(1 << 31) == -1
    assert lib.mt_set_max_steps(5) == 0 and lib.mt_get_max_steps() == 5
    assert lib.mt_set_max_steps(0) == 0 and lib.mt_get_max_steps() == 1 << 24
    assert lib.mt_get_table_probes() == 32
    assert lib.mt_set_table_probes(-2) == -1
    assert lib.mt_set_table_probes(33) == -1
    assert lib.mt_set_table_probes(0) == 0 and lib.mt_get_table_probes() == 0
    assert lib.mt_set_table_probes(-1) == 0 and lib.mt_get_table_probes() == 32
    r, g = ctypes.c_int(-9), ctypes.c_int(-9)
    assert lib.mt_get_schedule(ctypes.byref(r), ctypes.byref(g)) == 0 and (r.value, g.value) == (1, 2048)
    assert lib.mt_set_schedule(2, 0) == -1 and lib.mt_set_schedule(-2, 0) == -1
    assert lib.mt_set_schedule(0, -1) == -1 and lib.mt_set_schedule(0, 65537) == -1
    assert lib.mt_set_schedule(0, 64) == 0
    assert lib.mt_get_schedule(ctypes.byref(r), ctypes.byref(g)) == 0 and (r.value, g.value) == (0, 64)
    assert lib.mt_set_schedule(-1, 0) == 0
    assert lib.mt_get_schedule(ctypes.byref(r), None) == 0 and r.value == 1
    assert lib.mt_get_schedule(None, ctypes.byref(g)) == 0 and g.value == 2048
    assert lib.mt_set_counting(3) == -1 and lib.mt_set_counting(-1) == -1
    assert lib.mt_set_counting(2) == 0 and lib.mt_get_counting() == 2
    assert lib.mt_set_counting(0) == 0 and lib.mt_get_counting() == 0
    assert lib.mt_noalloc_scratch_bytes() == 64 << 20
    assert lib.mt_workspace_reset(None, 4096, None) == -6
    assert lib.mt_workspace_reset(ctypes.c_void_p(0x10010), 4096, None) == -6
    assert lib.mt_workspace_reset(ctypes.c_void_p(0x10000), 64, None) == -6


def test_binding_refuses_cpu_tensors():
    import torch

    import paper_2301_10838_amd.mt as mt

    with pytest.raises(TypeError):
        mt.mt_build(torch.zeros(4, 4))
