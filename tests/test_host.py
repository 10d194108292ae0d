"""Host-side contract, no GPU needed: the bench's single-GPU rule, the
binding's refusal to run without the built library, and the bench's
algorithmic-byte bookkeeping checked against counts worked out by hand."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr


def test_binding_without_library_raises(tmp_path):
    import paper_2301_10838_amd.mt as mt

    saved_path, saved_lib = mt.LIB_PATH, mt._lib
    try:
        mt._lib = None
        mt.LIB_PATH = str(tmp_path / "missing.so")
        with pytest.raises(RuntimeError):
            mt.load_library()
    finally:
        mt.LIB_PATH, mt._lib = saved_path, saved_lib


def test_face_edges_and_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    import paper_2301_10838_amd.mt as mt

    mt._lib = None
    mt.LIB_PATH = os.path.join(ROOT, "paper_2301_10838_amd", "libmt.so")
    if not os.path.exists(mt.LIB_PATH):
        pytest.skip("library not built")
    saved = mt.get_tile_shape(0)
    try:
        sh = {(s["tx"], s["ty"], s["tz"]): s["id"] for s in mt.tile_shapes() if s["dims_class"] == 0}
        mt.set_tile_shape(0, sh[(16, 16, 16)])
        # 512^3 in 16^3 tiles: 31 interior boundaries per axis, each crossed by 512^2 edges
        assert bench.face_edges((512, 512, 512), mt) == 3 * 31 * 512 * 512
        # a 2-D field has no z faces; 1-D has only x boundaries (default 2-D / 1-D shapes)
        assert bench.face_edges((40,), mt) == 0  # 40 < any 1-D tile: no interior boundary
    finally:
        mt.set_tile_shape(0, saved)
    N, P, M, Q, F = 1000, 30, 100, 50, 400
    assert bench.compulsory_bytes(N, P) == 12 * N + 16 * P
    assert bench.model_bytes("k_local", N, P, M) == 8 * N + 24 * M
    assert bench.model_bytes("k_repair_reg", N, P, M) == 16 * N
    assert bench.model_bytes("k_merge_q", N, P, M, Q) == 16 * Q + 16 * M
    assert bench.model_bytes("k_cross", N, P, M, Q, F) == 16 * F + 16 * Q
    assert bench.model_bytes("k_pairs_write", N, P, M) == 32 * P + N // 64
