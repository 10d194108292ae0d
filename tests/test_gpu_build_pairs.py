"""mt_build_pairs: tree and pairs in one call, the readout using the chunk
pair counts the build leaves.  Checked against the oracle, and against the
separate mt_build_tree + mt_persistence_pairs calls, on every kind of chunk
end (whole chunks, a last chunk ending inside a 64-vertex ballot word, fields
smaller than one word), on the checkerboard (every other vertex a pair birth:
several dense-lane passes per wave, and more pairs than the build stages per
chunk, so the readout takes those chunks from T), on a field mixing such
chunks with staged ones, on signed zeros (staged pair values rebuilt from
order keys must keep the sign of zero) and on a workspace reused across
shapes."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_matches_oracle, device, u32
from paper_2301_10838_amd import fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def fused(f: np.ndarray, dev, kind="merge", workspace=None):
    import paper_2301_10838_amd.mt as mt

    ft = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    T, b, d, bv, dv, nroots = mt.mt_build_pairs(ft, kind=kind, workspace=workspace)
    torch.cuda.synchronize()
    return u32(T).reshape(-1, 2), (u32(b), u32(d), bv.cpu().numpy(), dv.cpu().numpy(), nroots)


def separate(f: np.ndarray, dev, kind="merge"):
    import paper_2301_10838_amd.mt as mt

    ft = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    T = mt.mt_build(ft, workspace=ws, kind=kind)
    b, d, bv, dv, nroots = mt.mt_persistence_pairs(ft, T, workspace=ws)
    torch.cuda.synchronize()
    return u32(T).reshape(-1, 2), (u32(b), u32(d), bv.cpu().numpy(), dv.cpu().numpy(), nroots)


def same(a, b):
    Ta, (ba, da, bva, dva, ra) = a
    Tb, (bb, db, bvb, dvb, rb) = b
    assert np.array_equal(Ta, Tb)
    assert np.array_equal(ba, bb) and np.array_equal(da, db)
    assert np.array_equal(bva.view(np.uint32), bvb.view(np.uint32))
    assert np.array_equal(dva.view(np.uint32), dvb.view(np.uint32))
    assert ra == rb


CASES = [
    ("one_vertex", lambda: np.array([1.5], np.float32)),
    ("under_one_word", lambda: fields.uniform((37,), 90)),
    ("one_chunk_ragged_word", lambda: fields.uniform((4096 + 37,), 91)),
    ("whole_chunks", lambda: fields.uniform((64, 64, 64), 92)),
    ("ragged3d", lambda: fields.uniform((37, 29, 45), 93)),
    ("ties", lambda: np.random.default_rng(94).integers(0, 3, (33, 31, 29)).astype(np.float32)),
    ("grf2d", lambda: fields.lognormal_grf((300, 257), 95)),
    ("grf96", lambda: fields.lognormal_grf((96, 96, 96), 96)),
    ("checkerboard", lambda: np.indices((24, 24, 24)).sum(axis=0).astype(np.float32) % 2),
    ("half_checkerboard", lambda: _half_checkerboard()),
    ("signed_zeros", lambda: _signed_zeros()),
]


def _half_checkerboard():
    """z < 20: a checkerboard (every other vertex a pair birth: the chunk's
    staged lists overflow and the readout takes those chunks from T); above:
    a log-normal field (chunks read from the staged lists)."""
    f = fields.lognormal_grf((40, 64, 64), 102)
    f[:20] = (np.indices((20, 64, 64)).sum(axis=0) % 2).astype(np.float32) * 100.0
    return f


def _signed_zeros():
    """Values around zero with many exact +0.0 and -0.0 (equal in the order,
    told apart by id): pair values must still be bit copies, sign of zero
    included."""
    rng = np.random.default_rng(103)
    f = fields.lognormal_grf((33, 35, 37), 103) - 1.0
    z = rng.random(f.shape)
    f[z < 0.15] = 0.0
    f[(z >= 0.15) & (z < 0.3)] = -0.0
    return f.astype(np.float32)


@pytest.mark.parametrize("name,maker", CASES)
def test_build_pairs_matches_oracle(dev, name, maker):
    f = maker()
    print("case build_pairs", name, f.shape, flush=True)
    T, prs = fused(f, dev)
    assert_matches_oracle(f, T, prs, name)


@pytest.mark.parametrize("kind", ["merge", "split"])
@pytest.mark.parametrize("name", ["grf", "signed_zeros", "half_checkerboard"])
def test_build_pairs_equals_separate_calls(dev, kind, name):
    f = {"grf": lambda: fields.lognormal_grf((70, 66, 61), 97), "signed_zeros": _signed_zeros,
         "half_checkerboard": _half_checkerboard}[name]()
    print("case build_pairs vs separate", name, kind, flush=True)
    same(fused(f, dev, kind), separate(f, dev, kind))


def test_workspace_reused_across_shapes(dev):
    """Chunk counts left by a larger field's build are never read for a smaller one."""
    import paper_2301_10838_amd.mt as mt

    big = fields.uniform((80, 80, 80), 98)
    ws = mt.alloc_workspace(mt.workspace_bytes(big.shape), dev)
    for f in (big, fields.uniform((51, 47, 3), 99), fields.uniform((4096 * 3 + 5,), 100), big[:17, :, :].copy()):
        print("case reuse", f.shape, flush=True)
        T, prs = fused(f, dev, workspace=ws)
        assert_matches_oracle(f, T, prs, f"reuse {f.shape}")


def test_build_pairs_capacity_and_nan(dev):
    import paper_2301_10838_amd.mt as mt

    f = fields.uniform((30, 30, 30), 101)
    ft = torch.from_numpy(f).to(dev)
    rb, rd, _, _, _ = oracle.pairs(f, oracle.merge_tree(f))
    cap = 100
    with pytest.raises(mt.MTError) as e:
        mt.mt_build_pairs(ft, capacity=cap)
    assert e.value.status == -4
    # the first `capacity` pairs are still written, and the count is the full one
    lib = mt.load_library()
    N = f.size
    T = torch.empty((N, 2), dtype=torch.int32, device=dev)
    birth = torch.empty(cap, dtype=torch.int32, device=dev)
    death = torch.empty(cap, dtype=torch.int32, device=dev)
    bv = torch.empty(cap, dtype=torch.float32, device=dev)
    dv = torch.empty(cap, dtype=torch.float32, device=dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    n = ctypes.c_int64(0)
    rc = lib.mt_build_pairs(ft.data_ptr(), 30, 30, 30, 0, T.data_ptr(), birth.data_ptr(), death.data_ptr(),
                            bv.data_ptr(), dv.data_ptr(), cap, ctypes.byref(n), None, ws.data_ptr(), ws.numel(),
                            torch.cuda.current_stream(dev).cuda_stream)
    assert rc == -4 and n.value == rb.size
    assert np.array_equal(u32(birth), rb[:cap]) and np.array_equal(u32(death), rd[:cap])
    g = f.copy()
    g[5, 6, 7] = np.nan
    with pytest.raises(mt.MTError) as e:
        mt.mt_build_pairs(torch.from_numpy(g).to(dev))
    assert e.value.status == -3


def test_build_pairs_grf512(dev):
    """Full-size 512^3 log-normal field: the fused call equals the separate calls."""
    f = fields.workload("grf512")[0]
    print("case build_pairs grf512", flush=True)
    same(fused(f, dev), separate(f, dev))
