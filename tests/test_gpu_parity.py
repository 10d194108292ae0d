"""Bit-exact parity of the HIP path (through the C ABI) with the oracle."""
import json
import os

import numpy as np
import pytest
import torch

import brute
import oracle
from gpu_util import assert_matches_oracle, device, gpu_tree, u32
from paper_2301_10838_amd import fields

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


@pytest.fixture(scope="module")
def dev():
    return device()


def test_hand_examples(dev):
    with open(GOLDEN) as fh:
        exs = json.load(fh)["examples"]
    for ex in exs:
        f = np.array(ex["values"], dtype=np.float32).reshape(ex["shape"])
        if ex["name"] == "E6_signed_zero":
            f = np.array([0.0, -0.0], np.float32)
        print("case", ex["name"], flush=True)
        T, prs = gpu_tree(f, dev)
        assert T.tolist() == ex["T"], ex["name"]
        assert [[int(a), int(b)] for a, b in zip(prs[0], prs[1])] == ex["pairs"], ex["name"]
        assert_matches_oracle(f, T, prs, ex["name"])


TINY = [(1,), (2,), (7,), (1, 1), (2, 1), (1, 5), (3, 7), (5, 1, 4), (1, 1, 9), (4, 3, 2), (3, 3, 3), (2, 9, 33),
        (5, 17, 70), (9, 8, 35)]


@pytest.mark.parametrize("shape", TINY)
def test_tiny_random(dev, shape):
    rng = np.random.default_rng(abs(hash(shape)) % 2**32)
    for trial in range(6):
        if trial % 3 == 0:
            f = rng.integers(0, 3, size=shape).astype(np.float32)
        elif trial % 3 == 1:
            f = rng.random(shape).astype(np.float32)
        else:
            f = (rng.standard_normal(shape) * 100).astype(np.float32)
        print("case", shape, trial, flush=True)
        T, prs = gpu_tree(f, dev)
        assert_matches_oracle(f, T, prs, f"{shape}/{trial}")


def test_special_values(dev):
    f = np.array([[np.inf, 0.0, -0.0, 1.0], [-np.inf, -0.0, 0.0, np.inf], [3.0, -0.0, np.inf, -np.inf]],
                 np.float32)
    T, prs = gpu_tree(f, dev)
    assert np.array_equal(T, brute.brute_triplets(f))
    assert_matches_oracle(f, T, prs, "special")


@pytest.mark.parametrize("shape", [(40,), (6, 7), (5, 6, 7)])
def test_closed_forms(dev, shape):
    n = int(np.prod(shape))
    ramp = np.arange(n, dtype=np.float32).reshape(shape)
    T, prs = gpu_tree(ramp, dev)
    assert prs[0].size == 0 and prs[4] == 1 and np.all(T[1:, 1] == 0)
    assert_matches_oracle(ramp, T, prs, "ramp")
    for f in [ramp[::-1].copy() if len(shape) == 1 else -ramp, np.full(shape, 7.0, np.float32)]:
        T, prs = gpu_tree(f, dev)
        assert_matches_oracle(f, T, prs, "closed")


def test_checkerboard(dev):
    z, y, x = np.indices((33, 17, 40))
    f = ((x + y + z) % 2).astype(np.float32)
    T, prs = gpu_tree(f, dev)
    assert prs[0].size == (f.size + 1) // 2 - 1
    assert_matches_oracle(f, T, prs, "checkerboard")


@pytest.mark.parametrize("name,maker", [
    ("uniform_ragged", lambda: fields.uniform((37, 29, 45), 31)),
    ("ties_ragged", lambda: np.random.default_rng(3).integers(0, 4, (30, 33, 35)).astype(np.float32)),
    ("grf2d", lambda: fields.lognormal_grf((300, 257), 32)),
    ("uniform1d", lambda: fields.uniform((5001,), 33)),
    ("bumps96", lambda: fields.bumps((96, 96, 96), 34)),
    ("grf96", lambda: fields.lognormal_grf((96, 96, 96), 35)),
    ("grf_thin", lambda: fields.lognormal_grf((3, 200, 190), 36)),
])
def test_multi_tile(dev, name, maker):
    f = maker()
    print("case", name, f.shape, flush=True)
    T, prs = gpu_tree(f, dev)
    assert_matches_oracle(f, T, prs, name)


def test_uniform64_workload(dev):
    f = fields.workload("uniform64")[0]
    T, prs = gpu_tree(f, dev)
    assert_matches_oracle(f, T, prs, "uniform64")


def test_bumps256_workload(dev):
    f = fields.workload("bumps256")[0]
    print("case bumps256", flush=True)
    T, prs = gpu_tree(f, dev)
    assert_matches_oracle(f, T, prs, "bumps256")


def test_repeat_runs_identical(dev):
    import paper_2301_10838_amd.mt as mt

    f = fields.lognormal_grf((64, 64, 64), 37)
    ft = torch.from_numpy(f).to(dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    first = u32(mt.mt_build(ft, workspace=ws)).copy()
    for _ in range(20):
        T = mt.mt_build(ft, workspace=ws)
        assert np.array_equal(u32(T), first)
    assert np.array_equal(first.reshape(-1, 2), oracle.merge_tree(f))


def test_grf512_properties(dev):
    """Full-size 512^3 log-normal field: properties that fix the pairing."""
    import paper_2301_10838_amd.mt as mt

    f = fields.workload("grf512")[0]
    print("case grf512", flush=True)
    T, (b, d, bv, dv, nroots) = gpu_tree(f, dev)
    N = f.size
    ids = np.arange(N, dtype=np.uint32)
    s, v = T[:, 0], T[:, 1]
    # independent minimum test on the grid
    nmin = brute.count_minima(f)
    assert nroots == 1
    assert b.size == nmin - 1
    is_min = (s != ids) | (v == ids)
    assert int(is_min.sum()) == nmin
    flat = f.reshape(-1)
    # degree-two vertices point at a minimum that lies below them
    reg = ~is_min
    vv = v[reg]
    assert np.all(is_min[vv])
    fr, fv = flat[reg], flat[vv]
    assert np.all((fv < fr) | ((fv == fr) & (vv < ids[reg])))
    # a dying branch joins a deeper minimum at a saddle above its birth
    fb, fs = flat[b], flat[d]
    assert np.all((fb < fs) | ((fb == fs) & (b < d)))
    assert np.all(~is_min[d])
    assert np.array_equal(bv.view(np.uint32), flat[b].view(np.uint32))
    # the same tree again
    ft = torch.from_numpy(f).to(dev)
    T2 = u32(mt.mt_build(ft)).reshape(-1, 2)
    assert np.array_equal(T2, T)


def test_grf512_exact(dev):
    """Full-size 512^3 log-normal field, the benchmark's own configuration:
    every triplet and every pair against the oracle (about 40 s of one core)."""
    f = fields.workload("grf512")[0]
    print("case grf512 exact: gpu", flush=True)
    T, prs = gpu_tree(f, dev)
    print("case grf512 exact: oracle", flush=True)
    assert_matches_oracle(f, T, prs, "grf512")


def test_nan_reported(dev):
    import paper_2301_10838_amd.mt as mt

    f = fields.uniform((20, 20, 20), 3)
    f[3, 4, 5] = np.nan
    ft = torch.from_numpy(f).to(dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    # checked build: the binding reads the latched status and raises
    with pytest.raises(mt.MTError) as e:
        mt.mt_build(ft, workspace=ws)
    assert e.value.status == -3
    # unchecked build: the status stays latched for the pairs call on the same workspace
    T = mt.mt_build(ft, workspace=ws, check=False)
    with pytest.raises(mt.MTError) as e:
        mt.mt_persistence_pairs(ft, T, workspace=ws)
    assert e.value.status == -3
    # a workspace the build did not use starts clean (the binding resets it)
    ws2 = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    g = torch.from_numpy(fields.uniform((20, 20, 20), 5)).to(dev)
    T2 = mt.mt_build(g, workspace=ws2)
    ws3 = torch.full_like(ws2, 0xFF)  # every status bit set
    mt.workspace_reset(ws3)
    mt.mt_persistence_pairs(g, T2, workspace=ws3)


def test_capacity_reported(dev):
    import ctypes

    import paper_2301_10838_amd.mt as mt

    f = fields.uniform((30, 30, 30), 4)
    ft = torch.from_numpy(f).to(dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    T = mt.mt_build(ft, workspace=ws)
    want = oracle.pairs(f, oracle.merge_tree(f))[0].size
    cap = 100
    birth = torch.empty(cap, dtype=torch.int32, device=dev)
    death = torch.empty(cap, dtype=torch.int32, device=dev)
    bv = torch.empty(cap, dtype=torch.float32, device=dev)
    dv = torch.empty(cap, dtype=torch.float32, device=dev)
    n = ctypes.c_int64(0)
    lib = mt.load_library()
    rc = lib.mt_persistence_pairs(ft.data_ptr(), T.data_ptr(), 30, 30, 30, birth.data_ptr(), death.data_ptr(),
                                  bv.data_ptr(), dv.data_ptr(), cap, ctypes.byref(n), None, ws.data_ptr(),
                                  ws.numel(), torch.cuda.current_stream().cuda_stream)
    assert rc == -4 and n.value == want
    rb = oracle.pairs(f, oracle.merge_tree(f))[0]
    assert np.array_equal(u32(birth), rb[:cap])
