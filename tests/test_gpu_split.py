"""Split tree (superlevel sets, the setting of the paper's experiments, Sec. 4):
the merge tree of -f.  The oracle run on -f is the reference; pair values stay
bit copies of f."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import device, u32
from paper_2301_10838_amd import fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    return device()


def split_on_gpu(f, dev):
    import paper_2301_10838_amd.mt as mt

    ft = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    T = mt.mt_build(ft, workspace=ws, kind="split")
    b, d, bv, dv, nroots = mt.mt_persistence_pairs(ft, T, workspace=ws)
    torch.cuda.synchronize()
    return u32(T).reshape(-1, 2), (u32(b), u32(d), bv.cpu().numpy(), dv.cpu().numpy(), nroots)


def check_split(f, T, prs, what):
    neg = -np.asarray(f, np.float64)
    T_ref = oracle.merge_tree(neg)
    if not np.array_equal(T, T_ref):
        bad = np.nonzero(np.any(T != T_ref, axis=1))[0]
        raise AssertionError(f"{what}: {bad.size} triplets differ, first at u={bad[0]}")
    rb, rd, _, _, rroots = oracle.pairs(neg, T_ref)
    b, d, bv, dv, nroots = prs
    assert np.array_equal(b, rb) and np.array_equal(d, rd), what
    flat = np.asarray(f, np.float32).reshape(-1)
    assert np.array_equal(bv.view(np.uint32), flat[rb].view(np.uint32)), what
    assert np.array_equal(dv.view(np.uint32), flat[rd].view(np.uint32)), what
    assert nroots == rroots, what
    # in the split tree a pair is born at a maximum and dies at a lower saddle
    assert np.all(flat[rb] >= flat[rd]), what


@pytest.mark.parametrize("name,maker", [
    ("grf_ragged", lambda: fields.lognormal_grf((37, 29, 45), 71)),
    ("bumps", lambda: fields.bumps((40, 33, 50), 72)),
    ("grf2d", lambda: fields.lognormal_grf((300, 257), 73)),
    ("uniform1d", lambda: fields.uniform((5001,), 74)),
    ("ties", lambda: np.random.default_rng(75).integers(0, 4, (30, 33, 35)).astype(np.float32)),
    ("checker", lambda: ((np.indices((17, 20, 19)).sum(0)) % 2).astype(np.float32)),
    ("signed_zero_inf", lambda: np.random.default_rng(76).choice(
        np.array([0.0, -0.0, np.inf, -np.inf, 1.0, -1.0], np.float32), (12, 11, 10))),
])
def test_split_matches_oracle_on_negated_field(dev, name, maker):
    f = maker()
    print("case split", name, f.shape, flush=True)
    T, prs = split_on_gpu(f, dev)
    check_split(f, T, prs, name)


def test_split_equals_merge_tree_of_negated_field(dev):
    """The two GPU paths agree bit for bit: split(f) == merge(-f)."""
    import paper_2301_10838_amd.mt as mt

    f = fields.lognormal_grf((64, 64, 64), 77)
    a = u32(mt.mt_build(torch.from_numpy(f).to(dev), kind="split"))
    b = u32(mt.mt_build(torch.from_numpy(-f).to(dev)))
    torch.cuda.synchronize()
    assert np.array_equal(a, b)


def test_split_batch(dev):
    import paper_2301_10838_amd.mt as mt

    fs = [fields.lognormal_grf((23, 31, 19), 78), fields.uniform((90, 70), 79), fields.bumps((600,), 80),
          np.random.default_rng(81).integers(0, 3, (9, 1, 8)).astype(np.float32)]
    plan = mt.mt_batch_build([torch.from_numpy(f).to(dev) for f in fs], kind="split")
    offs = plan.pair_offsets.cpu().numpy()
    T_all = u32(plan.triplets).reshape(-1, 2)
    b_all, d_all = u32(plan.birth), u32(plan.death)
    for i, f in enumerate(fs):
        a, b = plan.vertex_offsets[i], plan.vertex_offsets[i + 1]
        neg = -f.astype(np.float64)
        T_ref = oracle.merge_tree(neg)
        assert np.array_equal(T_all[a:b], T_ref), i
        rb, rd, _, _, _ = oracle.pairs(neg, T_ref)
        assert np.array_equal(b_all[offs[i]:offs[i + 1]], rb) and np.array_equal(d_all[offs[i]:offs[i + 1]], rd), i
