"""Adjoint scatter of the pair readout: kernel vs oracle, FD, and a descent loop."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_util import device, u32
from paper_2301_10838_amd import fields

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


@pytest.fixture(scope="module")
def dev():
    return device()


def _topo_loss_torch(births, deaths, tau):
    pers = deaths - births
    return torch.where(pers < tau, pers * pers, torch.zeros_like(pers)).sum()


def test_hand_example_gradient(dev):
    import paper_2301_10838_amd.mt as mt

    with open(GOLDEN) as fh:
        ex = {e["name"]: e for e in json.load(fh)["examples"]}["E5_cross"]
    f = np.array(ex["values"], np.float32)
    plan = mt.BatchPlan([f.shape], dev)
    for item in ex["loss"]:
        x = torch.from_numpy(f).to(dev).reshape(-1).requires_grad_(True)
        b, d = mt.MergeTreePairs.apply(x, plan)
        L = _topo_loss_torch(b, d, item["tau"])
        L.backward()
        assert float(L) == item["L"]
        want = np.zeros(9)
        for k, v in item["grad"].items():
            want[int(k)] = v
        assert np.array_equal(x.grad.cpu().numpy().astype(np.float64), want)


def test_scatter_matches_oracle(dev):
    import paper_2301_10838_amd.mt as mt

    fs = [fields.lognormal_grf((30, 31, 17), 301), fields.uniform((90, 70), 302), fields.bumps((40,), 303)]
    plan = mt.mt_batch_build([torch.from_numpy(f).to(dev) for f in fs])
    P = plan.sync_status()
    rng = np.random.default_rng(0)
    gb = rng.standard_normal(P).astype(np.float32)
    gd = rng.standard_normal(P).astype(np.float32)
    for accumulate in (False, True):
        base = torch.full((plan.n_total,), 0.5, device=dev)
        g = plan.backward(torch.from_numpy(gb).to(dev), torch.from_numpy(gd).to(dev), grad_field=base,
                          accumulate=accumulate).cpu().numpy()
        offs = plan.pair_offsets.cpu().numpy()
        b_all, d_all = u32(plan.birth)[:P], u32(plan.death)[:P]
        for i, f in enumerate(fs):
            a0, a1 = plan.vertex_offsets[i], plan.vertex_offsets[i + 1]
            p0, p1 = offs[i], offs[i + 1]
            ref = oracle.pairs_scatter(f.size, b_all[p0:p1], d_all[p0:p1], gb[p0:p1].astype(np.float64),
                                       gd[p0:p1].astype(np.float64))
            if accumulate:
                ref = ref + 0.5
            assert np.allclose(g[a0:a1], ref, rtol=1e-6, atol=1e-6), i


def test_gradient_vs_fp64_finite_differences(dev):
    """GPU FP32 gradient of the simplification loss against FP64 central
    differences of the oracle loss on generic 16^3 fields."""
    import paper_2301_10838_amd.mt as mt

    tau, h = 0.05, 1e-7
    checked = 0
    for i in range(8):
        f32 = fields.generic_fd_field((16, 16, 16), 6000 + i)
        f64 = f32.astype(np.float64)
        flat = f64.ravel()
        T = oracle.merge_tree(f64)
        rb, rd, rbv, rdv, _ = oracle.pairs(f64, T)
        pers = rdv - rbv
        pers32 = (rdv.astype(np.float32) - rbv.astype(np.float32)).astype(np.float64)
        # genericity: distinct values and no threshold decision near tau in either precision
        if np.unique(flat).size != flat.size or np.any(np.abs(pers - tau) < 1e-5) or np.any(
                np.abs(pers32 - tau) < 1e-5):
            continue
        plan = mt.BatchPlan([f32.shape], dev)
        x = torch.from_numpy(f32).to(dev).reshape(-1).requires_grad_(True)
        b, d = mt.MergeTreePairs.apply(x, plan)
        _topo_loss_torch(b, d, tau).backward()
        g = x.grad.cpu().numpy().astype(np.float64)
        support = np.unique(np.concatenate([rb[pers < tau], rd[pers < tau]])).astype(np.int64)
        rng = np.random.default_rng(i)
        probe = np.unique(np.concatenate([support, rng.choice(flat.size, 64, replace=False)]))
        gfd = np.zeros(flat.size)
        for j in probe:
            fp = flat.copy(); fp[j] += h
            fm = flat.copy(); fm[j] -= h
            Lp, _ = oracle.topo_loss(fp.reshape(f64.shape), tau, want_grad=False)
            Lm, _ = oracle.topo_loss(fm.reshape(f64.shape), tau, want_grad=False)
            gfd[j] = (Lp - Lm) / (2 * h)
        scale = np.max(np.abs(gfd))
        assert scale > 0
        assert np.max(np.abs(g[probe] - gfd[probe])) <= 1e-4 * scale, i
        assert set(np.nonzero(g)[0].tolist()) == set(np.nonzero(np.abs(gfd) > 1e-6 * scale)[0].tolist())
        # and against the oracle's own FP64 gradient everywhere
        _, gref = oracle.topo_loss(f64, tau)
        assert np.max(np.abs(g - gref.ravel())) <= 1e-4 * np.max(np.abs(gref))
        checked += 1
    assert checked >= 4


def test_descent_loop_reduces_loss(dev):
    """Topological simplification by gradient descent on a small batch."""
    import paper_2301_10838_amd.mt as mt

    fs = [fields.bumps((32, 32, 32), 5000 + i) for i in range(4)]
    plan = mt.BatchPlan([f.shape for f in fs], dev)
    flat = torch.cat([torch.from_numpy(f).to(dev).reshape(-1) for f in fs])
    losses = []
    for _ in range(15):
        x = flat.clone().requires_grad_(True)
        b, d = mt.MergeTreePairs.apply(x, plan)
        L = _topo_loss_torch(b, d, 0.05)
        L.backward()
        losses.append(float(L))
        with torch.no_grad():
            flat -= 0.1 * x.grad
    assert losses[-1] < 0.5 * losses[0], losses


def test_stream_handle_matches_torch():
    """The binding's raw stream handle is torch's current stream, also on a
    side stream (the backward enqueues on whatever stream autograd made current)."""
    import paper_2301_10838_amd.mt as mt

    dev = device()
    assert mt._stream_ptr(dev) == torch.cuda.current_stream(dev).cuda_stream
    s = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(s):
        assert mt._stream_ptr(dev) == s.cuda_stream
    assert mt._stream_ptr(torch.device("cuda")) == torch.cuda.current_stream().cuda_stream
