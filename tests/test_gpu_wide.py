"""Ids beyond the signed 32-bit range: the 64-bit output variant
(mt_build_pairs64) against the oracle's 64-bit ids on small fields, its
equality with the 32-bit output, and one field of more than 2^31 vertices
(1300^3 = 2.197 G) built on the GPU and checked by the properties that fix
the tree plus sampled triplets computed one by one from the definition.

The full sweep of the oracle does not run at 1300^3 (it would need tens of
GB of host memory and many minutes of one core), so that size is checked by:
- the pair count: #pairs = #minima - #components (one component), with the
  minima counted by an independent neighbour test on the device;
- births in ascending id, each a minimum whose triplet names its death vertex,
  each death vertex no minimum, and death above birth in the order;
- every regular vertex pointing at a minimum below it;
- a sample of triplets (vertices drawn from the lowest values, where the
  components are small) recomputed by the oracle's flood from each vertex.
"""
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


def u64(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("name,maker", [
    ("grf_ragged", lambda: fields.lognormal_grf((37, 41, 45), 51)),
    ("ties", lambda: np.random.default_rng(52).integers(0, 3, (30, 17, 33)).astype(np.float32)),
    ("grf2d", lambda: fields.lognormal_grf((333, 301), 53)),
    ("line", lambda: fields.uniform((7001,), 54)),
    ("one", lambda: np.zeros((1,), np.float32)),
])
def test_wide_output_matches_oracle(dev, name, maker):
    import paper_2301_10838_amd.mt as mt

    f = maker()
    print("case", name, f.shape, flush=True)
    ft = torch.from_numpy(f).to(dev)
    T, b, d, bv, dv, nroots = mt.mt_build_pairs64(ft)
    torch.cuda.synchronize()
    assert T.dtype == torch.int64 and b.dtype == torch.int64
    T_ref = oracle.merge_tree(f)
    assert T_ref.dtype == np.uint64
    assert np.array_equal(u64(T).reshape(-1, 2), T_ref), name
    rb, rd, rbv, rdv, rroots = oracle.pairs(f, T_ref)
    assert np.array_equal(u64(b), rb) and np.array_equal(u64(d), rd), name
    flat = f.reshape(-1)
    assert np.array_equal(bv.cpu().numpy().view(np.uint32), flat[rb].view(np.uint32))
    assert np.array_equal(dv.cpu().numpy().view(np.uint32), flat[rd].view(np.uint32))
    assert nroots == rroots


def test_wide_equals_narrow(dev):
    import paper_2301_10838_amd.mt as mt

    f = fields.lognormal_grf((96, 96, 96), 55)
    ft = torch.from_numpy(f).to(dev)
    for kind in ("merge", "split"):
        T32, b32, d32, bv32, dv32, r32 = mt.mt_build_pairs(ft, kind=kind)
        T64, b64, d64, bv64, dv64, r64 = mt.mt_build_pairs64(ft, kind=kind)
        torch.cuda.synchronize()
        assert np.array_equal(u32(T32).reshape(-1, 2).astype(np.uint64), u64(T64).reshape(-1, 2))
        assert np.array_equal(u32(b32).astype(np.uint64), u64(b64))
        assert np.array_equal(u32(d32).astype(np.uint64), u64(d64))
        assert torch.equal(bv32, bv64) and torch.equal(dv32, dv64) and r32 == r64
    # the narrow result against the oracle once more
    T, b, d, bv, dv, r = mt.mt_build_pairs(ft)
    torch.cuda.synchronize()
    assert_matches_oracle(f, u32(T).reshape(-1, 2), (u32(b), u32(d), bv.cpu().numpy(), dv.cpu().numpy(), r), "grf96")


def _minimum_mask(f: torch.Tensor) -> torch.Tensor:
    """u is a minimum iff every axis neighbour comes after it in the (value,
    id) order: a lower-id neighbour must hold a strictly larger value, a
    higher-id neighbour a larger or equal one.  Computed slab by slab."""
    nz, ny, nx = f.shape
    out = torch.empty(f.shape, dtype=torch.bool, device=f.device)
    step = 64
    for z0 in range(0, nz, step):
        z1 = min(nz, z0 + step)
        c = f[z0:z1]
        m = torch.ones(c.shape, dtype=torch.bool, device=f.device)
        m[:, :, 1:] &= f[z0:z1, :, :-1] > c[:, :, 1:]
        m[:, :, :-1] &= f[z0:z1, :, 1:] >= c[:, :, :-1]
        m[:, 1:, :] &= f[z0:z1, :-1, :] > c[:, 1:, :]
        m[:, :-1, :] &= f[z0:z1, 1:, :] >= c[:, :-1, :]
        lo = f[z0 - 1:z1 - 1] if z0 > 0 else None
        if lo is not None:
            m &= lo > c
        else:
            m[1:] &= f[z0:z1 - 1] > c[1:]
        hi = f[z0 + 1:z1 + 1] if z1 < nz else None
        if hi is not None:
            m &= hi >= c
        else:
            m[:-1] &= f[z0 + 1:z1] >= c[:-1]
        out[z0:z1] = m
    return out


def test_minimum_mask_helper(dev):
    """The device neighbour test agrees with the oracle's minima (T[u] = (s, v),
    s != u or v == u) on fields with ties."""
    for f in [fields.lognormal_grf((70, 66, 130), 56),
              np.random.default_rng(57).integers(0, 3, (65, 20, 30)).astype(np.float32)]:
        T = oracle.merge_tree(f)
        ids = np.arange(f.size, dtype=np.uint64)
        want = (T[:, 0] != ids) | (T[:, 1] == ids)
        got = _minimum_mask(torch.from_numpy(f).to(dev)).cpu().numpy().reshape(-1)
        assert np.array_equal(got, want)


def test_more_than_2_31_vertices(dev):
    """1300^3 = 2,197,000,000 vertices (> 2^31): log-normal k^-3 field made on
    the device, tree + pairs with 64-bit ids, checked by properties and by
    sampled triplets from the definition."""
    import paper_2301_10838_amd.mt as mt

    side = 1300
    N = side ** 3
    assert N > 2 ** 31
    print("case 1300^3: generate", flush=True)
    ft = fields.lognormal_grf_device((side,) * 3, 61, dev)
    torch.cuda.synchronize()
    ws = mt.alloc_workspace(mt.workspace_bytes(ft.shape), dev)
    print("case 1300^3: build (64-bit ids)", flush=True)
    cap = N // 10
    T, b, d, bv, dv, nroots = mt.mt_build_pairs64(ft, capacity=cap, workspace=ws)
    torch.cuda.synchronize()
    P = b.numel()
    print("case 1300^3: pairs", P, "roots", nroots, flush=True)
    assert nroots == 1
    is_min = _minimum_mask(ft)
    n_min = int(is_min.sum())
    assert P == n_min - 1
    flat = ft.reshape(-1)
    Tf = T.reshape(-1, 2)
    # births ascending, each a minimum whose triplet names its death
    assert bool((b[1:] > b[:-1]).all())
    assert bool(is_min.reshape(-1)[b].all())
    assert bool((Tf[b, 0] == d).all()) and bool((d != b).all())
    assert not bool(is_min.reshape(-1)[d].any())
    fb, fd = flat[b], flat[d]
    assert bool(((fd > fb) | ((fd == fb) & (d > b))).all())
    assert torch.equal(bv, fb) and torch.equal(dv, fd)
    # regular vertices point at a minimum below them (chunked)
    chunk = 1 << 27
    for a in range(0, N, chunk):
        e = min(N, a + chunk)
        ids = torch.arange(a, e, device=dev, dtype=torch.int64)
        s, v = Tf[a:e, 0], Tf[a:e, 1]
        # a minimum is exactly a vertex with s != u (it dies) or v == u (a root)
        assert torch.equal(is_min.reshape(-1)[a:e], (s != ids) | (v == ids))
        reg = (s == ids) & (v != ids)
        vv = v[reg]
        assert bool(is_min.reshape(-1)[vv].all())
        fu, fv = flat[a:e][reg], flat[vv]
        assert bool(((fv < fu) | ((fv == fu) & (vv < ids[reg]))).all())
    del is_min
    # sampled triplets by the definition (oracle flood), low-valued vertices
    print("case 1300^3: sampled oracle", flush=True)
    g = torch.Generator(device=dev)
    g.manual_seed(62)
    thr = torch.kthvalue(flat[torch.randint(0, N, (1 << 20,), device=dev, generator=g)].cpu(), (1 << 20) // 50).values
    # (torch.nonzero over more than 2^31 elements fails on this stack: chunked)
    thr_d = thr.to(dev)
    low = torch.cat([torch.nonzero(flat[a:min(N, a + chunk)] <= thr_d).reshape(-1) + a for a in range(0, N, chunk)])
    pick = low[torch.randint(0, low.numel(), (20000,), device=dev, generator=g)]
    extra = torch.randint(0, N, (2000,), device=dev, generator=g)
    us = torch.cat([pick, extra])
    want = Tf[us].cpu().numpy().view(np.uint64)
    f_host = ft.cpu().numpy()
    s, v, ok = oracle.triplets_at(f_host, us.cpu().numpy(), max_visit=4096)
    print("case 1300^3: sampled", int(ok.sum()), "of", us.numel(), flush=True)
    assert ok.sum() >= 10000
    assert np.array_equal(s[ok], want[ok, 0]) and np.array_equal(v[ok], want[ok, 1])
