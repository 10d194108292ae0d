"""Adversarial inputs at multi-tile scale, the table-free paths of the build,
and the step cap, all through the C ABI and bit-exact against the oracle.

- Deep chains: a monotone path snaking through every tile.
- The most minima a grid can have (tilted checkerboard) and a lattice whose
  basins touch so many others that the in-tile pair table fills up.
- Half the domain on one exact plateau next to coarse noise (the sudden jump
  in sublevel volume discussed for the Richtmyer-Meshkov data, Sec. 4), with
  and without tiny noise on the plateau; nested exact-tie plateaus.
- The LDS pair tables (lowest edge per pair of basins, in a tile and across a
  tile face) limited to 0, 1, 2 or 4 probes, so that the overflow list and
  the direct merges inside the tile, and the as-is queueing across tiles, carry
  many or all edges.
- The step cap set to 1 from the host: every kernel leaves its bounded loops
  and the call reports MT_ERR_LIVELOCK; with the cap restored the same
  process gets the oracle's tree.
"""
import numpy as np
import pytest
import torch

from gpu_util import assert_matches_oracle, device, gpu_tree, u32
from paper_2301_10838_amd import fields

pytestmark = pytest.mark.gpu

ADVERSARIAL = [
    ("serpentine128", lambda: fields.serpentine((128, 128, 128), 11)),
    ("serpentine128_desc", lambda: fields.serpentine((128, 128, 128), 12, descending=True)),
    ("serpentine2d", lambda: fields.serpentine((1024, 1000), 13)),
    ("serpentine1d", lambda: fields.serpentine((200001,), 14)),
    ("tilted_checkerboard128", lambda: fields.tilted_checkerboard((128, 128, 128), 15)),
    ("parity_lattice130", lambda: fields.parity_lattice((130, 129, 131))),
    ("plateau_jump128", lambda: fields.plateau_jump((128, 128, 128), 16)),
    ("plateau_jump128_noise", lambda: fields.plateau_jump((128, 128, 128), 17, noise=1e-6)),
    ("nested_plateaus128", lambda: fields.nested_plateaus((128, 128, 128), 18)),
    ("nested_plateaus2d", lambda: fields.nested_plateaus((700, 900), 19, width=9)),
]


@pytest.fixture(scope="module")
def dev():
    return device()


@pytest.fixture
def restore_config():
    import paper_2301_10838_amd.mt as mt

    yield
    mt.set_table_probes(-1)
    mt.set_max_steps(0)


@pytest.mark.parametrize("name,maker", ADVERSARIAL, ids=[a[0] for a in ADVERSARIAL])
def test_adversarial(dev, name, maker):
    f = maker()
    print("case", name, f.shape, flush=True)
    T, prs = gpu_tree(f, dev)
    assert_matches_oracle(f, T, prs, name)


PROBE_CASES = [
    ("grf96", lambda: fields.lognormal_grf((96, 96, 96), 21)),
    ("uniform_ragged", lambda: fields.uniform((70, 45, 83), 22)),
    ("parity_lattice", lambda: fields.parity_lattice((66, 64, 70))),
    ("ties_2d", lambda: np.random.default_rng(23).integers(0, 4, (300, 333)).astype(np.float32)),
    ("serpentine", lambda: fields.serpentine((64, 66, 70), 24)),
]


@pytest.mark.parametrize("probes", [0, 1, 2, 4])
@pytest.mark.parametrize("name,maker", PROBE_CASES, ids=[a[0] for a in PROBE_CASES])
def test_table_fallbacks(dev, restore_config, name, maker, probes):
    import paper_2301_10838_amd.mt as mt

    f = maker()
    mt.set_table_probes(probes)
    assert mt.get_table_probes() == probes
    print("case", name, f.shape, "probes", probes, flush=True)
    T, prs = gpu_tree(f, dev)
    assert_matches_oracle(f, T, prs, f"{name} probes={probes}")


def test_table_fallbacks_batch(dev, restore_config):
    """The batch graph under a probe limit (the limit is part of the graph's
    cache key, so the default graph and the limited one are both replayed)."""
    import oracle
    import paper_2301_10838_amd.mt as mt

    fs = [fields.lognormal_grf((40, 50, 37), 25), fields.parity_lattice((30, 34, 33)),
          fields.lognormal_grf((300, 280), 26)]
    plan = mt.BatchPlan([f.shape for f in fs], dev)
    plan.load([torch.from_numpy(f).to(dev) for f in fs])
    results = []
    for probes in (-1, 0, 1, -1):
        mt.set_table_probes(probes)
        plan.launch()
        plan.sync_status()
        results.append(u32(plan.triplets).reshape(-1, 2).copy())
    for r in results[1:]:
        assert np.array_equal(r, results[0])
    for i, f in enumerate(fs):
        a, b = plan.vertex_offsets[i], plan.vertex_offsets[i + 1]
        assert np.array_equal(results[0][a:b], oracle.merge_tree(f)), f"field {i}"


def test_step_cap_reports_livelock(dev, restore_config):
    import paper_2301_10838_amd.mt as mt

    f = fields.lognormal_grf((64, 64, 64), 27)
    ft = torch.from_numpy(f).to(dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    assert mt.get_max_steps() == 1 << 24
    mt.set_max_steps(1)
    assert mt.get_max_steps() == 1
    print("case step cap 1: single field", flush=True)
    with pytest.raises(mt.MTError) as e:
        mt.mt_build(ft, workspace=ws)
    assert e.value.status == -5
    # the fused call reports it too
    with pytest.raises(mt.MTError) as e:
        mt.mt_build_pairs(ft, workspace=ws)
    assert e.value.status == -5
    # and the batch graph, through its status word
    print("case step cap 1: batch", flush=True)
    plan = mt.BatchPlan([f.shape, (200, 210)], dev)
    plan.load([ft, torch.from_numpy(fields.lognormal_grf((200, 210), 28)).to(dev)])
    plan.launch()
    with pytest.raises(mt.MTError) as e:
        plan.sync_status()
    assert e.value.status == -5
    # restored: the oracle's tree, in the same process and workspace
    mt.set_max_steps(0)
    assert mt.get_max_steps() == 1 << 24
    print("case step cap restored", flush=True)
    T, prs = gpu_tree(f, dev)
    assert_matches_oracle(f, T, prs, "after the cap")
    plan.launch()
    plan.sync_status()
    import oracle

    assert np.array_equal(u32(plan.triplets).reshape(-1, 2)[:f.size], oracle.merge_tree(f))

