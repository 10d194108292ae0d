"""The lock-free algorithm (Sec. 2, Alg. 1-5) under adversarial interleavings.

The simulator runs the parallel merge and repair phases with a seeded random
scheduler; whatever the interleaving and edge order, the result must be the
unique minimal triplet tree the oracle computes.  The three readings of the
printed pseudocode are pinned by traces where the literal text goes wrong.
"""
import json
import os

import numpy as np
import pytest

import oracle
import tmt_sim
from paper_2301_10838_amd import fields

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _fields_tiny():
    rng = np.random.default_rng(5)
    out = []
    for shape in [(9,), (3, 4), (4, 4), (2, 3, 3), (3, 3, 3)]:
        out.append(rng.integers(0, 3, size=shape).astype(np.float32))
        out.append(rng.random(shape).astype(np.float32))
    out.append(fields.bumps((6, 6, 6), 3, n_bumps=3, sigma=(1, 2)))
    out.append(fields.lognormal_grf((10, 12), 4))
    return out


@pytest.mark.parametrize("variant", ["paper", "prelink", "basins", "tiles", "tile_trees", "tile_trees_lowest"])
def test_interleavings_reach_oracle(variant):
    for i, f in enumerate(_fields_tiny()):
        want = oracle.merge_tree(f)
        for seed in range(12):
            got = tmt_sim.simulate(f, seed=1000 * i + seed, variant=variant)
            assert np.array_equal(got, want), (variant, i, seed)


def test_errata_traces():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    ex = {e["name"]: e for e in g["examples"]}
    tr = {t["name"]: t for t in g["errata_traces"]}

    e5 = np.array(ex["E5_cross"]["values"], np.float32)
    order = [tuple(e) for e in tr["E5b_root_remerge"]["edge_order"]]
    ok = tmt_sim.simulate(e5, variant="paper", edge_order=order, serial=True)
    assert ok.tolist() == ex["E5_cross"]["T"]
    bad = tmt_sim.simulate(e5, variant="paper", edge_order=order, serial=True, skip_root_remerge=False)
    assert bad.tolist() == tr["E5b_root_remerge"]["wrong_T_without_guard"]

    e1 = np.array(ex["E1_path"]["values"], np.float32)
    order = [tuple(e) for e in tr["E1_return_target"]["edge_order"]]
    ok = tmt_sim.simulate(e1, variant="paper", edge_order=order, serial=True)
    assert ok.tolist() == ex["E1_path"]["T"]
    bad = tmt_sim.simulate(e1, variant="paper", edge_order=order, serial=True, return_last=False)
    assert bad.tolist() == tr["E1_return_target"]["wrong_T_return_target"]

    # without the root guard the descent on (x, x, x) never ends
    with pytest.raises(tmt_sim.LivelockError):
        tmt_sim.simulate(e1, variant="paper", edge_order=order, serial=True, root_guard=False)


def test_prelink_is_a_reachable_state():
    # merging each vertex's steepest-descent edge, in decreasing order of the
    # upper vertex, leaves exactly T[u] = (u, w(u)): check on a small field
    f = np.random.default_rng(1).random((4, 5)).astype(np.float32)
    flat = f.ravel().astype(np.float64)
    key = lambda x: (flat[x], x)
    w = tmt_sim.steepest_lower(flat, f.shape)
    T = [(u, u) for u in range(f.size)]
    for u in sorted(range(f.size), key=key, reverse=True):
        if w[u] != u:
            for _ in tmt_sim.merge_thread(T, key, u, u, int(w[u])):
                pass
    assert T == [(u, int(w[u])) if w[u] != u else (u, u) for u in range(f.size)]


@pytest.mark.parametrize("variant", ["tiles", "tile_trees", "tile_trees_lowest"])
@pytest.mark.parametrize("box", [(1, 1, 1), (2, 2, 2), (3, 2, 1), (4, 4, 4)])
def test_two_level_boxes(box, variant):
    rng = np.random.default_rng(9)
    for i in range(6):
        shape = [(5, 6, 4), (7, 9), (20,)][i % 3]
        f = rng.integers(0, 4, size=shape).astype(np.float32) if i % 2 else rng.random(shape).astype(np.float32)
        want = oracle.merge_tree(f)
        for seed in range(4):
            got = tmt_sim.simulate(f, seed=seed, variant=variant, box=box)
            assert np.array_equal(got, want), (variant, box, i, seed)


@pytest.mark.parametrize("variant", ["paper", "basins", "tile_trees_lowest"])
@pytest.mark.parametrize("compress_after", [0, 2])
def test_path_compression_in_descents(variant, compress_after):
    """Merges that re-point a link they descend through (x -> y -> z with y's
    saddle not above x's becomes x -> z at x's saddle, by compare-and-swap)
    reach the oracle's tree under every interleaving: the early write is one
    step of Repair (Alg. 4, 5) and leaves every connection Merge relies on."""
    fs = _fields_tiny() + [fields.serpentine((6, 7, 8), 3), fields.serpentine((9, 10), 4, descending=True),
                           fields.plateau_jump((6, 5, 4), 5)]
    for i, f in enumerate(fs):
        want = oracle.merge_tree(f)
        for seed in range(10):
            got = tmt_sim.simulate(f, seed=77 * i + seed, variant=variant, compress_after=compress_after,
                                   box=(3, 2, 2))
            assert np.array_equal(got, want), (variant, compress_after, i, seed)
