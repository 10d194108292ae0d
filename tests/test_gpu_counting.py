"""The counting build (mt_set_counting): the same triplets as the timed
build, and counters that agree with each other and with the build's own
sizes (every queued cross-tile fact starts one merge, failed swaps are a
subset of swaps, every phase of the tile pass takes time)."""
import numpy as np
import pytest
import torch

from gpu_util import assert_matches_oracle, device, u32
from paper_2301_10838_amd import fields

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,maker", [
    ("grf", lambda: fields.lognormal_grf((70, 66, 61), 111)),
    ("ties", lambda: np.random.default_rng(112).integers(0, 4, (40, 33, 35)).astype(np.float32)),
])
def test_counting_build_same_tree_and_consistent_counts(name, maker):
    import paper_2301_10838_amd.mt as mt

    dev = device()
    f = maker()
    print("case counting", name, f.shape, flush=True)
    ft = torch.from_numpy(f).to(dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    T0 = mt.mt_build(ft, workspace=ws)
    torch.cuda.synchronize()
    mt.set_counting(True)
    try:
        T1 = mt.mt_build(ft, workspace=ws)
        c = mt.read_counters(ws)
        n_min, n_facts = mt.build_stats(ws)
    finally:
        mt.set_counting(False)
    assert torch.equal(T0, T1)
    b, d, bv, dv, r = mt.mt_persistence_pairs(ft, T1, workspace=ws)
    torch.cuda.synchronize()
    assert_matches_oracle(f, u32(T1).reshape(-1, 2), (u32(b), u32(d), bv.cpu().numpy(), dv.cpu().numpy(), r), name)
    assert c["gm_facts"] == n_facts
    assert c["gm_cas_fail"] <= c["gm_cas"] and c["lds_cas_fail"] <= c["lds_cas"]
    assert c["gm_descents"] <= c["gm_steps"] and c["gm_steps"] >= c["gm_facts"]
    assert c["lds_steps"] >= c["lds_merges"] > 0
    assert c["table_probes"] >= c["table_inserts"] - c["table_direct"]
    phases = [k for k in mt.COUNTER_NAMES if k.startswith("cyc_")]
    assert len(phases) == 10 and all(c[k] == 0 for k in phases)  # event mode clocks nothing
    # phase-clock mode: the same tree, every phase timed, no event counted
    mt.set_counting(2)
    try:
        T2 = mt.mt_build(ft, workspace=ws)
        c2 = mt.read_counters(ws)
    finally:
        mt.set_counting(False)
    assert torch.equal(T0, T2)
    assert all(c2[k] > 0 for k in phases), {k: c2[k] for k in phases}
    assert all(c2[k] == 0 for k in mt.COUNTER_NAMES if not k.startswith("cyc_"))
    # a timed build after it leaves the counters at zero
    mt.mt_build(ft, workspace=ws)
    assert all(v == 0 for v in mt.read_counters(ws).values())


@pytest.mark.parametrize("probes", [0, 2])
def test_counting_overflow_paths(probes):
    """A probe limit sends edges past the in-tile pair table: with no probe
    every offered edge overflows and every tile with more edges than the
    overflow list holds merges all its edges at once; with two probes some
    edges overflow.  The tree stays the oracle's either way."""
    import paper_2301_10838_amd.mt as mt

    dev = device()
    f = fields.lognormal_grf((64, 64, 64), 113)
    print("case counting overflow probes", probes, flush=True)
    ft = torch.from_numpy(f).to(dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    mt.set_table_probes(probes)
    mt.set_counting(True)
    try:
        T = mt.mt_build(ft, workspace=ws)
        c = mt.read_counters(ws)
        b, d, bv, dv, r = mt.mt_persistence_pairs(ft, T, workspace=ws)
        torch.cuda.synchronize()
    finally:
        mt.set_counting(False)
        mt.set_table_probes(-1)
    assert_matches_oracle(f, u32(T).reshape(-1, 2), (u32(b), u32(d), bv.cpu().numpy(), dv.cpu().numpy(), r),
                          f"overflow probes={probes}")
    assert c["table_direct"] > 0
    if probes == 0:
        assert c["table_probes"] == 0 and c["table_direct"] == c["table_inserts"]
        assert 0 < c["table_overflow_tiles"] <= 64  # 64 tiles of 16^3, each with hundreds of edges
    else:
        assert c["table_direct"] < c["table_inserts"]
