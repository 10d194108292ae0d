"""Autotuner: every candidate tile shape gives bit-identical triplets (checked
inside the library), the chosen shapes are applied, and results stay exact."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import device, gpu_tree
from paper_2301_10838_amd import fields

pytestmark = pytest.mark.gpu


def test_autotune_selects_and_stays_exact(dev=None, tmp_path=None):
    import paper_2301_10838_amd.mt as mt

    dev = device()
    fs = [fields.lognormal_grf((40, 36, 33), 401), fields.lognormal_grf((150, 170), 402),
          fields.uniform((3000,), 403)]
    before = {c: mt.get_tile_shape(c) for c in range(3)}
    try:
        res = mt.autotune([torch.from_numpy(f).to(dev) for f in fs], reps=1)
        assert set(res) == {0, 1, 2}
        shapes = {s["id"]: s for s in mt.tile_shapes()}
        for c, (sid, ms) in res.items():
            assert shapes[sid]["dims_class"] == c and ms > 0
            assert mt.get_tile_shape(c) == sid
        for f in fs:
            T, _ = gpu_tree(f, dev)
            assert np.array_equal(T, oracle.merge_tree(f))
        # every compiled shape, forced one by one, gives the oracle's tree
        for s in mt.tile_shapes():
            mt.set_tile_shape(s["dims_class"], s["id"])
            f = fs[s["dims_class"]]
            T, _ = gpu_tree(f, dev)
            assert np.array_equal(T, oracle.merge_tree(f)), s
    finally:
        for c, sid in before.items():
            mt.set_tile_shape(c, sid)


def test_tune_driver_cache(tmp_path, monkeypatch):
    import paper_2301_10838_amd.mt as mt
    from paper_2301_10838_amd import tune

    dev = device()
    monkeypatch.setenv("MT_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    before = {c: mt.get_tile_shape(c) for c in range(3)}
    try:
        fs = [torch.from_numpy(fields.lognormal_grf((24, 20, 18), 404)).to(dev)]
        first = tune.tune(fs, reps=1)
        assert (tmp_path / "tune.json").exists()
        mt.set_tile_shape(0, before[0])
        again = tune.tune(fs, reps=1)  # from the cache
        assert again == first
    finally:
        for c, sid in before.items():
            mt.set_tile_shape(c, sid)


def test_every_shape_checkerboard():
    """Tiles with as many local minima as a tile can hold (every other vertex)
    take the direct-merge path of the tile pass on every compiled shape."""
    import paper_2301_10838_amd.mt as mt

    dev = device()
    before = {c: mt.get_tile_shape(c) for c in range(3)}
    try:
        for s in mt.tile_shapes():
            c = s["dims_class"]
            ext = [2 * s["tx"] + 3, 2 * s["ty"] + 1, 2 * s["tz"] + 1][: 3 - c]
            idx = np.indices(ext[::-1])
            f = (idx.sum(0) % 2).astype(np.float32)
            mt.set_tile_shape(c, s["id"])
            print("case checkerboard", s, f.shape, flush=True)
            T, prs = gpu_tree(f, dev)
            assert np.array_equal(T, oracle.merge_tree(f)), s
            assert prs[0].size == (f.size + 1) // 2 - 1, s
    finally:
        for c, sid in before.items():
            mt.set_tile_shape(c, sid)


def test_schedule_tuner_and_every_schedule_exact(tmp_path, monkeypatch):
    """The schedule tuner checks bit-identity over its candidates and applies
    the winner; every schedule, forced, gives the oracle's tree (also in a
    batch graph, whose cache key includes the schedule)."""
    import paper_2301_10838_amd.mt as mt
    from paper_2301_10838_amd import tune

    dev = device()
    monkeypatch.setenv("MT_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    before = mt.get_schedule()
    assert before == (1, 2048)
    fs = [fields.lognormal_grf((70, 66, 61), 405), fields.lognormal_grf((300, 257), 406)]
    ts = [torch.from_numpy(f).to(dev) for f in fs]
    try:
        r, g, ms = mt.autotune_schedule(ts, reps=1)
        assert r in (0, 1) and g in (256, 1024, 2048, 8192) and ms > 0
        assert mt.get_schedule() == (r, g)
        got = tune.tune_schedule(ts, reps=1)
        assert (tmp_path / "tune.json").exists() and set(got) == {"xcd_remap", "merge_groups"}
        mt.set_schedule(-1, 0)
        assert tune.tune_schedule(ts, reps=1) == got  # from the cache
        refs = [oracle.merge_tree(f) for f in fs]
        for remap in (0, 1):
            for groups in (1, 256, 8192):
                mt.set_schedule(remap, groups)
                print("case schedule", remap, groups, flush=True)
                for f, ref in zip(fs, refs):
                    T, _ = gpu_tree(f, dev)
                    assert np.array_equal(T, ref), (remap, groups)
                plan = mt.BatchPlan([f.shape for f in fs], dev)
                mt.mt_batch_build(ts, plan=plan)
                Tb = plan.triplets.cpu().numpy().view(np.uint32)
                a = 0
                for f, ref in zip(fs, refs):
                    assert np.array_equal(Tb[a:a + f.size], ref), (remap, groups)
                    a += f.size
    finally:
        mt.set_schedule(*before)
    with pytest.raises(mt.MTError):
        mt.set_schedule(2, 0)
    with pytest.raises(mt.MTError):
        mt.set_schedule(1, -5)
