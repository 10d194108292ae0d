"""Benchmark of the triplet merge tree path on one MI355X.

One step = the whole single-field hot path on the 512^3 log-normal k^-3 field
(merge tree and persistence pairs in one mt_build_pairs call, which
synchronizes to return the pair count), with the field already resident in
HBM.  Prints one JSON line.

The timed loop runs with no event bracketing; per-kernel times come from a
separate pass with the library's HIP-event timing on.

Also reported (under "secondary"): the uneven 48-field batch in one graph
launch against 48 plain calls (synchronous, and as 48 asynchronous
single-field graph launches), the same batch with autotuned tile shapes, the
backward scatter of a 16 x 128^3 differentiable batch over 100 gradient
steps, the split tree of the timed field, adversarial fields, and the global
sort a rank-keyed build would start with (mt_vertex_ranks) set against the
step.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
SRCS = [os.path.join(ROOT, "paper_2301_10838_amd", "csrc", n) for n in ("mt.hip", "mt_device.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")

# Compulsory HBM bytes of the whole path: read the field (4 B) and write the
# triplet (8 B) of every vertex, write every pair (two 4-byte ids, two
# 4-byte values).  Nothing else has to cross HBM.
COMPULSORY_PER_VERTEX = 12
COMPULSORY_PER_PAIR = 16


def compulsory_bytes(n_vertices: int, n_pairs: int) -> float:
    return float(COMPULSORY_PER_VERTEX * n_vertices + COMPULSORY_PER_PAIR * n_pairs)


# The kernels' own byte model: what each kernel must move given the
# intermediate records this design passes between kernels (labels, minimum
# slots, queued facts).  It is a model of this implementation, reported as
# such, not the algorithm's compulsory traffic above.  "Minima" are the local
# minima of the tiles, whose 24-byte records (16-byte slot + 8-byte key) the
# kernels pass on to each other.
MODEL_BYTES_PER_VERTEX = {
    "k_local": 8,        # read f, write the local-basin label
    "k_cross": 0,        # per-face-edge and per-fact terms below
    "k_qscatter": 0,     # per-fact term below
    "k_merge_q": 0,      # per-fact and per-minimum terms below
    "k_repair_min": 0,   # per-minimum term below
    "k_repair_reg": 16,  # read label and f, write the triplet
    "k_pairs_count": 8,  # read the triplet
    "k_pairs_write": 0,  # staged readout after a build: per-pair and per-bucket terms below
}


def model_bytes(kernel: str, n_vertices: int, n_pairs: int, n_local_minima: int, n_facts: int = 0,
                n_face_edges: int = 0) -> float:
    b = MODEL_BYTES_PER_VERTEX[kernel] * n_vertices
    if kernel == "k_qscatter":
        b += 32 * n_facts          # every fact read from the queue and written to its bin
    if kernel == "k_merge_q":
        b += 16 * n_facts + 16 * n_local_minima  # read every queued fact, settle every slot
    if kernel == "k_local":
        b += 24 * n_local_minima   # write slot + key of every local minimum
    if kernel == "k_cross":
        b += 16 * n_face_edges + 16 * n_facts  # label + value of both ends, one fact out
    if kernel == "k_repair_min":
        b += 16 * n_local_minima   # read (and rewrite) every slot once
    if kernel == "k_pairs_write":
        # the staged pair (ids and value bits) read and written; one count byte per 64 vertices
        b += 32 * n_pairs + n_vertices // 64
    return float(b)


def face_edges(shape, mt) -> int:
    """Grid edges that cross a tile face under the active tile shape of the
    field's dims class."""
    nx, ny, nz = mt.grid_dims(shape)
    cls = 0 if nz > 1 else (1 if ny > 1 else 2)
    sh = {s["id"]: s for s in mt.tile_shapes()}[mt.get_tile_shape(cls)]
    tx, ty, tz = sh["tx"], sh["ty"], sh["tz"]
    cut = lambda n, t: (n + t - 1) // t - 1  # interior tile boundaries along one axis
    return cut(nx, tx) * ny * nz + cut(ny, ty) * nx * nz + cut(nz, tz) * nx * ny


def src_hash() -> str:
    """SHA-256 over the kernel sources (host + device)."""
    h = hashlib.sha256()
    for p in SRCS:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(workload: str):
    """HBM bytes per launch of every kernel, {name: bytes}, from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source
    and workload; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("src_sha256") != src_hash() or t.get("workload") != workload:
        return None
    return {k: float(v["fetch_bytes"] + v["write_bytes"]) for k, v in t.get("kernels", {}).items()}


class Single:
    """Preallocated buffers for repeated single-field calls through the C ABI."""

    def __init__(self, ft, lib, mt):
        import torch

        self.lib, self.mt = lib, mt
        self.ft = ft
        self.dims = mt.grid_dims(ft.shape)
        nx, ny, nz = self.dims
        self.N = nx * ny * nz
        dev = ft.device
        self.T = torch.empty((self.N, 2), dtype=torch.int32, device=dev)
        self.ws = mt.alloc_workspace(lib.mt_workspace_bytes(nx, ny, nz), dev)
        self.cap = self.N // 2 + 1
        self.b = torch.empty(self.cap, dtype=torch.int32, device=dev)
        self.d = torch.empty(self.cap, dtype=torch.int32, device=dev)
        self.bv = torch.empty(self.cap, dtype=torch.float32, device=dev)
        self.dv = torch.empty(self.cap, dtype=torch.float32, device=dev)
        self.np = ctypes.c_int64(0)
        self.nr = ctypes.c_int64(0)
        self.stream = torch.cuda.current_stream(dev).cuda_stream

    def step(self, kind=0):
        """Tree and pairs in one call (mt_build_pairs); kind 0 merge, 1 split."""
        nx, ny, nz = self.dims
        rc = self.lib.mt_build_pairs(self.ft.data_ptr(), nx, ny, nz, kind, self.T.data_ptr(), self.b.data_ptr(),
                                     self.d.data_ptr(), self.bv.data_ptr(), self.dv.data_ptr(), self.cap,
                                     ctypes.byref(self.np), ctypes.byref(self.nr), self.ws.data_ptr(),
                                     self.ws.numel(), self.stream)
        if rc != 0:
            raise self.mt.MTError(rc, "mt_build_pairs")
        return self.np.value, self.nr.value

    def build_stats(self):
        """Internal sizes of a build alone (the pairs call reuses the header)."""
        nx, ny, nz = self.dims
        rc = self.lib.mt_build(self.ft.data_ptr(), nx, ny, nz, self.T.data_ptr(), self.ws.data_ptr(),
                               self.ws.numel(), self.stream)
        if rc != 0:
            raise self.mt.MTError(rc, "mt_build")
        return self.mt.build_stats(self.ws)


def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model


def cpu_baseline(f: np.ndarray, T_gpu: np.ndarray, birth_gpu: np.ndarray, death_gpu: np.ndarray):
    """The oracle (serial sort + union-find sweep + pairs, one core) on the
    whole timed field, once; the GPU's triplets and pairs of the same field
    are checked against it bit for bit.  A z < 64 slab is timed beside it."""
    import oracle

    t0 = time.perf_counter()
    T_ref = oracle.merge_tree(f)
    rb, rd, _, _, _ = oracle.pairs(f, T_ref)
    dt = time.perf_counter() - t0
    exact = bool(np.array_equal(T_gpu, T_ref) and np.array_equal(birth_gpu, rb) and np.array_equal(death_gpu, rd))
    del T_ref
    slab = {}
    if f.ndim == 3 and f.shape[0] > 64:
        sample = np.ascontiguousarray(f[:64])
        t1 = time.perf_counter()
        Ts = oracle.merge_tree(sample)
        oracle.pairs(sample, Ts)
        ds = time.perf_counter() - t1
        slab = {"slab": f"z < 64, {list(sample.shape)}", "slab_s": ds, "slab_Mvertices_per_s": sample.size / ds / 1e6}
    return {
        "value": f.size / dt / 1e6,
        "unit": "Mvertices/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"the whole timed field {list(f.shape)} ({f.size} vertices), one run of {dt:.1f} s: serial "
                  f"sort + union-find sweep + pairs (gcc -O2, one thread)",
        "seconds": dt,
        "host_cores_available": os.cpu_count(),
        "host_cpu": cpu_info(),
        "gpu_bit_exact_on_sample": exact,
        **slab,
    }


def tiles_of(s, mt) -> int:
    """Tiles of the single field under the active tile shape of its dims class."""
    nx, ny, nz = s.dims
    cls = 0 if nz > 1 else (1 if ny > 1 else 2)
    sh = {t["id"]: t for t in mt.tile_shapes()}[mt.get_tile_shape(cls)]
    return -(-nx // sh["tx"]) * -(-ny // sh["ty"]) * -(-nz // sh["tz"])


def atomic_rates(s, mt, kstats, dev):
    """Compare-and-swap rates of the merge kernels against the measured
    ceilings: one counting build of the timed field (outside the timed
    region) gives the swaps each kernel issues per launch; divided by the
    kernel's average time from the timed kernels' pass."""
    from paper_2301_10838_amd import micro

    ceil = micro.ceilings(dev)
    mt.set_counting(True)
    try:
        s.build_stats()
        c = mt.read_counters(s.ws)
    finally:
        mt.set_counting(False)
    s.step()  # the timed kernels again (restores nothing: the output is the same)

    def avg_s(k):
        return kstats[k][0] / kstats[k][1] / 1e3 if k in kstats else None

    out = {"counts": {k: v for k, v in c.items() if not k.startswith("cyc_")}}
    # phase clocks of the tile pass (a build whose tile pass only clocks its
    # phases): share of its time per phase, workgroup-first-lane clock summed over tiles
    mt.set_counting(2)
    try:
        s.build_stats()
        cp = mt.read_counters(s.ws)
    finally:
        mt.set_counting(False)
    cyc = {k[4:]: v for k, v in cp.items() if k.startswith("cyc_")}
    tot = sum(cyc.values())
    if tot:
        out["k_local_phase_share"] = {k: v / tot for k, v in cyc.items()}
        out["k_local_phase_cycles_per_tile"] = tot / max(1, tiles_of(s, mt))
    t = avg_s("k_merge_q")
    if t:
        rate = c["gm_cas"] / t / 1e9
        peak = ceil["cas_Gops"]["mall_128MiB"]
        out["k_merge_q"] = {"cas_per_launch": c["gm_cas"], "cas_fail_frac": c["gm_cas_fail"] / max(1, c["gm_cas"]),
                            "Gcas_per_s": rate, "peak_Gcas_per_s": peak, "frac": rate / peak,
                            "steps_per_fact": c["gm_steps"] / max(1, c["gm_facts"]),
                            "peak_note": "uncontended random 64-bit CAS over 128 MiB (cache-resident, like the slots)"}
    t = avg_s("k_local")
    if t:
        ops = c["lds_cas"] + c["table_probes"]  # LDS compare-and-swaps and atomic-min probes
        rate = ops / t / 1e9
        peak = ceil["lds_cas_Gops"]
        out["k_local"] = {"lds_atomics_per_launch": ops, "lds_cas_fail_frac": c["lds_cas_fail"] / max(1, c["lds_cas"]),
                          "Gops_per_s": rate, "peak_Gops_per_s": peak, "frac": rate / peak,
                          "steps_per_merge": c["lds_steps"] / max(1, c["lds_merges"])}
    return ceil, out


def bench_batch(dev, mt, lib, reps: int = 5):
    """The uneven 48-field batch: one graph launch against per-field calls,
    both the synchronous fused call (mt_build_pairs, which waits for its pair
    count) and one asynchronous single-field graph launch per field with one
    wait at the end; then the batch again with tile shapes picked by the
    autotuner."""
    import torch

    from paper_2301_10838_amd import fields, tune

    fs = fields.workload("batch48")
    shapes = [f.shape for f in fs]
    plan = mt.BatchPlan(shapes, dev)
    plan.load([torch.from_numpy(f).to(dev) for f in fs])
    n_total = plan.n_total

    def time_batch(pl):
        for _ in range(2):
            pl.launch()
            pl.sync_status()
        torch.cuda.synchronize()
        tb = []
        P = 0
        for _ in range(reps):
            t0 = time.perf_counter()
            pl.launch()
            P = pl.sync_status()
            tb.append(time.perf_counter() - t0)
        return statistics.median(tb), P

    tb_med, P = time_batch(plan)
    # plain, synchronous: one mt_build_pairs call per field
    singles = [Single(plan.fields[plan.vertex_offsets[i]:plan.vertex_offsets[i + 1]].view(shapes[i]), lib, mt)
               for i in range(len(shapes))]
    for s in singles:
        s.step()
    torch.cuda.synchronize()
    tp = []
    for _ in range(reps):
        t0 = time.perf_counter()
        for s in singles:
            s.step()
        torch.cuda.synchronize()
        tp.append(time.perf_counter() - t0)
    # plain, asynchronous: one single-field graph launch per field, one wait
    aplans = []
    for i, shp in enumerate(shapes):
        ap = mt.BatchPlan([shp], dev)
        ap.load([plan.fields[plan.vertex_offsets[i]:plan.vertex_offsets[i + 1]]])
        aplans.append(ap)
    for ap in aplans:
        ap.launch()
    for ap in aplans:
        ap.sync_status()
    ta = []
    for _ in range(reps):
        t0 = time.perf_counter()
        for ap in aplans:
            ap.launch()
        torch.cuda.synchronize()
        ta.append(time.perf_counter() - t0)
    for ap in aplans:
        ap.sync_status()
    # identical results, field by field
    offs = plan.pair_offsets.cpu().numpy()
    T_all = plan.triplets.cpu().numpy().view(np.uint32)
    b_all = plan.birth.cpu().numpy().view(np.uint32)
    same = True
    for i, s in enumerate(singles):
        a, b = plan.vertex_offsets[i], plan.vertex_offsets[i + 1]
        p = s.np.value
        same &= bool(np.array_equal(T_all[a:b], s.T.cpu().numpy().view(np.uint32)))
        same &= bool(np.array_equal(T_all[a:b], aplans[i].triplets.cpu().numpy().view(np.uint32)))
        same &= bool(offs[i + 1] - offs[i] == p)
        same &= bool(np.array_equal(b_all[offs[i]:offs[i + 1]], s.b[:p].cpu().numpy().view(np.uint32)))
    del singles, aplans
    tp_med, ta_med = statistics.median(tp), statistics.median(ta)
    out = {
        "workload": "batch48",
        "fields": len(shapes),
        "vertices": n_total,
        "pairs": int(P),
        "batched_ms": tb_med * 1e3,
        "plain_ms": tp_med * 1e3,
        "plain_async_ms": ta_med * 1e3,
        "batched_Mvertices_per_s": n_total / tb_med / 1e6,
        "plain_Mvertices_per_s": n_total / tp_med / 1e6,
        "batched_over_plain": tp_med / tb_med,
        "batched_over_plain_async": ta_med / tb_med,
        "batched_equals_plain": same,
    }
    # autotuned tile shapes (timed by the library, bit-identity checked on
    # the device), then the batch again with them; defaults restored after
    saved = [mt.get_tile_shape(c) for c in range(3)]
    saved_sched = mt.get_schedule()
    saved_cache = os.environ.get("MT_AUTOTUNE_CACHE")
    os.environ["MT_AUTOTUNE_CACHE"] = os.path.join("/tmp", f"mt_autotune_bench_{os.getpid()}.json")
    try:
        tensors = [plan.fields[plan.vertex_offsets[i]:plan.vertex_offsets[i + 1]].view(shapes[i])
                   for i in range(len(shapes))]
        chosen = tune.tune(tensors, reps=3, force=True)
        sched = tune.tune_schedule(tensors, reps=3, force=True)
        tplan = mt.BatchPlan(shapes, dev)
        tplan.fields.copy_(plan.fields)
        tt_med, _ = time_batch(tplan)
        same_t = bool(torch.equal(tplan.triplets, plan.triplets))
        info = {s["id"]: s for s in mt.tile_shapes()}
        out["tuned"] = {"shapes": {k: [info[v]["tx"], info[v]["ty"], info[v]["tz"]] for k, v in chosen.items()},
                        "default_shapes": {tune.CLASS_NAMES[c]: [info[saved[c]]["tx"], info[saved[c]]["ty"],
                                                                 info[saved[c]]["tz"]] for c in range(3)},
                        "schedule": sched,
                        "default_schedule": {"xcd_remap": saved_sched[0], "merge_groups": saved_sched[1]},
                        "batched_ms": tt_med * 1e3, "over_default": tb_med / tt_med, "equals_default": same_t}
        del tplan
    finally:
        for c in range(3):
            mt.set_tile_shape(c, saved[c])
        mt.set_schedule(*saved_sched)
        if saved_cache is None:
            os.environ.pop("MT_AUTOTUNE_CACHE", None)
        else:
            os.environ["MT_AUTOTUNE_CACHE"] = saved_cache
    return out


def bench_adversarial(dev, mt, lib, side: int = 256, steps: int = 3):
    """Build + pairs time of the adversarial fields at side^3 against the
    log-normal field of the same size."""
    import torch

    from paper_2301_10838_amd import fields

    cases = [
        ("lognormal_grf", lambda: fields.lognormal_grf((side,) * 3, 41)),
        ("serpentine", lambda: fields.serpentine((side,) * 3, 42)),
        ("tilted_checkerboard", lambda: fields.tilted_checkerboard((side,) * 3, 43)),
        ("parity_lattice", lambda: fields.parity_lattice((side,) * 3)),
        ("plateau_jump", lambda: fields.plateau_jump((side,) * 3, 44)),
        ("plateau_jump_noise", lambda: fields.plateau_jump((side,) * 3, 45, noise=1e-6)),
        ("nested_plateaus", lambda: fields.nested_plateaus((side,) * 3, 46)),
    ]
    out = {}
    for name, maker in cases:
        f = maker()
        s = Single(torch.from_numpy(f).to(dev), lib, mt)
        s.step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            P, _ = s.step()
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"ms": dt * 1e3, "Mvertices_per_s": s.N / dt / 1e6, "pairs": P}
        del s
    worst = max(out, key=lambda k: out[k]["ms"])
    return {"shape": [side] * 3, "cases": out, "worst": worst}


def bench_split(ft, lib, mt, s, steps: int = 5):
    """The split tree (merge tree of -f) of the timed field, build + pairs, and
    its bit-identity with the merge tree of the negated field."""
    import torch

    nx, ny, nz = s.dims

    def step():
        s.step(mt.MT_TREE_SPLIT)

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    T_split = s.T.clone()
    neg = (-ft).contiguous()
    rc = lib.mt_build(neg.data_ptr(), nx, ny, nz, s.T.data_ptr(), s.ws.data_ptr(), s.ws.numel(), s.stream)
    if rc != 0:
        raise mt.MTError(rc, "mt_build")
    torch.cuda.synchronize()
    same = bool(torch.equal(T_split, s.T))
    del neg, T_split
    return {"workload": "grf512 split tree", "ms_per_step": dt * 1e3, "Mvertices_per_s": s.N / dt / 1e6,
            "pairs": s.np.value, "equals_merge_tree_of_negated_field": same}


def bench_ranks(ft, lib, mt, step_ms: float, steps: int = 5):
    """The first step of a rank-keyed build (every vertex's position in the
    (value, id) order: order keys, one global radix sort, positions back) on
    the timed field, set against the whole value-keyed step."""
    import torch

    nx, ny, nz = mt.grid_dims(ft.shape)
    ws = mt.alloc_workspace(lib.mt_rank_workspace_bytes(nx, ny, nz), ft.device)
    r = torch.empty(ft.numel(), dtype=torch.int32, device=ft.device)
    st = torch.cuda.current_stream(ft.device).cuda_stream

    def step():
        rc = lib.mt_vertex_ranks(ft.data_ptr(), nx, ny, nz, mt.MT_TREE_MERGE, r.data_ptr(), ws.data_ptr(),
                                 ws.numel(), st)
        if rc != 0:
            raise mt.MTError(rc, "mt_vertex_ranks")

    step()
    torch.cuda.synchronize()
    mt.profile_begin()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    ks = mt.profile_end()
    sort_ms = ks["radix_sort"][0] / ks["radix_sort"][1] if "radix_sort" in ks else None
    del ws, r
    return {"workload": "grf512 vertex ranks", "ms": dt * 1e3, "radix_sort_ms": sort_ms,
            "over_value_keyed_step": dt * 1e3 / step_ms}


def bench_backward(dev, mt, steps: int = 100):
    """Gradient descent on the topological simplification loss
    sum over pairs with d - b < 0.05 of (d - b)^2, 16 bump fields at 128^3.
    bwd = loss.backward() (the loss's own backward ops, the autograd function
    and the adjoint kernels), timed with events; the adjoint kernels alone
    with the library's event timing."""
    import torch

    from paper_2301_10838_amd import fields

    fs = fields.workload("diff16x128")
    plan = mt.BatchPlan([f.shape for f in fs], dev)
    flat = torch.cat([torch.from_numpy(f).to(dev).reshape(-1) for f in fs])
    tau, lr = 0.05, 0.1
    bwd_us, fwd_ms, host_bwd_us, losses, pairs = [], [], [], [], []
    # the descent itself runs without the library's per-kernel events (they
    # add host time around every launch); the adjoint kernels are timed in a
    # short second pass
    for it in range(steps):
        x = flat.clone().requires_grad_(True)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        births, deaths = mt.MergeTreePairs.apply(x, plan)
        pers = deaths - births
        loss = torch.where(pers < tau, pers * pers, torch.zeros_like(pers)).sum()
        e1.record()
        h0 = time.perf_counter()
        loss.backward()
        e2.record()
        torch.cuda.synchronize()
        host_bwd_us.append((time.perf_counter() - h0) * 1e6)
        fwd_ms.append(e0.elapsed_time(e1))
        bwd_us.append(e1.elapsed_time(e2) * 1e3)
        losses.append(float(loss.detach()))
        pairs.append(births.numel())
        with torch.no_grad():
            flat -= lr * x.grad
    kpass = 10
    mt.profile_begin()
    for it in range(kpass):
        x = flat.clone().requires_grad_(True)
        births, deaths = mt.MergeTreePairs.apply(x, plan)
        pers = deaths - births
        torch.where(pers < tau, pers * pers, torch.zeros_like(pers)).sum().backward()
    torch.cuda.synchronize()
    ks = mt.profile_end()
    # the adjoint alone, called the way the autograd function calls it: host
    # time to enqueue (the rest of loss.backward() is the loss's own backward
    # ops and the autograd engine)
    P_last = pairs[-1]
    gb = torch.ones(P_last, dtype=torch.float32, device=dev)
    gd = torch.ones(P_last, dtype=torch.float32, device=dev)
    grad = torch.empty(plan.n_total, dtype=torch.float32, device=dev)
    lib = mt.load_library()
    st = torch.cuda.current_stream(dev).cuda_stream
    b_ids, d_ids, offs = plan.birth, plan.death, plan.pair_offsets
    torch.cuda.synchronize()
    t_host = []
    for _ in range(20):
        h0 = time.perf_counter()
        rc = lib.mt_pairs_backward(plan._dims_c, len(plan.dims), offs.data_ptr(), P_last, b_ids.data_ptr(),
                                   d_ids.data_ptr(), gb.data_ptr(), gd.data_ptr(), grad.data_ptr(), 0, st)
        t_host.append((time.perf_counter() - h0) * 1e6)
        if rc != 0:
            raise mt.MTError(rc, "mt_pairs_backward")
    torch.cuda.synchronize()
    adjoint_call_host_us = statistics.median(t_host)
    kern = {k: ks[k] for k in ("k_fill0", "k_scatter") if k in ks}
    kern_us = sum(v[0] for v in kern.values()) / kpass * 1e3
    P = statistics.median(pairs)
    # compulsory bytes of the adjoint: zero every gradient entry (4 B/vertex),
    # read each pair's two ids and two upstream gradients (16 B), read and
    # write the two gradient entries it lands on (16 B)
    adj_bytes = 4 * plan.n_total + 32 * P
    return {
        "workload": "diff16x128",
        "vertices": plan.n_total,
        "steps": steps,
        "pairs_median": P,
        "bwd_us_median": statistics.median(bwd_us[2:]),
        "bwd_host_us_median": statistics.median(host_bwd_us[2:]),
        "adjoint_call_host_us": adjoint_call_host_us,
        "bwd_kernel_us": kern_us,
        "bwd_kernels": {k: {"avg_us": v[0] / v[1] * 1e3, "launches": v[1]} for k, v in kern.items()},
        "adjoint_roofline": {"bound": "hbm", "bytes": adj_bytes, "achieved_GBps": adj_bytes / (kern_us * 1e3),
                             "frac": adj_bytes / (kern_us * 1e3) / HBM_PEAK_GBS},
        "fwd_ms_median": statistics.median(fwd_ms[2:]),
        "loss_first": losses[0],
        "loss_last": losses[-1],
    }


def summarize_profiles(trace_dir: str, fetch_dir: str, write_dir: str, workload: str, command: str):
    """Turn rocprofv3 CSV output (kernel trace + two counter passes) into the
    committed summaries: profiles/<kernel table>.md and profiles/traffic.json.

    HBM traffic per launch = counter reading scaled by what the same counter
    reads for the plain 1 GiB copy of --calibrate-copy (bytes moved / reading).
    """
    import csv
    import glob

    def rows(d, name):
        path = glob.glob(os.path.join(d, "**", f"*{name}"), recursive=True)
        if not path:
            raise FileNotFoundError(f"no {name} under {d}")
        with open(path[0]) as fh:
            return list(csv.DictReader(fh))

    stats = rows(trace_dir, "kernel_stats.csv")
    counters, peak = {}, {}
    for d, cname in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        per = {}
        for r in rows(d, "counter_collection.csv"):
            if r["Counter_Name"] != cname:
                continue
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)  # KiB -> bytes
        counters[cname] = {k: sum(v) / len(v) for k, v in per.items()}
        peak[cname] = {k: max(v) for k, v in per.items()}
    # the calibration copy is the largest dispatch of torch's elementwise kernel
    copy_name = next((k for k in counters["FETCH_SIZE"] if "elementwise" in k.lower()), None)
    calib = 1 << 30
    f_fac = calib / peak["FETCH_SIZE"][copy_name] if copy_name else None
    w_fac = calib / peak["WRITE_SIZE"][copy_name] if copy_name else None
    kernels = {}
    for k in set(counters["FETCH_SIZE"]) & set(counters["WRITE_SIZE"]):
        if not k.startswith("k_"):
            continue
        kernels[k] = {
            "fetch_bytes": counters["FETCH_SIZE"][k] * (f_fac or 1.0),
            "write_bytes": counters["WRITE_SIZE"][k] * (w_fac or 1.0),
            "fetch_raw_kib": counters["FETCH_SIZE"][k] / 1024.0,
            "write_raw_kib": counters["WRITE_SIZE"][k] / 1024.0,
        }
    traffic = {"workload": workload, "src_sha256": src_hash(), "copy_kernel": copy_name,
               "fetch_scale": f_fac, "write_scale": w_fac, "kernels": kernels,
               "command": command}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(traffic, fh, indent=1, sort_keys=True)
    lines = [f"# rocprofv3 kernel summary: {workload}", "", "Command (run from /tmp with TMPDIR=/tmp):", "",
             "```", command, "```", "",
             "| Kernel | Calls | Avg ms | Total % | HBM read MB/launch | HBM write MB/launch |",
             "|---|---|---|---|---|---|"]
    for r in stats:
        k = r["Name"]
        t = kernels.get(k, {})
        rd = f"{t['fetch_bytes'] / 1e6:.1f}" if t else "-"
        wr = f"{t['write_bytes'] / 1e6:.1f}" if t else "-"
        lines.append(f"| {k} | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | {float(r['Percentage']):.1f} | "
                     f"{rd} | {wr} |")
    lines += ["", f"Counter scale from the plain copy kernel `{copy_name}` (1 GiB read, 1 GiB written): "
              f"FETCH x{f_fac:.3f}, WRITE x{w_fac:.3f}." if copy_name else "", ""]
    out = os.path.join(ROOT, "profiles", f"kernels_{workload}.md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print(out, TRAFFIC_FILE)


def progress(msg: str):
    """One line on stderr when a phase of the run ends (the JSON line stays
    alone on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def summarize_counters(dirs, workload: str, command: str):
    """Turn rocprofv3 SQ counter passes (CSV) into profiles/counters_<workload>.md:
    per kernel, the instruction mix per wave and the share of the waves'
    resident cycles spent issuing and waiting (SQ_*_CYCLES and SQ_WAIT_* count
    in units of four cycles, alike, so their ratios need no scale)."""
    import csv
    import glob

    per = {}
    for d in dirs:
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not path:
            raise FileNotFoundError(f"no counter_collection.csv under {d}")
        with open(path[0]) as fh:
            for r in csv.DictReader(fh):
                per.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(
                    float(r["Counter_Value"]))
    avg = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in per.items()}
    order = ["k_local", "k_repair_reg", "k_merge_q", "k_cross", "k_repair_min", "k_pairs_write", "k_qscatter"]
    lines = [f"# rocprofv3 SQ counters: {workload}", "", "Command (run from /tmp with TMPDIR=/tmp), one run per pass:",
             "", "```", command, "```", "",
             "Per launch (average over launches). Instructions are counted per wave; cycle counters are in the "
             "SQ's four-cycle units, so only their ratios are used.", "",
             "| Kernel | waves | VALU/wave | SALU/wave | LDS/wave | VMEM rd/wave | VMEM wr/wave | issuing | "
             "waiting | LDS bank-conflict share of LDS cycles |",
             "|---|---|---|---|---|---|---|---|---|---|"]

    def g(k, c):
        return avg[k].get(c)

    for k in order:
        if k not in avg:
            continue
        w = g(k, "SQ_WAVES") or 0
        def pw(c):
            v = g(k, c)
            return f"{v / w:.0f}" if (v is not None and w) else "-"
        wc = g(k, "SQ_WAVE_CYCLES")
        iss = f"{g(k, 'SQ_ACTIVE_INST_ANY') / wc:.2f}" if wc and g(k, "SQ_ACTIVE_INST_ANY") is not None else "-"
        wt = f"{g(k, 'SQ_WAIT_ANY') / wc:.2f}" if wc and g(k, "SQ_WAIT_ANY") is not None else "-"
        lds = g(k, "SQ_ACTIVE_INST_LDS")
        bc = f"{g(k, 'SQ_LDS_BANK_CONFLICT') / lds:.2f}" if lds else "-"
        lines.append(f"| {k} | {w:.0f} | {pw('SQ_INSTS_VALU')} | {pw('SQ_INSTS_SALU')} | {pw('SQ_INSTS_LDS')} | "
                     f"{pw('SQ_INSTS_VMEM_RD')} | {pw('SQ_INSTS_VMEM_WR')} | {iss} | {wt} | {bc} |")
    lines += ["", "Raw averages per launch:", ""]
    for k in order:
        if k in avg:
            lines.append(f"- `{k}`: " + ", ".join(f"{c} {v:.4g}" for c, v in sorted(avg[k].items())))
    lines.append("")
    out = os.path.join(ROOT, "profiles", f"counters_{workload}.md")
    with open(out, "w") as fh:
        fh.write("\n".join(lines))
    print(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grf512")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (3 times), the reference for HBM counters")
    ap.add_argument("--summarize-profiles", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/ summaries from rocprofv3 CSV output and exit (no GPU)")
    ap.add_argument("--summarize-counters", nargs="+", metavar="PASS_DIR",
                    help="write profiles/counters_<workload>.md from rocprofv3 SQ counter passes and exit (no GPU)")
    ap.add_argument("--profile-command", default="", help="command line recorded in the summary")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles, args.workload, args.profile_command)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.workload, args.profile_command)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the merge-tree path here runs on a single MI355X and has no "
              "multi-GPU mode; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2301_10838_amd.mt as mt
    from paper_2301_10838_amd import fields

    lib = mt.load_library()
    dev = torch.device("cuda:0")
    f = fields.workload(args.workload)[0]
    progress(f"field {args.workload} {list(f.shape)} generated")
    ft = torch.from_numpy(f).to(dev)
    s = Single(ft, lib, mt)
    for _ in range(args.warmup):
        s.step()
    torch.cuda.synchronize()

    # timed region: K whole steps, nothing else on the stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P, R = s.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = (t1 - t0) / args.steps
    N = s.N
    progress(f"timed {args.steps} steps: {dt * 1e3:.3f} ms per step")

    # per-kernel times in a separate pass (HIP events around every launch)
    mt.profile_begin()
    for _ in range(args.steps):
        s.step()
    torch.cuda.synchronize()
    kstats = mt.profile_end()

    n_min, n_facts = s.build_stats()  # local minima records and queued cross-tile facts (untimed)
    s.step()
    torch.cuda.synchronize()
    n_face = face_edges(f.shape, mt)
    per_kernel = {k: {"avg_ms": v[0] / v[1], "launches": v[1]} for k, v in sorted(kstats.items())}
    kernel_ms_sum = sum(v[0] for v in kstats.values()) / args.steps
    traffic = stored_traffic(args.workload)

    # roofline of the dominant kernel: the path's per-vertex compulsory bytes
    # (read f, write T: 12 B) times the vertices one launch sweeps
    dom = max((k for k in kstats if k in MODEL_BYTES_PER_VERTEX), key=lambda k: kstats[k][0])
    avg_s = kstats[dom][0] / kstats[dom][1] / 1e3
    ab = float(COMPULSORY_PER_VERTEX * N)
    achieved = ab / avg_s / 1e9
    roofline = {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic.get(dom) if traffic else None,
        "kernel": dom,
        "kernel_avg_ms": avg_s * 1e3,
        "algo_bytes_per_launch": ab,
        "algo_bytes_rule": "12 B per vertex of the launch (read f, write T)",
    }
    cb = compulsory_bytes(N, P)
    path = {
        "compulsory_bytes": cb,
        "compulsory_frac": cb / dt / 1e9 / HBM_PEAK_GBS,
        "kernel_ms_sum": kernel_ms_sum,
        "counter_bytes": None,
        "counter_frac_step": None,
        "counter_frac_kernels": None,
    }
    if traffic:
        ctot = sum(traffic.get(k, 0.0) for k in kstats)
        path.update(counter_bytes=ctot, counter_frac_step=ctot / dt / 1e9 / HBM_PEAK_GBS,
                    counter_frac_kernels=ctot / (kernel_ms_sum * 1e6) / HBM_PEAK_GBS)
    model = {k: {"bytes": model_bytes(k, N, P, n_min, n_facts, n_face),
                 "GBps": model_bytes(k, N, P, n_min, n_facts, n_face) / (kstats[k][0] / kstats[k][1] * 1e6)}
             for k in kstats if k in MODEL_BYTES_PER_VERTEX}

    out = {
        "metric": "Mvertices/s merge tree+pairs (bit-exact), batched vs plain; %HBM peak; bwd μs",
        "value": N / dt / 1e6,
        "unit": "Mvertices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "shape": list(f.shape), "vertices": N, "connectivity": 6,
                   "pairs": P, "roots": R, "tile_local_minima": n_min,
                   "cross_tile_facts": n_facts, "tile_face_edges": n_face},
        "roofline": roofline,
        "path": path,
        "kernels": per_kernel,
        "model_bytes": model,
    }
    if args.calibrate_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # one elementwise kernel: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst
    if not args.no_secondary:
        out["ceilings"], out["atomics"] = atomic_rates(s, mt, kstats, dev)
        progress("ceilings and atomic rates")
        if dom in out["atomics"]:
            roofline["atomic"] = out["atomics"][dom]
    T_host = s.T.cpu().numpy().view(np.uint32).reshape(-1, 2)
    b_host = s.b[:P].cpu().numpy().view(np.uint32)
    d_host = s.d[:P].cpu().numpy().view(np.uint32)
    if not args.no_secondary:
        sec = {}
        sec["split_tree"] = bench_split(ft, lib, mt, s)
        progress("split_tree")
        sec["rank_keys"] = bench_ranks(ft, lib, mt, dt * 1e3)
        progress("rank_keys")
        del s
        torch.cuda.empty_cache()
        sec["batched"] = bench_batch(dev, mt, lib)
        progress("batched")
        sec["backward"] = bench_backward(dev, mt)
        progress("backward")
        sec["adversarial"] = bench_adversarial(dev, mt, lib)
        progress("adversarial")
        out["secondary"] = sec
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(f, T_host, b_host, d_host)
        progress("cpu baseline")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
