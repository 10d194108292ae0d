"""Benchmark of the triplet merge tree path on one MI355X.

One step = the whole single-field hot path on the 512^3 log-normal k^-3 field
(merge tree and persistence pairs in one mt_build_pairs call, which
synchronizes to return the pair count), with the field already resident in
HBM.  Prints one JSON line.

Also reported (under "secondary"): the uneven 48-field batch in one graph
launch against 48 plain calls, the backward scatter of a 16 x 128^3
differentiable batch, the split tree of the timed field, and the global sort
a rank-keyed build would start with (mt_vertex_ranks) set against the step.

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

# Compulsory HBM bytes each kernel must move, per vertex of its launch (plus
# the per-minimum and per-pair terms noted in algo_bytes).  "Minima" here are
# the local minima of the tiles, whose 24-byte records (16-byte slot + 8-byte
# key) the kernels pass on to each other.
ALGO_BYTES_PER_VERTEX = {
    "k_local": 8,        # read f, write the local-basin label
    "k_cross": 0,        # per-face-edge and per-fact terms below
    "k_qscatter": 0,     # per-fact term below
    "k_merge_q": 0,      # per-fact and per-minimum terms below
    "k_repair_min": 0,   # per-minimum term below
    "k_repair_reg": 16,  # read label and f, write the triplet
    "k_pairs_count": 8,  # read the triplet
    "k_pairs_write": 8,  # read the triplet (+24 per pair: both values read, the pair written)
}


def algo_bytes(kernel: str, n_vertices: int, n_pairs: int, n_local_minima: int, n_facts: int = 0,
               n_face_edges: int = 0) -> float:
    b = ALGO_BYTES_PER_VERTEX[kernel] * n_vertices
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
        b += 24 * n_pairs          # f at birth and death read; birth, death ids and values written
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


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("src_sha256") != src_hash() or t.get("workload") != workload:
        return None
    k = t.get("kernels", {}).get(kernel)
    if not k:
        return None
    return float(k["fetch_bytes"] + k["write_bytes"])


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


def cpu_baseline(f: np.ndarray, dev, mt, lib):
    """Oracle (serial, one core) on a bounded slab of the workload, and the GPU
    on the same slab, checked bit for bit."""
    import torch

    import oracle

    nz = f.shape[0]
    slab_z = 64 if f.ndim == 3 and nz > 64 else nz
    sample = np.ascontiguousarray(f[:slab_z])
    t0 = time.perf_counter()
    T_ref = oracle.merge_tree(sample)
    rb, rd, _, _, _ = oracle.pairs(sample, T_ref)
    dt = time.perf_counter() - t0
    s = Single(torch.from_numpy(sample).to(dev), lib, mt)
    P, _ = s.step()
    torch.cuda.synchronize()
    exact = bool(np.array_equal(s.T.cpu().numpy().view(np.uint32), T_ref)
                 and np.array_equal(s.b[:P].cpu().numpy().view(np.uint32), rb)
                 and np.array_equal(s.d[:P].cpu().numpy().view(np.uint32), rd))
    return {
        "value": sample.size / dt / 1e6,
        "unit": "Mvertices/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"z < {slab_z} slab {list(sample.shape)} ({sample.size} vertices) of the timed field; "
                  f"serial sort + union-find sweep + pairs, {dt:.1f} s",
        "host_cores_available": os.cpu_count(),
        "gpu_bit_exact_on_sample": exact,
    }


def bench_batch(dev, mt, lib, reps: int = 5):
    import torch

    from paper_2301_10838_amd import fields

    fs = fields.workload("batch48")
    shapes = [f.shape for f in fs]
    plan = mt.BatchPlan(shapes, dev)
    plan.load([torch.from_numpy(f).to(dev) for f in fs])
    n_total = plan.n_total
    for _ in range(2):
        plan.launch()
        plan.sync_status()
    torch.cuda.synchronize()
    tb = []
    for _ in range(reps):
        t0 = time.perf_counter()
        plan.launch()
        P = plan.sync_status()
        tb.append(time.perf_counter() - t0)
    # plain: one mt_build_pairs call per field
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
    # identical results, field by field
    offs = plan.pair_offsets.cpu().numpy()
    T_all = plan.triplets.cpu().numpy().view(np.uint32)
    b_all = plan.birth.cpu().numpy().view(np.uint32)
    same = True
    for i, s in enumerate(singles):
        a, b = plan.vertex_offsets[i], plan.vertex_offsets[i + 1]
        p = s.np.value
        same &= bool(np.array_equal(T_all[a:b], s.T.cpu().numpy().view(np.uint32)))
        same &= bool(offs[i + 1] - offs[i] == p)
        same &= bool(np.array_equal(b_all[offs[i]:offs[i + 1]], s.b[:p].cpu().numpy().view(np.uint32)))
    tb_med, tp_med = statistics.median(tb), statistics.median(tp)
    return {
        "workload": "batch48",
        "fields": len(shapes),
        "vertices": n_total,
        "pairs": int(P),
        "batched_ms": tb_med * 1e3,
        "plain_ms": tp_med * 1e3,
        "batched_Mvertices_per_s": n_total / tb_med / 1e6,
        "plain_Mvertices_per_s": n_total / tp_med / 1e6,
        "batched_over_plain": tp_med / tb_med,
        "batched_equals_plain": same,
    }


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


def bench_backward(dev, mt, steps: int = 20):
    import torch

    from paper_2301_10838_amd import fields

    fs = fields.workload("diff16x128")
    plan = mt.BatchPlan([f.shape for f in fs], dev)
    flat = torch.cat([torch.from_numpy(f).to(dev).reshape(-1) for f in fs])
    tau, lr = 0.05, 0.1
    bwd_us, fwd_ms, losses = [], [], []
    mt.profile_begin()
    for it in range(steps):
        x = flat.clone().requires_grad_(True)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        births, deaths = mt.MergeTreePairs.apply(x, plan)
        pers = deaths - births
        loss = torch.where(pers < tau, pers * pers, torch.zeros_like(pers)).sum()
        e1.record()
        loss.backward()
        e2.record()
        torch.cuda.synchronize()
        fwd_ms.append(e0.elapsed_time(e1))
        bwd_us.append(e1.elapsed_time(e2) * 1e3)
        losses.append(float(loss))
        with torch.no_grad():
            flat -= lr * x.grad
    ks = mt.profile_end()
    kern_ms = sum(ks.get(k, (0.0, 0))[0] for k in ("k_fill0", "k_scatter"))
    return {
        "workload": "diff16x128",
        "vertices": plan.n_total,
        "steps": steps,
        "bwd_kernel_us": kern_ms / steps * 1e3,
        "bwd_us_median": statistics.median(bwd_us[2:]),
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
    ap.add_argument("--profile-command", default="", help="command line recorded in the summary")
    args = ap.parse_args()
    if args.summarize_profiles:
        summarize_profiles(*args.summarize_profiles, args.workload, args.profile_command)
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
    ft = torch.from_numpy(f).to(dev)
    s = Single(ft, lib, mt)
    for _ in range(args.warmup):
        s.step()
    torch.cuda.synchronize()

    mt.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        P, R = s.step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kstats = mt.profile_end()
    dt = (t1 - t0) / args.steps
    N = s.N

    n_min, n_facts = s.build_stats()  # local minima records and queued cross-tile facts (untimed)
    n_face = face_edges(f.shape, mt)
    dom = max((k for k in kstats if k in ALGO_BYTES_PER_VERTEX), key=lambda k: kstats[k][0])
    avg_s = kstats[dom][0] / kstats[dom][1] / 1e3
    ab = algo_bytes(dom, N, P, n_min, n_facts, n_face)
    achieved = ab / avg_s / 1e9
    traffic = stored_traffic(dom, args.workload)
    roofline = {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "kernel": dom,
        "kernel_avg_ms": avg_s * 1e3,
        "algo_bytes_per_launch": ab,
    }
    per_kernel = {k: {"avg_ms": v[0] / v[1], "launches": v[1]} for k, v in sorted(kstats.items())}
    path_bytes = sum(algo_bytes(k, N, P, n_min, n_facts, n_face) for k in ALGO_BYTES_PER_VERTEX)

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
        "path_algo_GBps": path_bytes / dt / 1e9,
        "kernels": per_kernel,
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
        out["secondary"] = {"batched": bench_batch(dev, mt, lib), "backward": bench_backward(dev, mt),
                            "split_tree": bench_split(ft, lib, mt, s),
                            "rank_keys": bench_ranks(ft, lib, mt, dt * 1e3)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(f, dev, mt, lib)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
