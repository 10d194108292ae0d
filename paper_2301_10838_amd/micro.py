"""Binding of libmt_micro.so (ctypes): the measured ceilings the merge-tree
kernels are set against.  Measurement only; the merge-tree path never calls it.

ceilings(device) runs each kernel at a few sizes and returns rates:
- copy: streaming HBM copy, GB/s counting bytes read + written;
- cas: returning 64-bit compare-and-swap at hashed addresses, Gops/s, over
  arrays sized like the merge's minimum slots (L2 / last-level cache / HBM
  resident) and over a handful of words (contended);
- lds_cas: returning 64-bit LDS compare-and-swap over the whole chip, Gops/s;
- chase: dependent loads along a random cycle, ns per step for one chain per
  lane at low occupancy, and Gloads/s with many chains in flight.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmt_micro.so")
_lib = None


def load_library():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    D = ctypes.POINTER(ctypes.c_double)
    lib.mtm_copy.argtypes = [P, P, I64, I, P, D]
    lib.mtm_cas.argtypes = [P, I64, I64, I, I, P, P, D]
    lib.mtm_lds_cas.argtypes = [I64, I, I, P, P, D]
    lib.mtm_chase.argtypes = [P, I64, I, I64, I, P, P, D]
    for f in (lib.mtm_copy, lib.mtm_cas, lib.mtm_lds_cas, lib.mtm_chase):
        f.restype = ctypes.c_int
    _lib = lib
    return lib


def _ok(rc, what):
    if rc != 0:
        raise RuntimeError(f"{what}: status {rc}")


def ceilings(device) -> dict:
    lib = load_library()
    dev = torch.device(device)
    st = torch.cuda.current_stream(dev).cuda_stream
    ms = ctypes.c_double(0.0)
    out = {}
    # streaming copy of 1 GiB
    nb = 1 << 30
    src = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    _ok(lib.mtm_copy(src.data_ptr(), dst.data_ptr(), nb, 5, st, ctypes.byref(ms)), "mtm_copy")
    out["copy_GBps"] = 2 * nb / (ms.value * 1e6)
    del src, dst
    sink = torch.zeros(1, dtype=torch.int64, device=dev)
    # random 64-bit CAS: 2^22 lanes x 16 swaps per launch
    lanes, per = 1 << 22, 16
    cas = {}
    for label, words in (("l2_2MiB", 1 << 18), ("mall_128MiB", 1 << 24), ("hbm_2GiB", 1 << 28),
                         ("contended_64_words", 64), ("contended_1_word", 1)):
        a = torch.zeros(words, dtype=torch.int64, device=dev)
        lw = lanes if words >= 1024 else lanes // 64  # contended: fewer lanes, the rate is serial anyway
        _ok(lib.mtm_cas(a.data_ptr(), words, lw, per, 3, st, sink.data_ptr(), ctypes.byref(ms)), "mtm_cas")
        cas[label] = lw * per / (ms.value * 1e6)  # Gops/s
        del a
    out["cas_Gops"] = cas
    # LDS CAS: 8 workgroups per CU
    blocks, per = 256 * 8 * 4, 256
    _ok(lib.mtm_lds_cas(blocks, per, 3, st, sink.data_ptr(), ctypes.byref(ms)), "mtm_lds_cas")
    out["lds_cas_Gops"] = blocks * 256 * per / (ms.value * 1e6)
    # dependent loads
    chase = {}
    for label, n in (("l2_2MiB", 1 << 19), ("mall_128MiB", 1 << 25), ("hbm_1GiB", 1 << 28)):
        g = torch.Generator(device=dev)
        g.manual_seed(7)
        perm = torch.randperm(n, device=dev, generator=g, dtype=torch.int64)
        nxt = torch.empty(n, dtype=torch.int32, device=dev)
        nxt[perm] = torch.roll(perm, -1).to(torch.int32)  # one cycle through every entry
        del perm
        res = torch.empty(1 << 22, dtype=torch.int32, device=dev)
        steps = 64
        _ok(lib.mtm_chase(nxt.data_ptr(), n, steps, 256, 3, st, res.data_ptr(), ctypes.byref(ms)), "mtm_chase")
        lat_ns = ms.value * 1e6 / steps
        chains = 1 << 22
        _ok(lib.mtm_chase(nxt.data_ptr(), n, steps, chains, 3, st, res.data_ptr(), ctypes.byref(ms)), "mtm_chase")
        chase[label] = {"latency_ns": lat_ns, "Gloads_per_s": chains * steps / (ms.value * 1e6)}
        del nxt, res
    out["chase"] = chase
    return out
