"""Serial CPU oracle for triplet merge trees -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library (``paper_2301_10838_amd``) never
does, and the two share no code: this wrapper loads ``liboracle.so``, built
from ``oracle.c`` with gcc, and nothing else.

Functions (each follows the passage cited in ``oracle.c``):

- ``merge_tree(f)``: unique normalized, minimal triplets ``T[u] = (s, v)`` of
  the merge tree of ``f`` (Sec. 2.1 sweep; Sec. 2 triplet conditions).
- ``pairs(f, T)``: zero-dimensional persistence pairs, one per branch (Sec. 1).
- ``pairs_scatter``: chain rule of a loss on the pair values (double).
- ``topo_loss(f, tau)``: the simplification loss and its gradient (double).
- ``vertex_ranks(f)``: each vertex's position in the (value, id) order (Sec. 2).
- ``triplets_at(f, us)``: T[u] for sampled vertices u straight from the
  definition (Sec. 2), by a bounded flood from each u, for fields too large
  for the sweep.

Ids are 64-bit throughout (uint64 outputs).

Every value is handled in double precision; float32 fields are widened
exactly before the call, which keeps the order of values unchanged.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_INVALID_ARG, ERR_TOO_LARGE, ERR_NAN, ERR_CAPACITY, ERR_NOMEM = 0, -1, -2, -3, -4, -8


class OracleError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: oracle status {status}")
        self.status = status


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, one thread of work)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_merge_tree.argtypes = [P, I64, I64, I64, P]
        lib.oracle_merge_tree.restype = ctypes.c_int
        lib.oracle_pairs.argtypes = [P, P, I64, P, P, P, P, I64, P]
        lib.oracle_pairs.restype = I64
        lib.oracle_pairs_scatter.argtypes = [I64, P, P, P, P, I64, P]
        lib.oracle_pairs_scatter.restype = ctypes.c_int
        lib.oracle_topo_loss.argtypes = [P, I64, I64, I64, ctypes.c_double, P, P]
        lib.oracle_topo_loss.restype = ctypes.c_int
        lib.oracle_vertex_ranks.argtypes = [P, I64, P]
        lib.oracle_vertex_ranks.restype = ctypes.c_int
        lib.oracle_triplets_at.argtypes = [P, ctypes.c_int, I64, I64, I64, P, I64, I64, P, P, P]
        lib.oracle_triplets_at.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dims(f: np.ndarray):
    """Grid dims (nx, ny, nz) of a C-contiguous [nz][ny][nx] (or lower-rank) array."""
    if f.ndim == 1:
        return f.shape[0], 1, 1
    if f.ndim == 2:
        return f.shape[1], f.shape[0], 1
    if f.ndim == 3:
        return f.shape[2], f.shape[1], f.shape[0]
    raise ValueError("field must be 1-D, 2-D or 3-D")


def _as_f64(f) -> np.ndarray:
    a = np.asarray(f)
    if a.dtype not in (np.float32, np.float64):
        raise TypeError("field must be float32 or float64")
    return np.ascontiguousarray(a, dtype=np.float64)


def merge_tree(f) -> np.ndarray:
    """Triplets of the merge tree of f: uint64 array [N, 2] with T[u] = (s, v)."""
    f64 = _as_f64(f)
    nx, ny, nz = _dims(f64)
    T = np.empty((f64.size, 2), dtype=np.uint64)
    st = _load().oracle_merge_tree(f64.ctypes.data, nx, ny, nz, T.ctypes.data)
    if st != OK:
        raise OracleError(st, "merge_tree")
    return T


def pairs(f, T: np.ndarray):
    """(birth ids, death ids, birth values, death values, n_roots), ascending birth id."""
    f64 = _as_f64(f).reshape(-1)
    T = np.ascontiguousarray(T, dtype=np.uint64).reshape(-1, 2)
    N = f64.size
    lib = _load()
    cap = N // 2 + 1
    b = np.empty(cap, np.uint64)
    d = np.empty(cap, np.uint64)
    bv = np.empty(cap, np.float64)
    dv = np.empty(cap, np.float64)
    nroots = ctypes.c_int64(0)
    p = lib.oracle_pairs(f64.ctypes.data, T.ctypes.data, N, b.ctypes.data, d.ctypes.data,
                         bv.ctypes.data, dv.ctypes.data, cap, ctypes.byref(nroots))
    if p < 0:
        raise OracleError(int(p), "pairs")
    if p > cap:
        raise OracleError(ERR_CAPACITY, "pairs")
    return b[:p].copy(), d[:p].copy(), bv[:p].copy(), dv[:p].copy(), int(nroots.value)


def pairs_scatter(N: int, birth, death, gb, gd, grad=None) -> np.ndarray:
    """grad[birth[k]] += gb[k]; grad[death[k]] += gd[k] in double."""
    birth = np.ascontiguousarray(birth, np.uint64)
    death = np.ascontiguousarray(death, np.uint64)
    gb = np.ascontiguousarray(gb, np.float64)
    gd = np.ascontiguousarray(gd, np.float64)
    g = np.zeros(N, np.float64) if grad is None else np.ascontiguousarray(grad, np.float64)
    st = _load().oracle_pairs_scatter(N, birth.ctypes.data, death.ctypes.data, gb.ctypes.data,
                                      gd.ctypes.data, birth.size, g.ctypes.data)
    if st != OK:
        raise OracleError(st, "pairs_scatter")
    return g


def topo_loss(f, tau: float, want_grad: bool = True):
    """Loss sum_{d-b<tau} (d-b)^2 over the pairs of f and its gradient (double)."""
    f64 = _as_f64(f)
    nx, ny, nz = _dims(f64)
    loss = ctypes.c_double(0.0)
    g = np.empty(f64.shape, np.float64) if want_grad else None
    st = _load().oracle_topo_loss(f64.ctypes.data, nx, ny, nz, float(tau), ctypes.byref(loss),
                                  g.ctypes.data if want_grad else None)
    if st != OK:
        raise OracleError(st, "topo_loss")
    return float(loss.value), g


def vertex_ranks(f) -> np.ndarray:
    """rank[u] = number of vertices preceding u in the (value, id) order; uint64 [N]."""
    f64 = _as_f64(f).reshape(-1)
    r = np.empty(f64.size, np.uint64)
    st = _load().oracle_vertex_ranks(f64.ctypes.data, f64.size, r.ctypes.data)
    if st != OK:
        raise OracleError(st, "vertex_ranks")
    return r


def triplets_at(f, us, max_visit: int = 1 << 20):
    """T[u] for each u in `us` by the definition (a bounded flood from u).

    f: float32 or float64 array (its shape gives the grid).  Returns
    (s, v, ok): uint64 arrays and a bool array; ok[i] is False where the flood
    would add more than max_visit vertices (s[i], v[i] then meaningless)."""
    a = np.asarray(f)
    if a.dtype == np.float32:
        is32, buf = 1, np.ascontiguousarray(a)
    else:
        is32, buf = 0, _as_f64(a)
    nx, ny, nz = _dims(buf)
    us = np.ascontiguousarray(us, dtype=np.int64).reshape(-1)
    s = np.empty(us.size, np.uint64)
    v = np.empty(us.size, np.uint64)
    stat = np.empty(us.size, np.int32)
    st = _load().oracle_triplets_at(buf.ctypes.data, is32, nx, ny, nz, us.ctypes.data, us.size, int(max_visit),
                                    s.ctypes.data, v.ctypes.data, stat.ctypes.data)
    if st != OK:
        raise OracleError(st, "triplets_at")
    if np.any(stat == ERR_NAN):
        raise OracleError(ERR_NAN, "triplets_at")
    return s, v, stat == OK


def build_batch(fields):
    """Per-field oracle over a list of fields (concatenated T, list of pair tuples)."""
    Ts, prs = [], []
    for f in fields:
        T = merge_tree(f)
        Ts.append(T)
        prs.append(pairs(f, T))
    return Ts, prs
