"""Definition-level brute force for merge-tree triplets on tiny grids.

Test infrastructure.  It shares nothing with the oracle's sweep: connectivity
of every sublevel set comes from ``scipy.ndimage.label`` (a library
connected-components routine), recomputed from scratch at every level.

By the definitions of Sec. 2 (triplet merge trees) and Sec. 2.1 (sublevel sets
G_c): for a vertex u, look at u's component in the sublevel set at increasing
levels, starting at u's own level.  At the first level lam whose component
holds a vertex deeper than u, the triplet is (u, lam, deepest vertex of that
component): lam == u for a vertex that is not a minimum (degree two in the
merge tree), lam is the saddle where u's branch dies for a minimum.  A vertex
whose component never gains a deeper vertex is the global minimum of its
connected component: (u, u, u).

Ties are broken by the linear id, as everywhere in this package.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage


def order_of(f: np.ndarray) -> np.ndarray:
    flat = np.asarray(f, dtype=np.float64).ravel()
    # Python float comparison treats -0.0 == 0.0, so the id decides between them.
    return np.array(sorted(range(flat.size), key=lambda i: (float(flat[i]), i)), dtype=np.int64)


def brute_triplets(f: np.ndarray) -> np.ndarray:
    f = np.asarray(f)
    N = f.size
    order = order_of(f)
    rank = np.empty(N, dtype=np.int64)
    rank[order] = np.arange(N)
    structure = ndimage.generate_binary_structure(max(f.ndim, 1), 1)
    T = np.full((N, 2), -1, dtype=np.int64)
    for k in range(N):
        mask = (rank <= k).reshape(f.shape)
        lab, nlab = ndimage.label(mask, structure=structure)
        lab = lab.ravel()
        # deepest vertex (smallest rank) of every component at this level
        deep_rank = np.full(nlab + 1, N, dtype=np.int64)
        np.minimum.at(deep_rank, lab[mask.ravel()], rank[mask.ravel()])
        level_vertex = order[k]
        for u in order[: k + 1]:
            if T[u, 0] >= 0:
                continue
            d = deep_rank[lab[u]]
            if d < rank[u]:
                T[u] = (level_vertex, order[d])
    for u in range(N):
        if T[u, 0] < 0:
            T[u] = (u, u)
    return T.astype(np.uint32)


def count_minima(f: np.ndarray) -> int:
    """Vertices with no axis neighbour preceding them (independent neighbour test)."""
    f = np.asarray(f, dtype=np.float64)
    ids = np.arange(f.size).reshape(f.shape)
    is_min = np.ones(f.shape, dtype=bool)
    for ax in range(f.ndim):
        n = f.shape[ax]
        if n < 2:
            continue
        lo = [slice(None)] * f.ndim
        hi = [slice(None)] * f.ndim
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        lo, hi = tuple(lo), tuple(hi)
        # the neighbour at lo precedes the vertex at hi?
        prec_lo = (f[lo] < f[hi]) | ((f[lo] == f[hi]) & (ids[lo] < ids[hi]))
        is_min[hi] &= ~prec_lo
        prec_hi = (f[hi] < f[lo]) | ((f[hi] == f[lo]) & (ids[hi] < ids[lo]))
        is_min[lo] &= ~prec_hi
    return int(is_min.sum())


def count_components(shape) -> int:
    """A regular grid with every axis edge present is connected."""
    return 1
