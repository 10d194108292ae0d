"""Interleaving simulator of the lock-free triplet merge tree algorithm.

Test infrastructure.  It runs the parallel algorithm of Sec. 2 (Alg. 1: init,
merge every edge, repair every vertex; Alg. 2 CAS; Alg. 3 Merge; Alg. 4
Representative; Alg. 5 Repair) with each logical thread written as a Python
generator that yields before every access to the shared map T.  A seeded
scheduler picks which thread advances next, so every run is one sequentially
consistent interleaving of the threads' atomic steps; phases are separated
as in Alg. 1.

Readings of the printed pseudocode that the simulator implements (and that
the tests below pin against the oracle):

- Descents stop at roots: a triplet (x, x, x) has no lower vertex to move to,
  and following it would loop forever.
- After a successful CAS that replaced a root (v, v, v), no displaced
  triplet needs to be merged again; merging (u, v, v) again would assert a
  connection at the level of v that does not hold.
- Representative returns the last vertex reached by the chase (the deepest
  vertex found), not the target stored in that vertex's triplet.

Variants used by the GPU design, each checked to give the same unique T:

- ``prelink``: every non-minimum first points at its lowest lower neighbour,
  T[u] = (u, w(u)), which is the state reached by merging those edges one
  after another in decreasing order of their upper vertex; the remaining
  edges are merged as usual.
- ``basins``: as prelink, with the pointer chains compressed to the minimum
  z(u) reached by steepest descent, T[u] = (u, z(u)); an edge whose ends
  descend to the same minimum is already implied and is skipped, and the
  other edges are merged between the two minima, Merge(z(a), max(a, b), z(b)).
- ``tiles``: as basins, in two levels.  The grid is cut into boxes and every
  minimum belongs to the box holding it.  First, for every box on its own,
  the edges owned by the box's vertices whose two minima both belong to that
  box are merged (interleaved within the box), then those minima are
  repaired; every other edge is merged afterwards, and a final repair runs
  over all vertices.
- ``tile_trees``: the grid is cut into boxes; every box first builds the
  merge tree of its own subgraph (steepest descent inside the box, chains
  compressed to the box-local minimum, every edge inside the box merged
  between box-local minima, then those minima repaired); afterwards the
  edges that cross box faces are merged between the box-local minima of
  their ends, and a final repair runs over all vertices.
- ``tile_trees_lowest``: as tile_trees, but of all edges joining the same two
  basins only the one with the lowest upper end is merged (inside a box, and
  across each box face): a connection at a lower level implies the same
  connection at every higher one, so the others add nothing.

Any variant can also run its merges with path compression in the descents
(``compress_after``, see merge_thread).
"""
from __future__ import annotations

import random

import numpy as np


class LivelockError(RuntimeError):
    pass


def _keyer(flat):
    def key(x):
        return (float(flat[x]), int(x))
    return key


def grid_edges(shape):
    """Axis edges of a C-order grid of the given numpy shape, as (a, b) id pairs."""
    ids = np.arange(int(np.prod(shape))).reshape(shape)
    edges = []
    for ax in range(len(shape)):
        if shape[ax] < 2:
            continue
        lo = [slice(None)] * len(shape)
        hi = [slice(None)] * len(shape)
        lo[ax] = slice(0, shape[ax] - 1)
        hi[ax] = slice(1, shape[ax])
        a = ids[tuple(lo)].ravel()
        b = ids[tuple(hi)].ravel()
        edges.extend(zip(a.tolist(), b.tolist()))
    return edges


def neighbours(shape):
    nb = {u: [] for u in range(int(np.prod(shape)))}
    for a, b in grid_edges(shape):
        nb[a].append(b)
        nb[b].append(a)
    return nb


# -- threads ---------------------------------------------------------------

def merge_thread(T, key, u, s, v, root_guard=True, skip_root_remerge=True, cap=100000, compress_after=None):
    """Alg. 3 as a loop (its recursion is a tail call), yielding before each T access.

    compress_after (None: off) adds path compression to the descents once the
    merge has taken that many descent steps: when a descent passes x -> y (at
    saddle sx) and then y -> z at a saddle sy not above sx, x is re-pointed
    at z at its own saddle by a compare-and-swap, (sx, y) -> (sx, z).  x and z
    are connected at the level of sx through y, and z lies below y, so this is
    one step of Repair's chase (Alg. 4) written back early; a swap that finds
    x changed does nothing.
    """
    ks = key(s)
    prev = [None, None]  # per side: (x, sx, y) of the link just followed
    steps = 0
    for _ in range(cap):
        yield
        su, u1 = T[u]
        u_root = (u1 == u) and (su == u)
        if (not u_root or not root_guard) and key(su) < ks:
            steps += 1
            if compress_after is not None and steps > compress_after and prev[0] is not None:
                x, sx, y = prev[0]
                if y == u and key(su) <= key(sx):
                    yield
                    if T[x] == (sx, y):
                        T[x] = (sx, u1)
            prev[0] = (u, su, u1)
            u = u1
            continue
        yield
        sv, v1 = T[v]
        v_root = (v1 == v) and (sv == v)
        if (not v_root or not root_guard) and key(sv) < ks:
            steps += 1
            if compress_after is not None and steps > compress_after and prev[1] is not None:
                x, sx, y = prev[1]
                if y == v and key(sv) <= key(sx):
                    yield
                    if T[x] == (sx, y):
                        T[x] = (sx, v1)
            prev[1] = (v, sv, v1)
            v = v1
            continue
        if u == v:
            return
        if key(v) < key(u):
            u, v = v, u
            su, u1, sv, v1 = sv, v1, su, u1
            prev = [prev[1], prev[0]]
        yield
        if T[v] == (sv, v1):  # CAS, atomic in one scheduler step
            T[v] = (s, u)
            if skip_root_remerge and v1 == v and sv == v:
                return
            s, v = sv, v1
            ks = key(s)
            prev[1] = None
        # CAS failed: start again with the same (u, s, v)
    raise LivelockError("merge exceeded step cap")


def repair_thread(T, key, u, return_last=True, cap=100000):
    """Alg. 5 with Alg. 4 inlined; yields before each T access."""
    yield
    s, v = T[u]
    ks = key(s)
    x = u
    sx, vx = s, v
    for _ in range(cap):
        if (vx == x and sx == x) or key(sx) > ks:
            break
        x = vx
        yield
        sx, vx = T[x]
    else:
        raise LivelockError("repair exceeded step cap")
    r = x if return_last else vx
    if r != u:
        yield
        T[u] = (s, r)


def run_phase(threads, rng, max_steps=10_000_000):
    live = list(threads)
    steps = 0
    while live:
        i = rng.randrange(len(live))
        try:
            next(live[i])
        except StopIteration:
            live[i] = live[-1]
            live.pop()
        steps += 1
        if steps > max_steps:
            raise LivelockError("phase exceeded step cap")


# -- the algorithm and its variants ---------------------------------------

def steepest_lower(flat, shape):
    key = _keyer(flat)
    nb = neighbours(shape)
    w = np.arange(flat.size)
    for u in range(flat.size):
        best = u
        for x in nb[u]:
            if key(x) < key(best):
                best = x
        w[u] = best
    return w


def _box_of(shape, box):
    """Box index of every vertex for a box shape given in (x, y, z) order."""
    idx = np.indices(shape)  # (z, y, x) or lower rank, numpy axis order
    nd = len(shape)
    coords = [idx[nd - 1 - d] // box[d] for d in range(nd)]  # x, y, z
    nb = [(shape[nd - 1 - d] + box[d] - 1) // box[d] for d in range(nd)]
    b = np.zeros(shape, dtype=np.int64)
    mul = 1
    for d in range(nd):
        b += coords[d] * mul
        mul *= nb[d]
    return b.ravel()


def simulate(f, seed=0, variant="paper", edge_order=None, serial=False,
             root_guard=True, skip_root_remerge=True, return_last=True, box=(2, 2, 2), compress_after=None):
    """Run Alg. 1 (or a variant) under one seeded interleaving; returns T [N, 2]."""
    f = np.asarray(f)
    shape = f.shape
    flat = f.ravel().astype(np.float64)
    N = flat.size
    key = _keyer(flat)
    rng = random.Random(seed)
    edges = list(edge_order) if edge_order is not None else grid_edges(shape)
    if edge_order is None:
        rng.shuffle(edges)

    T = [(u, u) for u in range(N)]
    merges = []
    if variant == "paper":
        for a, b in edges:
            hi, lo = (a, b) if key(b) < key(a) else (b, a)
            merges.append((hi, hi, lo))
    elif variant in ("tile_trees", "tile_trees_lowest"):
        bx = _box_of(shape, box[: len(shape)])
        nb = neighbours(shape)
        zl = np.arange(N)
        for u in range(N):  # steepest descent inside the box
            best = u
            for x in nb[u]:
                if bx[x] == bx[u] and key(x) < key(best):
                    best = x
            zl[u] = best
        for u in range(N):
            T[u] = (u, int(zl[u])) if zl[u] != u else (u, u)
        for it in range(N):
            z2 = zl[zl]
            if np.array_equal(z2, zl):
                break
            zl = z2
        for u in range(N):
            if zl[u] != u:
                T[u] = (u, int(zl[u]))
        local = {}
        lowest = {}
        for a, b in edges:
            hi = a if key(b) < key(a) else b
            m = (int(zl[a]), hi, int(zl[b]))
            if variant == "tile_trees_lowest":
                if zl[a] == zl[b]:
                    continue
                pair = (min(m[0], m[2]), max(m[0], m[2]))
                if pair not in lowest or key(hi) < key(lowest[pair][1]):
                    lowest[pair] = m
                continue
            if bx[a] == bx[b]:
                if zl[a] != zl[b]:
                    local.setdefault(int(bx[a]), []).append(m)
            else:
                merges.append(m)
        for pair, m in lowest.items():
            if bx[m[0]] == bx[m[2]]:
                local.setdefault(int(bx[m[0]]), []).append(m)
            else:
                merges.append(m)
        boxes = list(local.items())
        rng.shuffle(boxes)
        for bidx, ms in boxes:
            th = [merge_thread(T, key, u, s_, v, root_guard, skip_root_remerge, compress_after=compress_after)
                  for (u, s_, v) in ms]
            run_phase(th, rng)
            mins = [u for u in range(N) if zl[u] == u and bx[u] == bidx]
            run_phase([repair_thread(T, key, u, return_last) for u in mins], rng)
    elif variant in ("prelink", "basins", "tiles"):
        w = steepest_lower(flat, shape)
        for u in range(N):
            T[u] = (u, int(w[u])) if w[u] != u else (u, u)
        if variant == "prelink":
            for a, b in edges:
                hi, lo = (a, b) if key(b) < key(a) else (b, a)
                if w[hi] == lo:
                    continue  # already merged by the pre-link
                merges.append((hi, hi, lo))
        else:
            z = w.copy()
            for u in range(N):
                x = u
                while z[x] != x:
                    x = z[x]
                z[u] = x
            for u in range(N):
                if z[u] != u:
                    T[u] = (u, int(z[u]))
            if variant == "basins":
                for a, b in edges:
                    if z[a] == z[b]:
                        continue  # implied by the two descents
                    hi = a if key(b) < key(a) else b
                    merges.append((int(z[a]), hi, int(z[b])))
            else:
                bx = _box_of(shape, box[: len(shape)])
                local = {}
                for a, b in edges:
                    if z[a] == z[b]:
                        continue
                    hi = a if key(b) < key(a) else b
                    own = min(a, b)  # the edge belongs to its lower-id end's box
                    m = (int(z[a]), hi, int(z[b]))
                    if bx[z[a]] == bx[own] and bx[z[b]] == bx[own]:
                        local.setdefault(int(bx[own]), []).append(m)
                    else:
                        merges.append(m)
                boxes = list(local.items())
                rng.shuffle(boxes)
                for bidx, ms in boxes:
                    th = [merge_thread(T, key, u, s_, v, root_guard, skip_root_remerge, compress_after=compress_after)
                  for (u, s_, v) in ms]
                    run_phase(th, rng)
                    mins = [u for u in range(N) if z[u] == u and bx[u] == bidx]
                    run_phase([repair_thread(T, key, u, return_last) for u in mins], rng)
    else:
        raise ValueError(variant)

    def mk_merges():
        return [merge_thread(T, key, u, s, v, root_guard, skip_root_remerge, compress_after=compress_after)
                for (u, s, v) in merges]

    if serial:
        for th in mk_merges():
            for _ in th:
                pass
        for u in range(N):
            for _ in repair_thread(T, key, u, return_last):
                pass
    else:
        run_phase(mk_merges(), rng)
        run_phase([repair_thread(T, key, u, return_last) for u in range(N)], rng)
    return np.array(T, dtype=np.uint32)
