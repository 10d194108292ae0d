"""Pins of the CPU oracle against things other than itself (no GPU needed).

- hand-worked examples (tests/golden/hand_examples.json),
- the definition, via brute-force connectivity of every sublevel set,
  exhaustively over rank permutations on tiny grids,
- closed forms (ramps, constants, checkerboards),
- a library routine (scipy's minimum spanning tree),
- the invariant #pairs = #minima - #components,
- finite differences for the gradient.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import minimum_spanning_tree

import brute
import oracle
from paper_2301_10838_amd import fields

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")


def _examples():
    with open(GOLDEN) as fh:
        return json.load(fh)["examples"]


@pytest.mark.parametrize("ex", _examples(), ids=lambda e: e["name"])
def test_hand_examples(ex):
    f = np.array(ex["values"], dtype=np.float32).reshape(ex["shape"])
    if ex["name"] == "E6_signed_zero":
        f = np.array([0.0, -0.0], dtype=np.float32)
    T = oracle.merge_tree(f)
    assert T.tolist() == ex["T"]
    b, d, bv, dv, nroots = oracle.pairs(f, T)
    assert [[int(x), int(y)] for x, y in zip(b, d)] == ex["pairs"]
    assert [[x, y] for x, y in zip(bv.tolist(), dv.tolist())] == [[float(a), float(c)] for a, c in ex["pair_values"]]
    assert nroots == len(ex["roots"])
    roots = [u for u in range(f.size) if T[u, 0] == u and T[u, 1] == u]
    assert roots == ex["roots"]
    for item in ex.get("loss", []):
        L, g = oracle.topo_loss(f, item["tau"])
        assert L == item["L"]
        want = np.zeros(f.size)
        for k, v in item["grad"].items():
            want[int(k)] = v
        assert np.array_equal(g.ravel(), want)


def test_signed_zero_raw_bits_would_differ():
    # the reading pinned by E6: IEEE equality, not bit order
    T = oracle.merge_tree(np.array([0.0, -0.0], np.float32))
    assert T.tolist() == [[0, 0], [1, 0]]
    T2 = oracle.merge_tree(np.array([-0.0, 0.0], np.float32))
    assert T2.tolist() == [[0, 0], [1, 0]]


SHAPES_TINY = [(5,), (8,), (2, 3), (3, 3), (2, 2, 2), (3, 2, 2), (1, 4), (4, 1), (2, 1, 3), (3, 3, 3), (4, 5), (2, 3, 4)]


@pytest.mark.parametrize("shape", SHAPES_TINY)
def test_brute_force_random(shape):
    rng = np.random.default_rng(hash(shape) % 2**32)
    for trial in range(40):
        if trial % 3 == 0:
            f = rng.integers(0, 3, size=shape).astype(np.float32)  # heavy ties
        elif trial % 3 == 1:
            f = rng.random(shape).astype(np.float32)
        else:
            f = (rng.standard_normal(shape) * 1e3).astype(np.float32)
        assert np.array_equal(oracle.merge_tree(f), brute.brute_triplets(f)), (shape, f.ravel().tolist())


@pytest.mark.parametrize("shape", [(7,), (2, 3), (2, 2, 2)])
def test_brute_force_all_rank_permutations(shape):
    n = int(np.prod(shape))
    for perm in itertools.permutations(range(n)):
        f = np.array(perm, dtype=np.float32).reshape(shape)
        assert np.array_equal(oracle.merge_tree(f), brute.brute_triplets(f)), perm


def test_brute_force_3x3_sampled_permutations():
    rng = np.random.default_rng(7)
    for _ in range(3000):
        f = rng.permutation(9).astype(np.float32).reshape(3, 3)
        assert np.array_equal(oracle.merge_tree(f), brute.brute_triplets(f))


def test_brute_force_5cube():
    rng = np.random.default_rng(11)
    for _ in range(6):
        f = rng.integers(0, 20, size=(5, 5, 5)).astype(np.float32)
        assert np.array_equal(oracle.merge_tree(f), brute.brute_triplets(f))


# -- closed forms -------------------------------------------------------------

@pytest.mark.parametrize("shape", [(10,), (4, 6), (3, 4, 5)])
def test_increasing_ramp(shape):
    n = int(np.prod(shape))
    f = np.arange(n, dtype=np.float32).reshape(shape)
    T = oracle.merge_tree(f)
    assert T[0].tolist() == [0, 0]
    assert all(T[u].tolist() == [u, 0] for u in range(1, n))
    assert oracle.pairs(f, T)[0].size == 0


@pytest.mark.parametrize("shape", [(10,), (4, 6), (3, 4, 5)])
def test_reverse_ramp(shape):
    n = int(np.prod(shape))
    f = np.arange(n, 0, -1, dtype=np.float32).reshape(shape)
    T = oracle.merge_tree(f)
    assert T[n - 1].tolist() == [n - 1, n - 1]
    assert all(T[u].tolist() == [u, n - 1] for u in range(n - 1))


@pytest.mark.parametrize("shape", [(6,), (3, 5), (4, 3, 2)])
def test_constant(shape):
    f = np.full(shape, 2.5, np.float32)
    T = oracle.merge_tree(f)
    n = f.size
    assert T[0].tolist() == [0, 0]
    assert all(T[u].tolist() == [u, 0] for u in range(1, n))


def test_axis_ramp_with_ties():
    nz, ny, nx = 4, 5, 6
    f = np.broadcast_to(np.arange(nx, dtype=np.float32), (nz, ny, nx)).copy()
    T = oracle.merge_tree(f)
    assert T[0].tolist() == [0, 0]
    assert np.all(T[1:, 1] == 0) and np.all(T[1:, 0] == np.arange(1, f.size))


@pytest.mark.parametrize("shape", [(5, 4, 3), (6, 6, 6), (7, 5, 3)])
def test_checkerboard_3d(shape):
    z, y, x = np.indices(shape)
    f = ((x + y + z) % 2).astype(np.float32)
    T = oracle.merge_tree(f)
    b, d, _, _, nroots = oracle.pairs(f, T)
    n = f.size
    assert nroots == 1 and T[0].tolist() == [0, 0]
    assert b.size == math.ceil(n / 2) - 1
    even = ((x + y + z) % 2 == 0).ravel()
    assert set(b.tolist()) == set(np.nonzero(even)[0].tolist()) - {0}
    # every even vertex other than 0 dies at its first odd neighbour in id order
    assert np.all(~even[d])


@pytest.mark.parametrize("shape", [(5, 7), (6, 6), (9, 4)])
def test_egg_crate_2d(shape):
    y, x = np.indices(shape)
    f = ((x % 2) + (y % 2)).astype(np.float32)
    T = oracle.merge_tree(f)
    b, d, _, _, nroots = oracle.pairs(f, T)
    ny, nx = shape
    assert b.size == math.ceil(nx / 2) * math.ceil(ny / 2) - 1
    assert nroots == 1


# -- library routine: minimum spanning tree -------------------------------------

def _mst_check(f):
    f = np.asarray(f)
    N = f.size
    order = np.lexsort((np.arange(N), f.ravel().astype(np.float64)))
    rank = np.empty(N, np.int64)
    rank[order] = np.arange(N)
    ids = np.arange(N).reshape(f.shape)
    rows, cols, w = [], [], []
    for ax in range(f.ndim):
        if f.shape[ax] < 2:
            continue
        lo = [slice(None)] * f.ndim
        hi = [slice(None)] * f.ndim
        lo[ax] = slice(0, f.shape[ax] - 1)
        hi[ax] = slice(1, f.shape[ax])
        a = ids[tuple(lo)].ravel()
        b = ids[tuple(hi)].ravel()
        rows.append(a)
        cols.append(b)
        w.append(1.0 + np.maximum(rank[a], rank[b]))
    rows, cols, w = np.concatenate(rows), np.concatenate(cols), np.concatenate(w)
    G = coo_matrix((w, (rows, cols)), shape=(N, N)).tocsr()
    mst = minimum_spanning_tree(G)
    mst_w = np.sort(mst.data - 1.0).astype(np.int64)

    T = oracle.merge_tree(f)
    b, d, _, _, _ = oracle.pairs(f, T)
    regular = np.nonzero((T[:, 0] == np.arange(N)) & (T[:, 1] != np.arange(N)))[0]
    want = np.sort(np.concatenate([rank[regular], rank[d.astype(np.int64)]]))
    assert np.array_equal(mst_w, want)


@pytest.mark.parametrize("maker", ["uniform", "ties", "bumps"])
def test_mst_death_vertices(maker):
    if maker == "uniform":
        f = fields.uniform((16, 16, 16), 21)
    elif maker == "ties":
        f = np.random.default_rng(3).integers(0, 5, size=(12, 10, 8)).astype(np.float32)
    else:
        f = fields.bumps((24, 24, 24), 22, n_bumps=6, sigma=(2, 5))
    _mst_check(f)


def test_mst_2d():
    _mst_check(fields.lognormal_grf((64, 48), 23))


# -- invariant -------------------------------------------------------------------

@pytest.mark.parametrize("name,maker", [
    ("uniform64", lambda: fields.workload("uniform64")[0]),
    ("grf32", lambda: fields.lognormal_grf((32, 32, 32), 9)),
    ("grf2d", lambda: fields.lognormal_grf((200, 150), 10)),
    ("bumps", lambda: fields.bumps((40, 40, 40), 12)),
])
def test_pairs_equal_minima_minus_components(name, maker):
    f = maker()
    T = oracle.merge_tree(f)
    b, d, bv, dv, nroots = oracle.pairs(f, T)
    assert nroots == brute.count_components(f.shape) == 1
    assert b.size == brute.count_minima(f) - 1
    assert np.all(bv <= dv)
    # births strictly ascending, values are bit copies
    assert np.all(np.diff(b.astype(np.int64)) > 0)
    assert np.array_equal(bv, f.ravel()[b].astype(np.float64))
    assert np.array_equal(dv, f.ravel()[d].astype(np.float64))


def test_uniform64_minimum_count_statistics():
    # i.i.d. values: a vertex is a minimum with probability 1/(deg+1)
    n = 64
    f = fields.workload("uniform64")[0]
    inner = (n - 2) ** 3
    faces = 6 * (n - 2) ** 2
    edges = 12 * (n - 2)
    expect = inner / 7 + faces / 6 + edges / 5 + 8 / 4
    got = brute.count_minima(f)
    assert abs(got - expect) < 5 * math.sqrt(expect)


# -- gradient --------------------------------------------------------------------

def test_gradient_matches_finite_differences():
    tau = 0.05
    h = 1e-7
    checked = 0
    for i in range(8):
        f32 = fields.generic_fd_field((16, 16, 16), 6000 + i)
        f = f32.astype(np.float64)
        flat = f.ravel()
        T = oracle.merge_tree(f)
        b, d, bv, dv, _ = oracle.pairs(f, T)
        pers = dv - bv
        # genericity: distinct values, and no persistence near the threshold
        if np.unique(flat).size != flat.size or np.any(np.abs(pers - tau) < 10 * h):
            continue
        L, g = oracle.topo_loss(f, tau)
        g = g.ravel()
        support = np.unique(np.concatenate([b[pers < tau], d[pers < tau]])).astype(np.int64)
        rng = np.random.default_rng(i)
        probe = np.unique(np.concatenate([support, rng.choice(flat.size, 64, replace=False)]))
        gfd = np.zeros(flat.size)
        for j in probe:
            fp = flat.copy(); fp[j] += h
            fm = flat.copy(); fm[j] -= h
            Lp, _ = oracle.topo_loss(fp.reshape(f.shape), tau, want_grad=False)
            Lm, _ = oracle.topo_loss(fm.reshape(f.shape), tau, want_grad=False)
            gfd[j] = (Lp - Lm) / (2 * h)
        scale = np.max(np.abs(gfd))
        assert scale > 0
        assert np.max(np.abs(g[probe] - gfd[probe])) <= 1e-4 * scale
        assert set(np.nonzero(np.abs(gfd) > 1e-6 * scale)[0].tolist()) == set(np.nonzero(g)[0].tolist())
        checked += 1
    assert checked >= 4


def test_pairs_scatter_matches_topo_loss_gradient():
    f = fields.generic_fd_field((12, 12, 12), 77).astype(np.float64)
    T = oracle.merge_tree(f)
    b, d, bv, dv, _ = oracle.pairs(f, T)
    pers = dv - bv
    m = pers < 0.05
    gb = np.where(m, -2 * pers, 0.0)
    gd = np.where(m, 2 * pers, 0.0)
    g = oracle.pairs_scatter(f.size, b, d, gb, gd)
    _, g2 = oracle.topo_loss(f, 0.05)
    assert np.allclose(g, g2.ravel(), rtol=0, atol=1e-15)


# -- error paths -------------------------------------------------------------------

def test_nan_rejected():
    f = np.zeros((3, 3), np.float32)
    f[1, 2] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.merge_tree(f)
    assert e.value.status == oracle.ERR_NAN


def test_infinities_are_values():
    f = np.array([np.inf, 1.0, -np.inf, 0.0], np.float32)
    assert np.array_equal(oracle.merge_tree(f), brute.brute_triplets(f))


def test_empty_rejected():
    with pytest.raises(oracle.OracleError) as e:
        oracle.merge_tree(np.zeros((0,), np.float32))
    assert e.value.status == oracle.ERR_INVALID_ARG


def test_single_vertex():
    T = oracle.merge_tree(np.array([3.0], np.float32))
    assert T.tolist() == [[0, 0]]


# --- vertex ranks (the (value, id) order of Sec. 2 as integer keys) ---------

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_vertex_ranks_brute_force(seed):
    """rank[u] = #{w : f[w] < f[u] or (f[w] == f[u] and w < u)}, counted
    directly on small fields with repeated values and both signed zeros."""
    rng = np.random.default_rng(seed)
    f = rng.integers(-3, 4, 400).astype(np.float32)
    f[rng.random(400) < 0.1] = -0.0
    f[rng.random(400) < 0.05] = np.inf
    r = oracle.vertex_ranks(f)
    fv = f.astype(np.float64)
    ids = np.arange(f.size)
    before = (fv[None, :] < fv[:, None]) | ((fv[None, :] == fv[:, None]) & (ids[None, :] < ids[:, None]))
    assert np.array_equal(r, before.sum(axis=1).astype(np.uint32))


def test_vertex_ranks_permutation_and_reversal():
    rng = np.random.default_rng(7)
    f = rng.standard_normal(1000).astype(np.float32)  # distinct values
    r = oracle.vertex_ranks(f)
    assert np.array_equal(np.sort(r), np.arange(f.size, dtype=np.uint32))
    # distinct values: the order of -f is the reverse order
    assert np.array_equal(oracle.vertex_ranks(-f), (f.size - 1 - r).astype(np.uint32))
    # a constant field is ordered by id alone
    assert np.array_equal(oracle.vertex_ranks(np.full(50, 2.5, np.float32)), np.arange(50, dtype=np.uint32))


def test_vertex_ranks_nan_rejected():
    with pytest.raises(oracle.OracleError):
        oracle.vertex_ranks(np.array([1.0, np.nan], np.float32))


# --- 64-bit ids --------------------------------------------------------------

def test_ids_are_64_bit():
    """Every id the oracle returns is uint64, and the sweep's values do not
    depend on the width (the hand example E4 as uint64)."""
    f = np.array([5, 1, 6, 2, 9, 3, 7, 4, 8], np.float32).reshape(3, 3)
    T = oracle.merge_tree(f)
    assert T.dtype == np.uint64
    b, d, _, _, _ = oracle.pairs(f, T)
    assert b.dtype == np.uint64 and d.dtype == np.uint64
    assert T.tolist() == [[0, 1], [1, 1], [2, 1], [0, 1], [4, 1], [2, 1], [6, 1], [6, 1], [8, 1]]
    assert oracle.vertex_ranks(f).dtype == np.uint64


# --- one triplet from its definition (the flood), against the sweep -----------

@pytest.mark.parametrize("maker", [
    lambda: fields.uniform((9, 10, 11), 1),
    lambda: fields.lognormal_grf((20, 21, 22), 2),
    lambda: np.random.default_rng(3).integers(0, 3, (7, 8, 9)).astype(np.float32),
    lambda: fields.plateau_jump((10, 11, 12), 4),
    lambda: fields.lognormal_grf((60, 70), 5),
    lambda: fields.uniform((300,), 6),
    lambda: np.array([[np.inf, 0.0, -0.0, 1.0], [-np.inf, -0.0, 0.0, np.inf]], np.float32),
    lambda: fields.serpentine((6, 7, 9), 7),
])
def test_triplets_at_equals_sweep_everywhere(maker):
    """The flood computes every triplet of small fields exactly as the sweep
    does: two independent constructions of the same definition (a sorted
    union-find sweep over the whole field, and a priority flood from one
    vertex), in float32 and float64 input."""
    f = maker()
    T = oracle.merge_tree(f)
    us = np.arange(f.size)
    for arr in (f, f.astype(np.float64)):
        s, v, ok = oracle.triplets_at(arr, us, max_visit=1 << 16)
        assert ok.all()
        assert np.array_equal(s, T[:, 0]) and np.array_equal(v, T[:, 1])


def test_triplets_at_reports_budget():
    """A flood that would add more than max_visit vertices is flagged, not
    answered; the ones that fit agree with the sweep."""
    f = fields.lognormal_grf((40, 40, 40), 8)
    T = oracle.merge_tree(f)
    us = np.random.default_rng(9).integers(0, f.size, 500)
    s, v, ok = oracle.triplets_at(f, us, max_visit=64)
    assert 0 < ok.sum() < ok.size
    assert np.array_equal(s[ok], T[us[ok], 0]) and np.array_equal(v[ok], T[us[ok], 1])
    with pytest.raises(oracle.OracleError):
        oracle.triplets_at(np.array([1.0, np.nan, 0.5], np.float32), [0, 1, 2])


# --- closed forms of the adversarial generators --------------------------------

def test_parity_lattice_minima():
    """(x mod 2) + (y mod 2) + (z mod 2): the all-even vertices are exactly the
    minima, so #pairs = ceil(nx/2) ceil(ny/2) ceil(nz/2) - 1."""
    for shape in [(6, 7, 9), (5, 5, 5), (2, 9, 4)]:
        f = fields.parity_lattice(shape)
        T = oracle.merge_tree(f)
        b, _, _, _, roots = oracle.pairs(f, T)
        want = int(np.prod([(n + 1) // 2 for n in shape])) - 1
        assert b.size == want and roots == 1
        z, y, x = np.unravel_index(b.astype(np.int64), shape)
        assert np.all((x % 2 == 0) & (y % 2 == 0) & (z % 2 == 0))


def test_tilted_checkerboard_minima():
    """Every even-parity vertex is a minimum (all its neighbours sit one unit
    higher), so #pairs = ceil(N/2) - 1, and the global minimum is vertex 0."""
    for shape in [(7, 8, 9), (11, 13)]:
        f = fields.tilted_checkerboard(shape, 3)
        T = oracle.merge_tree(f)
        b, _, _, _, roots = oracle.pairs(f, T)
        assert b.size == (f.size + 1) // 2 - 1 and roots == 1
        assert T[0].tolist() == [0, 0]


def test_serpentine_2d_single_branch():
    """In 2-D every vertex off the path touches it, so the path's start is the
    only minimum: no pairs, and every vertex's target is the start (its
    reverse for the descending path)."""
    f = fields.serpentine((9, 12), 5)
    T = oracle.merge_tree(f)
    assert oracle.pairs(f, T)[0].size == 0
    assert np.all(T[:, 1] == 0)
    g = fields.serpentine((9, 12), 5, descending=True)
    Tg = oracle.merge_tree(g)
    end = int(np.argmin(g))
    assert oracle.pairs(g, Tg)[0].size == 0 and np.all(Tg[:, 1] == end)
