/*
 * oracle.c -- serial CPU reference for merge trees on regular grids.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into its own shared
 * library (liboracle.so) and is loaded solely by the test suite, by the
 * smoke check and by the CPU-baseline leg of the benchmark.  The product
 * library never includes, links or calls it, and it shares no header, helper,
 * table or constant generator with the HIP code.  The only thing the two
 * agree on is the numbering of status codes, which each side writes down on
 * its own.
 *
 * What it computes, each by its plain definition rather than by the
 * parallel algorithm the product implements:
 *
 *  1. The merge tree of f on the grid graph (paper Sec. 2.1, "Merge trees").
 *     The vertices are visited in increasing order of f; a union-find
 *     structure tells, for each vertex, which of the three cases of that
 *     section holds: it starts a new component (a local minimum), it joins
 *     exactly one existing component, or it merges several.
 *
 *  2. The unique normalized and minimal triplet representation of that tree
 *     (paper Sec. 2, "Triplet merge trees"): every vertex u is the first
 *     vertex of exactly one triplet (u, s, v), stored as T[u] = (s, v), and v
 *     is the deepest vertex of u's component of the sublevel set at the level
 *     of s.  A global minimum of a component is the triplet (u, u, u); a
 *     vertex of degree two in the merge tree is (u, u, v).  When several
 *     components meet at a vertex, every component except the one holding
 *     the deepest vertex ends there (its branch dies), which is what the
 *     minimality condition forces.
 *
 *  3. The zero-dimensional persistence pairs, one per branch (paper Sec. 1):
 *     the branch born at minimum u that dies at saddle s gives the point
 *     (f(u), f(s)).  In triplet terms these are exactly the u with s != u.
 *     Branches that never die (one per connected component) are counted as
 *     roots and are not pairs.
 *
 *  4. The gradient, in double precision, of a loss written on the pairs with
 *     respect to the field values: the birth value of a pair is f at its
 *     minimum and the death value is f at its saddle, so the upstream
 *     derivatives land on those two vertices (the scatter is the chain rule
 *     and nothing else).
 *
 *  5. One triplet by itself, straight from its definition (Sec. 2), for
 *     checking samples of outputs too large for the sweep: a flood from u
 *     that always takes the lowest vertex on its boundary visits u's
 *     component of every sublevel set in turn, so the level at which it first
 *     reaches a vertex deeper than u is u's saddle, and the deepest vertex it
 *     has met by the time the boundary rises above that level is the
 *     triplet's target.
 *
 * Conventions.
 *  - Grid: nx*ny*nz vertices stored C-contiguous as [nz][ny][nx]; vertex id
 *    u = x + nx*(y + ny*z).  Edges join axis neighbours (6 in 3-D, 4 when
 *    nz == 1, 2 when also ny == 1), the grid graph of Sec. 1.
 *  - Order: u precedes w iff f(u) < f(w), or f(u) == f(w) and u < w.  The
 *    comparison is the IEEE one, so -0.0 and +0.0 compare equal and the id
 *    decides.  The paper writes strict inequalities assuming distinct values;
 *    this index tie-break is the reading taken where values repeat.
 *  - NaN anywhere is an error; +-Inf are ordinary values.
 *  - Ids are 64-bit here (uint64_t in every output), so no field size is
 *    excluded by the id width; the paper's GPU layout packs two 32-bit ids
 *    into one word (Sec. 3.2) and names wider ids as future work (Sec. 5).
 *
 * All arithmetic on values is double; float input is converted exactly by
 * the Python wrapper before it gets here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Status codes (same numbers as the product library, written out here). */
#define OR_OK 0
#define OR_ERR_INVALID_ARG (-1)
#define OR_ERR_TOO_LARGE (-2)
#define OR_ERR_NAN (-3)
#define OR_ERR_CAPACITY (-4)
#define OR_ERR_NOMEM (-8)

/* The total order on vertices: value first, then id. */
static int precedes(const double *f, int64_t a, int64_t b)
{
    return f[a] < f[b] || (f[a] == f[b] && a < b);
}

typedef struct {
    double val;
    uint64_t id;
} keyed;

static int cmp_keyed(const void *pa, const void *pb)
{
    const keyed *a = (const keyed *)pa;
    const keyed *b = (const keyed *)pb;
    if (a->val < b->val) return -1;
    if (a->val > b->val) return 1;
    return (a->id < b->id) ? -1 : (a->id > b->id) ? 1 : 0;
}

/* Union-find with union by size and path halving. */
static uint64_t uf_find(uint64_t *parent, uint64_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

static int validate(int64_t nx, int64_t ny, int64_t nz)
{
    if (nx < 1 || ny < 1 || nz < 1) return OR_ERR_INVALID_ARG;
    /* keep N and its byte counts inside 64-bit arithmetic */
    if (nx >= (1LL << 40) || ny >= (1LL << 40) || nz >= (1LL << 40)) return OR_ERR_TOO_LARGE;
    if (nx * ny >= (1LL << 40) || (nx * ny) * nz >= (1LL << 40)) return OR_ERR_TOO_LARGE;
    return OR_OK;
}

/*
 * Rank of every vertex in the total order above (Sec. 2: value, then id):
 * rank[u] = the number of vertices that precede u.  These are the keys a
 * rank-keyed build would compare instead of values.
 */
int oracle_vertex_ranks(const double *f, int64_t N, uint64_t *rank)
{
    if (!f || !rank || N < 1) return OR_ERR_INVALID_ARG;
    if (N >= (1LL << 40)) return OR_ERR_TOO_LARGE;
    for (int64_t i = 0; i < N; ++i)
        if (isnan(f[i])) return OR_ERR_NAN;
    keyed *order = (keyed *)malloc((size_t)N * sizeof(keyed));
    if (!order) return OR_ERR_NOMEM;
    for (int64_t i = 0; i < N; ++i) {
        order[i].val = f[i];
        order[i].id = (uint64_t)i;
    }
    qsort(order, (size_t)N, sizeof(keyed), cmp_keyed);
    for (int64_t i = 0; i < N; ++i) rank[order[i].id] = (uint64_t)i;
    free(order);
    return OR_OK;
}

/*
 * Merge tree of f by the sorted union-find sweep of Sec. 2.1, written out as
 * its triplet representation (Sec. 2).  T receives 2*N uint64: T[2u] = s,
 * T[2u+1] = v.
 */
int oracle_merge_tree(const double *f, int64_t nx, int64_t ny, int64_t nz, uint64_t *T)
{
    int st = validate(nx, ny, nz);
    if (st != OR_OK) return st;
    if (!f || !T) return OR_ERR_INVALID_ARG;
    const int64_t N = nx * ny * nz;
    for (int64_t i = 0; i < N; ++i)
        if (isnan(f[i])) return OR_ERR_NAN;

    keyed *order = (keyed *)malloc((size_t)N * sizeof(keyed));
    uint64_t *parent = (uint64_t *)malloc((size_t)N * sizeof(uint64_t));
    uint64_t *size = (uint64_t *)malloc((size_t)N * sizeof(uint64_t));
    uint64_t *deepest = (uint64_t *)malloc((size_t)N * sizeof(uint64_t)); /* valid at set roots */
    if (!order || !parent || !size || !deepest) {
        free(order); free(parent); free(size); free(deepest);
        return OR_ERR_NOMEM;
    }
    for (int64_t i = 0; i < N; ++i) {
        order[i].val = f[i];
        order[i].id = (uint64_t)i;
        parent[i] = (uint64_t)i;
        size[i] = 1;
        deepest[i] = (uint64_t)i;
    }
    qsort(order, (size_t)N, sizeof(keyed), cmp_keyed);

    const int64_t sx = 1, sy = nx, sz = nx * ny;
    for (int64_t i = 0; i < N; ++i) {
        const int64_t u = order[i].id;
        const int64_t x = u % nx, y = (u / nx) % ny, z = u / (nx * ny);
        int64_t nb[6];
        int nn = 0;
        if (x > 0) nb[nn++] = u - sx;
        if (x + 1 < nx) nb[nn++] = u + sx;
        if (y > 0) nb[nn++] = u - sy;
        if (y + 1 < ny) nb[nn++] = u + sy;
        if (z > 0) nb[nn++] = u - sz;
        if (z + 1 < nz) nb[nn++] = u + sz;

        /* Components of the sublevel set below u that touch u: a neighbour
           has already been swept exactly when it precedes u. */
        uint64_t roots[6];
        int nr = 0;
        for (int k = 0; k < nn; ++k) {
            if (!precedes(f, nb[k], u)) continue;
            uint64_t r = uf_find(parent, (uint64_t)nb[k]);
            int seen = 0;
            for (int j = 0; j < nr; ++j) seen |= (roots[j] == r);
            if (!seen) roots[nr++] = r;
        }

        if (nr == 0) {
            /* Case (1): u is a local minimum and starts a component.  Until
               that component merges into an older one, u is its deepest
               vertex and its triplet is (u, u, u). */
            T[2 * u] = (uint64_t)u;
            T[2 * u + 1] = (uint64_t)u;
            continue;
        }

        /* Cases (2) and (3).  The deepest vertex of the merged component is
           the deepest of the deepest vertices of the parts. */
        int best = 0;
        for (int j = 1; j < nr; ++j)
            if (precedes(f, deepest[roots[j]], deepest[roots[best]])) best = j;
        const uint64_t m1 = deepest[roots[best]];

        /* u itself: degree-two vertex (u, u, m1). */
        T[2 * u] = (uint64_t)u;
        T[2 * u + 1] = m1;

        /* Every other part's branch, born at its deepest vertex m, ends at u
           and joins the branch of m1: triplet (m, u, m1). */
        for (int j = 0; j < nr; ++j) {
            if (j == best) continue;
            const uint64_t m = deepest[roots[j]];
            T[2 * m] = (uint64_t)u;
            T[2 * m + 1] = m1;
        }

        /* Union everything with u. */
        uint64_t r = (uint64_t)u;
        for (int j = 0; j < nr; ++j) {
            uint64_t a = uf_find(parent, r), b = roots[j];
            if (a == b) continue;
            if (size[a] < size[b]) { uint64_t t = a; a = b; b = t; }
            parent[b] = a;
            size[a] += size[b];
            r = a;
        }
        deepest[uf_find(parent, (uint64_t)u)] = m1;
    }

    free(order); free(parent); free(size); free(deepest);
    return OR_OK;
}

/*
 * Persistence pairs read off the triplets (Sec. 1: one point per branch).
 * The branch born at u dies at s exactly when T[u] = (s, v) with s != u.
 * Pairs are emitted in ascending birth id.  Returns the number of pairs (or a
 * negative status); when it exceeds capacity nothing beyond capacity is
 * written and the full count is still returned.  *n_roots (if not NULL)
 * receives the number of triplets (u, u, u).
 */
int64_t oracle_pairs(const double *f, const uint64_t *T, int64_t N,
                     uint64_t *birth, uint64_t *death, double *birth_val, double *death_val,
                     int64_t capacity, int64_t *n_roots)
{
    if (!f || !T || N < 0) return OR_ERR_INVALID_ARG;
    int64_t p = 0, roots = 0;
    for (int64_t u = 0; u < N; ++u) {
        const uint64_t s = T[2 * u], v = T[2 * u + 1];
        if (s == (uint64_t)u) {
            if (v == (uint64_t)u) ++roots;
            continue;
        }
        if (p < capacity) {
            birth[p] = (uint64_t)u;
            death[p] = s;
            birth_val[p] = f[u];
            death_val[p] = f[s];
        }
        ++p;
    }
    if (n_roots) *n_roots = roots;
    return p;
}

/*
 * Chain rule for a loss written on the pair values: the birth value is f at
 * the birth vertex and the death value is f at the death vertex, so
 * grad[birth[k]] += gb[k] and grad[death[k]] += gd[k].  grad is accumulated
 * into, in double.
 */
int oracle_pairs_scatter(int64_t N, const uint64_t *birth, const uint64_t *death,
                         const double *gb, const double *gd, int64_t P, double *grad)
{
    if (!grad || (P > 0 && (!birth || !death || !gb || !gd))) return OR_ERR_INVALID_ARG;
    for (int64_t k = 0; k < P; ++k) {
        if (birth[k] >= (uint64_t)N || death[k] >= (uint64_t)N) return OR_ERR_INVALID_ARG;
        grad[birth[k]] += gb[k];
        grad[death[k]] += gd[k];
    }
    return OR_OK;
}

/*
 * Topological-simplification loss on the persistence pairs of f:
 * L = sum over pairs with (death - birth) < tau of (death - birth)^2, and,
 * if grad is not NULL, dL/df written into grad (overwritten, length N).
 * Returns the loss through *loss.  All in double.
 */
int oracle_topo_loss(const double *f, int64_t nx, int64_t ny, int64_t nz, double tau,
                     double *loss, double *grad)
{
    int st = validate(nx, ny, nz);
    if (st != OR_OK) return st;
    const int64_t N = nx * ny * nz;
    uint64_t *T = (uint64_t *)malloc((size_t)N * 2 * sizeof(uint64_t));
    if (!T) return OR_ERR_NOMEM;
    st = oracle_merge_tree(f, nx, ny, nz, T);
    if (st != OR_OK) { free(T); return st; }

    double L = 0.0;
    if (grad) memset(grad, 0, (size_t)N * sizeof(double));
    for (int64_t u = 0; u < N; ++u) {
        const uint64_t s = T[2 * u];
        if (s == (uint64_t)u) continue;
        const double b = f[u], d = f[s];
        const double pers = d - b;
        if (!(pers < tau)) continue;
        L += pers * pers;
        if (grad) {
            grad[u] += -2.0 * pers;
            grad[s] += 2.0 * pers;
        }
    }
    free(T);
    *loss = L;
    return OR_OK;
}

/*
 * Sampled triplets by their definition (item 5 above).  For each u in us[0..n)
 * it computes T[u] = (s, v) without the sweep:
 *  - u has a lower neighbour: s = u, and v is the deepest vertex of u's
 *    component of the sublevel set at the level of u;
 *  - u is a local minimum: its branch ends at the first level at which its
 *    component holds a vertex deeper than u; s is the vertex at that level
 *    and v the deepest vertex of the component there; if no such level
 *    exists u is the deepest vertex of its connected component, (u, u).
 * A flood from u that always adds the lowest vertex next to the vertices it
 * has added (a priority queue in the order of the values, ties by id) adds
 * u's component at every level L completely before any vertex above L, so:
 * lam, the highest vertex added so far, is the level reached; the first
 * added vertex that precedes u (for a minimum u) fixes s = lam; after that
 * (or from the start, for a vertex that is no minimum, with s = u) the flood
 * goes on while the lowest boundary vertex is at or below s, and v is the
 * deepest vertex added.
 *
 * f is float (is_f32 = 1) or double values; the comparison is the same IEEE
 * one either way.  status[i] = OR_OK, or OR_ERR_CAPACITY when the flood from
 * us[i] would add more than max_visit vertices (s, v then undefined), or
 * OR_ERR_NAN when it meets a NaN.
 */
static double valat(const void *f, int is_f32, int64_t i)
{
    return is_f32 ? (double)((const float *)f)[i] : ((const double *)f)[i];
}

static int prec2(const void *f, int is_f32, int64_t a, int64_t b)
{
    const double fa = valat(f, is_f32, a), fb = valat(f, is_f32, b);
    return fa < fb || (fa == fb && a < b);
}

int oracle_triplets_at(const void *f, int is_f32, int64_t nx, int64_t ny, int64_t nz, const int64_t *us,
                       int64_t n, int64_t max_visit, uint64_t *s_out, uint64_t *v_out, int32_t *status)
{
    int st = validate(nx, ny, nz);
    if (st != OR_OK) return st;
    if (!f || !us || !s_out || !v_out || !status || n < 0 || max_visit < 1) return OR_ERR_INVALID_ARG;
    const int64_t N = nx * ny * nz, sy = nx, sz = nx * ny;
    /* every added vertex puts at most 6 on the boundary */
    const int64_t heap_cap = 6 * max_visit + 8;
    int64_t hsz = 64;
    while (hsz < 8 * max_visit + 64) hsz <<= 1;
    int64_t *heap = (int64_t *)malloc((size_t)heap_cap * sizeof(int64_t));
    int64_t *seen = (int64_t *)malloc((size_t)hsz * sizeof(int64_t));       /* open addressing, -1 empty */
    int64_t *touched = (int64_t *)malloc((size_t)(heap_cap + 8) * sizeof(int64_t));
    if (!heap || !seen || !touched) {
        free(heap); free(seen); free(touched);
        return OR_ERR_NOMEM;
    }
    for (int64_t i = 0; i < hsz; ++i) seen[i] = -1;

    for (int64_t q = 0; q < n; ++q) {
        const int64_t u = us[q];
        if (u < 0 || u >= N) { free(heap); free(seen); free(touched); return OR_ERR_INVALID_ARG; }
        int64_t hn = 0, nt = 0, added = 0;
        int rc = OR_OK;
        /* mark x as discovered; returns 0 if it already was, -1 if the set is full */
        #define DISCOVER(x, res)                                                     \
            do {                                                                     \
                uint64_t hh = ((uint64_t)(x) * 0x9E3779B97F4A7C15ull) >> 20;         \
                int64_t slot = (int64_t)(hh & (uint64_t)(hsz - 1));                  \
                res = 1;                                                             \
                while (seen[slot] != -1) {                                           \
                    if (seen[slot] == (x)) { res = 0; break; }                       \
                    slot = (slot + 1) & (hsz - 1);                                   \
                }                                                                    \
                if (res) {                                                           \
                    if (nt >= heap_cap + 8) { res = -1; break; }                     \
                    seen[slot] = (x);                                                \
                    touched[nt++] = slot;                                            \
                }                                                                    \
            } while (0)
        #define HEAP_PUSH(x)                                                         \
            do {                                                                     \
                int64_t i_ = hn++;                                                   \
                heap[i_] = (x);                                                      \
                while (i_ > 0) {                                                     \
                    const int64_t p_ = (i_ - 1) / 2;                                 \
                    if (!prec2(f, is_f32, heap[i_], heap[p_])) break;                \
                    const int64_t t_ = heap[i_]; heap[i_] = heap[p_]; heap[p_] = t_; \
                    i_ = p_;                                                         \
                }                                                                    \
            } while (0)
        int res = 0;
        DISCOVER(u, res);
        HEAP_PUSH(u);
        int is_min = 1;
        {
            const int64_t x = u % nx, y = (u / nx) % ny, z = u / sz;
            if (x > 0 && prec2(f, is_f32, u - 1, u)) is_min = 0;
            if (x + 1 < nx && prec2(f, is_f32, u + 1, u)) is_min = 0;
            if (y > 0 && prec2(f, is_f32, u - sy, u)) is_min = 0;
            if (y + 1 < ny && prec2(f, is_f32, u + sy, u)) is_min = 0;
            if (z > 0 && prec2(f, is_f32, u - sz, u)) is_min = 0;
            if (z + 1 < nz && prec2(f, is_f32, u + sz, u)) is_min = 0;
        }
        int64_t s = is_min ? -1 : u; /* -1: the saddle is not reached yet */
        int64_t lam = u, deepest = u;
        while (hn > 0) {
            const int64_t top = heap[0];
            if (s >= 0 && prec2(f, is_f32, s, top)) break; /* the boundary is above level s */
            /* pop */
            heap[0] = heap[--hn];
            {
                int64_t i_ = 0;
                for (;;) {
                    const int64_t l_ = 2 * i_ + 1, r_ = l_ + 1;
                    int64_t m_ = i_;
                    if (l_ < hn && prec2(f, is_f32, heap[l_], heap[m_])) m_ = l_;
                    if (r_ < hn && prec2(f, is_f32, heap[r_], heap[m_])) m_ = r_;
                    if (m_ == i_) break;
                    const int64_t t_ = heap[i_]; heap[i_] = heap[m_]; heap[m_] = t_;
                    i_ = m_;
                }
            }
            if (isnan(valat(f, is_f32, top))) { rc = OR_ERR_NAN; break; }
            if (++added > max_visit) { rc = OR_ERR_CAPACITY; break; }
            if (prec2(f, is_f32, lam, top)) lam = top;
            if (prec2(f, is_f32, top, deepest)) deepest = top;
            if (s < 0 && prec2(f, is_f32, top, u)) s = lam; /* first vertex deeper than u: u's branch ends at lam */
            const int64_t x = top % nx, y = (top / nx) % ny, z = top / sz;
            int64_t nb[6];
            int nn = 0;
            if (x > 0) nb[nn++] = top - 1;
            if (x + 1 < nx) nb[nn++] = top + 1;
            if (y > 0) nb[nn++] = top - sy;
            if (y + 1 < ny) nb[nn++] = top + sy;
            if (z > 0) nb[nn++] = top - sz;
            if (z + 1 < nz) nb[nn++] = top + sz;
            for (int k = 0; k < nn && rc == OR_OK; ++k) {
                DISCOVER(nb[k], res);
                if (res < 0) rc = OR_ERR_CAPACITY;
                else if (res > 0) {
                    if (hn >= heap_cap) rc = OR_ERR_CAPACITY;
                    else HEAP_PUSH(nb[k]);
                }
            }
            if (rc != OR_OK) break;
        }
        #undef DISCOVER
        #undef HEAP_PUSH
        for (int64_t i = 0; i < nt; ++i) seen[touched[i]] = -1;
        status[q] = rc;
        if (rc != OR_OK) continue;
        if (s < 0) { /* the flood emptied u's connected component: u is its deepest vertex */
            s_out[q] = (uint64_t)u;
            v_out[q] = (uint64_t)u;
        } else {
            s_out[q] = (uint64_t)s;
            v_out[q] = (uint64_t)deepest;
        }
    }
    free(heap); free(seen); free(touched);
    return OR_OK;
}
