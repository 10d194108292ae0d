// mt.hip -- triplet merge trees on gfx950 (MI355X): kernels and the C ABI.
//
// The method is the triplet merge tree of "Fast Merge Tree Computation via
// SYCL" (arXiv 2301.10838), Sec. 2 (Alg. 1-5) with the GPU data layout of
// Sec. 3.2: T is an array of (saddle, target) pairs of 32-bit ids packed into
// one 64-bit word per vertex, so a single 64-bit compare-and-swap updates a
// triplet atomically.
//
// Pipeline of one build (all fields of a batch at once):
//   k_setup        field table + status word into the workspace
//   k_descend      LDS tile + halo: lowest lower neighbour of every vertex,
//                  chains followed inside the tile, NaN check, roots (u,u,u)
//   k_resolve      chains followed across tiles: minimum each vertex reaches
//   k_merge        lock-free Merge (Alg. 3) for every grid edge whose ends
//                  reach different minima, between those two minima
//   k_repair_min   Repair (Alg. 5) of the minima: target -> representative
//   k_repair_reg   every other vertex u: (u, u, representative at level u)
//   k_pairs_*      count / scan / ordered compaction of the pairs
//
// Why the first two steps are legitimate: pointing every vertex at its lowest
// lower neighbour is what Merge produces when those edges are merged one by
// one in decreasing order of their upper vertex, and Alg. 1 merges edges in
// any order.  Compressing each chain to the minimum it reaches (the chain
// links all lie below the vertex) leaves a normalized representation of the
// same sublevel connectivity.  An edge whose two ends reach the same minimum
// connects vertices that are already connected below its upper end, so it
// changes no sublevel component and is skipped; any other edge (a, b) states
// that the minima z(a), z(b) are connected at level max(a, b), and that is
// the fact merged.  The tree is unique (normalization + minimality), so the
// result equals the serial one bit for bit.
//
// Order: vertices compare by (value, id) with IEEE semantics; the value is
// mapped to an order-preserving uint32 (with -0.0 folded onto +0.0) and the
// id is appended, so every comparison is one 64-bit integer compare.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "mt.h"

namespace {

constexpr uint32_t kMask = 0x7fffffffu;      // vertex id bits of a label
constexpr uint32_t kResolved = 0x80000000u;  // label names the final minimum
constexpr int kBlock = 256;                  // threads per workgroup (4 waves)
constexpr int kMaxTileVol = 1024;            // vertices per stencil tile
constexpr int kMaxHalo = 4096;               // tile + halo cells in LDS
constexpr int kChunk = 4096;                 // vertices per block in flat passes
constexpr int kSetupMax = 12;                // field descriptors per k_setup
constexpr int kBwdGroup = 64;                // fields per backward launch

constexpr uint32_t ST_NAN = 1u, ST_LIVELOCK = 2u, ST_CAPACITY = 4u, ST_CORRUPT = 8u;

struct FieldDesc {
    int32_t nx, ny, nz;
    int32_t tx, ty, tz;     // tile shape of the stencil passes
    int32_t ntx, nty, ntz;  // tiles along each axis
    int32_t pad;
    int64_t offset;         // global id of the field's first vertex
    int64_t n;              // vertices
    int64_t tile_start;     // first tile of the field
    int64_t chunk_start;    // first chunk of the field
};

struct Header {
    uint32_t status;
    uint32_t pad;
    int64_t total_pairs;
    int64_t roots;
    int64_t reserved[5];
};

// ---------------------------------------------------------------------------
// device helpers

__device__ __forceinline__ uint32_t okey(float x)
{
    uint32_t b = __float_as_uint(x);
    b = (b == 0x80000000u) ? 0u : b;                 // -0.0 == +0.0
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ uint64_t vkey(const float *__restrict__ f, uint32_t id)
{
    return ((uint64_t)okey(f[id]) << 32) | id;
}

__device__ __forceinline__ uint32_t lo32(uint64_t t) { return (uint32_t)t; }
__device__ __forceinline__ uint32_t hi32(uint64_t t) { return (uint32_t)(t >> 32); }
__device__ __forceinline__ uint64_t pack(uint32_t s, uint32_t v) { return (uint64_t)s | ((uint64_t)v << 32); }

// Coherent read of a triplet while other waves may CAS it (merge phase).
__device__ __forceinline__ uint64_t ld_coherent(uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Untorn 64-bit read/write where stale values are harmless (repair phase).
__device__ __forceinline__ uint64_t ld_relaxed(uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void st_relaxed(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ int find_field(const int64_t *__restrict__ starts, int nf, int64_t t)
{
    int lo = 0, hi = nf;  // starts[lo] <= t < starts[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (starts[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// run of tiles so neighbouring tiles (which share halo lines) share an L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G, int remap)
{
    if (!remap || G < 8) return b;
    const int64_t per = G / 8, rem = G % 8;
    const int64_t x = b % 8, j = b / 8;
    return x * per + (x < rem ? x : rem) + j;
}

struct Tile {
    int64_t off;
    int nx, ny, nz, tx, ty, tz;
    int x0, y0, z0, ex, ey, ez;
    int64_t sxy;
};

__device__ __forceinline__ Tile decode_tile(const FieldDesc *__restrict__ D, const int64_t *__restrict__ ts,
                                            int nf, int64_t t)
{
    const int fi = find_field(ts, nf, t);
    const FieldDesc d = D[fi];
    Tile c;
    const int64_t lt = t - d.tile_start;
    const int bx = (int)(lt % d.ntx);
    const int64_t r = lt / d.ntx;
    const int by = (int)(r % d.nty);
    const int bz = (int)(r / d.nty);
    c.off = d.offset;
    c.nx = d.nx; c.ny = d.ny; c.nz = d.nz;
    c.tx = d.tx; c.ty = d.ty; c.tz = d.tz;
    c.x0 = bx * d.tx; c.y0 = by * d.ty; c.z0 = bz * d.tz;
    c.ex = min(d.tx, d.nx - c.x0);
    c.ey = min(d.ty, d.ny - c.y0);
    c.ez = min(d.tz, d.nz - c.z0);
    c.sxy = (int64_t)d.nx * d.ny;
    return c;
}

// Representative (Alg. 4, with the chase returning the last vertex reached):
// follow T from x while the saddle is at or below `level` and x is no root.
// Every id read back from memory is checked against n before it is used as
// an address; a failed check (a broken invariant) latches ST_CORRUPT.
__device__ __forceinline__ uint32_t chase(uint64_t *__restrict__ T, const float *__restrict__ f, uint32_t n,
                                          uint32_t x, uint64_t level, uint32_t cap, uint32_t &err)
{
    for (uint32_t step = 0; step < cap; ++step) {
        const uint64_t t = ld_relaxed(T + x);
        const uint32_t v = hi32(t), s = lo32(t);
        if (v >= n || s >= n) { err |= ST_CORRUPT; return x; }
        if (v == x) return x;                       // root
        if (vkey(f, s) > level) return x;           // joins above the level
        x = v;
    }
    err |= ST_LIVELOCK;
    return x;
}

// Merge (Alg. 3) of the fact "u and v are connected at level s", as a loop.
// Descents stop at roots; after a CAS that replaced a root nothing was
// displaced; otherwise the displaced triplet (v, s_v, v') is merged again as
// (u, s_v, v').  A lost CAS restarts with the value the CAS saw.
__device__ void tmt_merge(uint64_t *__restrict__ T, const float *__restrict__ f, uint32_t n, uint32_t u,
                          uint32_t s, uint64_t ks, uint32_t v, uint32_t cap, uint32_t &err)
{
    uint64_t tu = ld_coherent(T + u);
    uint64_t tv = ld_coherent(T + v);
    for (uint32_t step = 0; step < cap; ++step) {
        const uint32_t u1 = hi32(tu), su = lo32(tu), v1 = hi32(tv), sv = lo32(tv);
        if (max(max(u1, su), max(v1, sv)) >= n) { err |= ST_CORRUPT; return; }
        if (u1 != u && vkey(f, su) < ks) { u = u1; tu = ld_coherent(T + u); continue; }
        if (v1 != v && vkey(f, sv) < ks) { v = v1; tv = ld_coherent(T + v); continue; }
        if (u == v) return;
        if (vkey(f, v) < vkey(f, u)) {               // the upper one is re-pointed
            const uint32_t w = u; u = v; v = w;
            const uint64_t tw = tu; tu = tv; tv = tw;
        }
        uint64_t seen = tv;
        if (__hip_atomic_compare_exchange_strong(T + v, &seen, pack(s, u), __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
            if (hi32(tv) == v) return;               // v was a root
            s = lo32(tv);
            ks = vkey(f, s);
            v = hi32(tv);
            tv = ld_coherent(T + v);
        } else {
            tv = seen;
        }
        tu = ld_coherent(T + u);
    }
    err |= ST_LIVELOCK;
}

// ---------------------------------------------------------------------------
// kernels

struct SetupArgs {
    FieldDesc d[kSetupMax];
    int32_t first, count, nf;
    uint32_t clear_status;  // status bits to clear
    int32_t zero_counts;
    int32_t pad;
    int64_t total_tiles, total_chunks;
};

__global__ void k_setup(SetupArgs a, FieldDesc *D, int64_t *ts, int64_t *cs, Header *h)
{
    const int i = threadIdx.x;
    if (i < a.count) {
        D[a.first + i] = a.d[i];
        ts[a.first + i] = a.d[i].tile_start;
        cs[a.first + i] = a.d[i].chunk_start;
    }
    if (i == 0) {
        if (a.first + a.count == a.nf) {
            ts[a.nf] = a.total_tiles;
            cs[a.nf] = a.total_chunks;
        }
        if (a.clear_status) h->status &= ~a.clear_status;
        if (a.zero_counts) { h->total_pairs = 0; h->roots = 0; }
    }
}

// Lowest lower neighbour of every vertex of a tile, chains followed inside the
// tile.  lbl[u] = the minimum reached (with kResolved) or the first vertex
// outside the tile on the descent.  Minima get the root triplet (u, u, u).
__global__ __launch_bounds__(kBlock) void k_descend(const float *__restrict__ f, uint32_t *__restrict__ lbl,
                                                    uint64_t *__restrict__ T, const FieldDesc *__restrict__ D,
                                                    const int64_t *__restrict__ ts, int nf, int64_t n_tiles,
                                                    int remap, uint32_t *__restrict__ status)
{
    __shared__ uint32_t hk[kMaxHalo];        // order keys of tile + halo
    __shared__ uint32_t wg[kMaxTileVol];     // descent target, global id
    __shared__ int16_t wl[kMaxTileVol];      // descent target in tile, -1 outside, self at minima

    const int64_t t = xcd_tile(blockIdx.x, gridDim.x, remap);
    if (t >= n_tiles) return;
    const Tile c = decode_tile(D, ts, nf, t);
    const int ox = c.nx > 1, oy = c.ny > 1, oz = c.nz > 1;
    const int hx = c.tx + 2 * ox, hy = c.ty + 2 * oy, hz = c.tz + 2 * oz;
    const int hvol = hx * hy * hz;
    const float *__restrict__ fb = f + c.off;

    bool nan = false;
    for (int i = threadIdx.x; i < hvol; i += kBlock) {
        const int ix = i % hx, iy = (i / hx) % hy, iz = i / (hx * hy);
        const int gx = c.x0 - ox + ix, gy = c.y0 - oy + iy, gz = c.z0 - oz + iz;
        uint32_t k = 0xffffffffu;
        if (gx >= 0 && gx < c.nx && gy >= 0 && gy < c.ny && gz >= 0 && gz < c.nz) {
            const float v = fb[gx + (int64_t)c.nx * gy + c.sxy * gz];
            nan |= (v != v);
            k = okey(v);
        }
        hk[i] = k;
    }
    if (__ballot(nan) != 0ull && (threadIdx.x & 63) == 0) atomicOr(status, ST_NAN);
    __syncthreads();

    const int vol = c.tx * c.ty * c.tz;
    const int dhy = hx, dhz = hx * hy;
    for (int i = threadIdx.x; i < vol; i += kBlock) {
        const int lx = i % c.tx, ly = (i / c.tx) % c.ty, lz = i / (c.tx * c.ty);
        if (lx >= c.ex || ly >= c.ey || lz >= c.ez) continue;
        const int gx = c.x0 + lx, gy = c.y0 + ly, gz = c.z0 + lz;
        const int64_t lid = gx + (int64_t)c.nx * gy + c.sxy * gz;
        const uint32_t uid = (uint32_t)(c.off + lid);
        const int h = (lx + ox) + hx * ((ly + oy) + hy * (lz + oz));
        uint64_t best = ((uint64_t)hk[h] << 32) | uid;
        int bd = 0;  // 0 none, else direction code
        uint32_t bid = uid;
#define MT_CAND(cond, dh, did, code)                                                        \
        if (cond) {                                                                         \
            const uint32_t nid = (uint32_t)((int64_t)uid + (did));                         \
            const uint64_t k = ((uint64_t)hk[h + (dh)] << 32) | nid;                       \
            if (k < best) { best = k; bd = (code); bid = nid; }                            \
        }
        MT_CAND(gx > 0, -1, -1, 1)
        MT_CAND(gx + 1 < c.nx, 1, 1, 2)
        MT_CAND(gy > 0, -dhy, -(int64_t)c.nx, 3)
        MT_CAND(gy + 1 < c.ny, dhy, (int64_t)c.nx, 4)
        MT_CAND(gz > 0, -dhz, -c.sxy, 5)
        MT_CAND(gz + 1 < c.nz, dhz, c.sxy, 6)
#undef MT_CAND
        wg[i] = bid;
        if (bd == 0) {
            wl[i] = (int16_t)i;
        } else {
            int qx = lx, qy = ly, qz = lz;
            if (bd == 1) --qx; else if (bd == 2) ++qx; else if (bd == 3) --qy;
            else if (bd == 4) ++qy; else if (bd == 5) --qz; else ++qz;
            const bool inside = qx >= 0 && qx < c.ex && qy >= 0 && qy < c.ey && qz >= 0 && qz < c.ez;
            wl[i] = inside ? (int16_t)(qx + c.tx * (qy + c.ty * qz)) : (int16_t)-1;
        }
    }
    __syncthreads();

    for (int i = threadIdx.x; i < vol; i += kBlock) {
        const int lx = i % c.tx, ly = (i / c.tx) % c.ty, lz = i / (c.tx * c.ty);
        if (lx >= c.ex || ly >= c.ey || lz >= c.ez) continue;
        const int64_t lid = (c.x0 + lx) + (int64_t)c.nx * (c.y0 + ly) + c.sxy * (c.z0 + lz);
        const uint32_t uid = (uint32_t)(c.off + lid);
        // keys fall strictly along wl, so the walk ends within vol steps
        int x = i;
        uint32_t e = wg[i];
        for (int step = 0; step <= vol; ++step) {
            const int y = wl[x];
            if (y == x) { e = wg[x] | kResolved; break; }
            if (y < 0) { e = wg[x]; break; }
            x = y;
        }
        lbl[uid] = e;
        if (wl[i] == i) T[uid] = pack(uid, uid);
    }
}

// Follow exit pointers across tiles to the minimum (in place; a concurrent
// write only ever replaces a label by one further down the same descent).
__global__ __launch_bounds__(kBlock) void k_resolve(uint32_t *__restrict__ lbl, int64_t n, uint32_t cap,
                                                    uint32_t *__restrict__ status)
{
    const int64_t u = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (u >= n) return;
    const uint32_t e = lbl[u];
    if (e & kResolved) return;
    uint32_t x = e;
    uint32_t err = ST_LIVELOCK;
    for (uint32_t step = 0; step < cap; ++step) {
        if ((int64_t)x >= n) { err = ST_CORRUPT; break; }
        const uint32_t y = __hip_atomic_load(lbl + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        if (y & kResolved) { x = y & kMask; err = 0; break; }
        x = y;
    }
    if (err) { atomicOr(status, err); x = (uint32_t)u; }
    __hip_atomic_store(lbl + u, x | kResolved, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Merge phase (Alg. 1, second loop): every vertex owns its +x, +y, +z edges.
__global__ __launch_bounds__(kBlock) void k_merge(const float *__restrict__ f, const uint32_t *__restrict__ lbl,
                                                  uint64_t *__restrict__ T, const FieldDesc *__restrict__ D,
                                                  const int64_t *__restrict__ ts, int nf, int64_t n_tiles,
                                                  uint32_t n, int remap, uint32_t cap, uint32_t *__restrict__ status)
{
    const int64_t t = xcd_tile(blockIdx.x, gridDim.x, remap);
    if (t >= n_tiles) return;
    const Tile c = decode_tile(D, ts, nf, t);
    const int vol = c.tx * c.ty * c.tz;
    uint32_t err = 0;
    for (int i = threadIdx.x; i < vol; i += kBlock) {
        const int lx = i % c.tx, ly = (i / c.tx) % c.ty, lz = i / (c.tx * c.ty);
        if (lx >= c.ex || ly >= c.ey || lz >= c.ez) continue;
        const int gx = c.x0 + lx, gy = c.y0 + ly, gz = c.z0 + lz;
        const uint32_t uid = (uint32_t)(c.off + gx + (int64_t)c.nx * gy + c.sxy * gz);
        const uint32_t zu = lbl[uid] & kMask;
        if (zu >= n) { err |= ST_CORRUPT; continue; }
        const uint64_t ku = vkey(f, uid);
#define MT_EDGE(cond, did)                                                                  \
        if (cond) {                                                                         \
            const uint32_t nb = (uint32_t)((int64_t)uid + (did));                          \
            const uint32_t zn = lbl[nb] & kMask;                                           \
            if (zn >= n) {                                                                 \
                err |= ST_CORRUPT;                                                         \
            } else if (zn != zu) {                                                         \
                const uint64_t kn = vkey(f, nb);                                           \
                const bool up = kn < ku;                                                   \
                tmt_merge(T, f, n, zu, up ? uid : nb, up ? ku : kn, zn, cap, err);          \
            }                                                                               \
        }
        MT_EDGE(gx + 1 < c.nx, 1)
        MT_EDGE(gy + 1 < c.ny, (int64_t)c.nx)
        MT_EDGE(gz + 1 < c.nz, c.sxy)
#undef MT_EDGE
    }
    if (err) atomicOr(status, err);
}

// Repair (Alg. 5) of every minimum that is not a root.
__global__ __launch_bounds__(kBlock) void k_repair_min(const float *__restrict__ f, const uint32_t *__restrict__ lbl,
                                                       uint64_t *__restrict__ T, int64_t n, uint32_t cap,
                                                       uint32_t *__restrict__ status)
{
    const int64_t u64 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (u64 >= n) return;
    const uint32_t u = (uint32_t)u64;
    if ((lbl[u] & kMask) != u) return;
    const uint64_t t = ld_relaxed(T + u);
    const uint32_t v = hi32(t);
    if (v == u) return;
    const uint32_t s = lo32(t);
    uint32_t err = 0;
    if ((int64_t)v >= n || (int64_t)s >= n) {
        err = ST_CORRUPT;
    } else {
        const uint32_t r = chase(T, f, (uint32_t)n, v, vkey(f, s), cap, err);
        if (r != v) st_relaxed(T + u, pack(s, r));
    }
    if (err) atomicOr(status, err);
}

// Every non-minimum u: triplet (u, u, representative of its minimum at the
// level of u).  Written with field-local ids (these entries are never read
// by other threads).
__global__ __launch_bounds__(kBlock) void k_repair_reg(const float *__restrict__ f, const uint32_t *__restrict__ lbl,
                                                       uint64_t *__restrict__ T, const FieldDesc *__restrict__ D,
                                                       const int64_t *__restrict__ cs, int nf, uint32_t n,
                                                       uint32_t cap, uint32_t *__restrict__ status)
{
    const int64_t c = blockIdx.x;
    const FieldDesc d = D[find_field(cs, nf, c)];
    const int64_t lo = (c - d.chunk_start) * kChunk;
    const int64_t hi = min(lo + (int64_t)kChunk, d.n);
    const uint32_t off = (uint32_t)d.offset;
    uint32_t err = 0;
    for (int64_t j = lo + threadIdx.x; j < hi; j += kBlock) {
        const uint32_t u = off + (uint32_t)j;
        const uint32_t z = lbl[u] & kMask;
        if (z == u) continue;
        if (z >= n) { err |= ST_CORRUPT; continue; }
        const uint32_t r = chase(T, f, n, z, vkey(f, u), cap, err);
        T[u] = pack(u - off, r - off);
    }
    if (err) atomicOr(status, err);
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Pair flags.  kFromLbl: minima come from the labels and T still holds global
// ids for them (batch build); otherwise T alone, local ids (public readout).
// Ids read from T are checked to lie in the field; a bad one is no pair and
// latches ST_CORRUPT.
template <bool kFromLbl>
__device__ __forceinline__ bool classify(const uint64_t *__restrict__ T, const uint32_t *__restrict__ lbl,
                                         uint32_t off, uint32_t n, int64_t j, uint32_t &s_loc, bool &root,
                                         uint32_t &err)
{
    const uint32_t u = off + (uint32_t)j;
    root = false;
    const uint64_t t = kFromLbl ? 0ull : T[u];
    if (kFromLbl) {
        if ((lbl[u] & kMask) != u) return false;
        const uint64_t tm = T[u];
        const uint32_t sl = lo32(tm) - off, vl = hi32(tm) - off;  // wraps high when below off
        if (sl >= n || vl >= n) { err |= ST_CORRUPT; return false; }
        if (vl == (uint32_t)j) { root = true; return false; }
        s_loc = sl;
        return true;
    }
    const uint32_t s = lo32(t), v = hi32(t);
    if (s >= n || v >= n) { err |= ST_CORRUPT; return false; }
    if (s == (uint32_t)j) { root = (v == (uint32_t)j); return false; }
    s_loc = s;
    return true;
}

template <bool kFromLbl>
__global__ __launch_bounds__(kBlock) void k_pairs_count(const uint64_t *__restrict__ T, const uint32_t *__restrict__ lbl,
                                                        const FieldDesc *__restrict__ D, const int64_t *__restrict__ cs,
                                                        int nf, uint32_t *__restrict__ cnt, Header *__restrict__ h)
{
    uint32_t err = 0;
    __shared__ uint32_t sp[kBlock / 64], sr[kBlock / 64];
    const int64_t c = blockIdx.x;
    const FieldDesc d = D[find_field(cs, nf, c)];
    const int64_t lo = (c - d.chunk_start) * kChunk;
    const int64_t hi = min(lo + (int64_t)kChunk, d.n);
    uint32_t np = 0, nr = 0;
    for (int64_t j = lo + threadIdx.x; j < hi; j += kBlock) {
        uint32_t s;
        bool root;
        np += classify<kFromLbl>(T, lbl, (uint32_t)d.offset, (uint32_t)d.n, j, s, root, err) ? 1u : 0u;
        nr += root ? 1u : 0u;
    }
    if (err) atomicOr(&h->status, err);
    for (int o = 32; o > 0; o >>= 1) {
        np += __shfl_xor(np, o);
        nr += __shfl_xor(nr, o);
    }
    if ((threadIdx.x & 63) == 0) { sp[threadIdx.x >> 6] = np; sr[threadIdx.x >> 6] = nr; }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
        for (int w = 0; w < kBlock / 64; ++w) { a += sp[w]; b += sr[w]; }
        cnt[c] = a;
        if (b) atomicAdd((unsigned long long *)&h->roots, (unsigned long long)b);
    }
}

// Exclusive scan of the chunk counts (one workgroup of 1024), totals, and the
// per-field pair offsets.
__global__ __launch_bounds__(1024) void k_pairs_scan(uint32_t *__restrict__ cnt, int64_t n_chunks,
                                                     const FieldDesc *__restrict__ D, int nf,
                                                     int64_t *__restrict__ pair_offsets, int64_t capacity,
                                                     Header *__restrict__ h)
{
    __shared__ uint64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (n_chunks + 1023) / 1024;
    const int64_t a = min((int64_t)tid * per, n_chunks), b = min(a + per, n_chunks);
    uint64_t s = 0;
    for (int64_t i = a; i < b; ++i) s += cnt[i];
    part[tid] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const uint64_t v = tid >= o ? part[tid - o] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint64_t run = part[tid] - s;  // exclusive prefix of this segment
    for (int64_t i = a; i < b; ++i) {
        const uint32_t v = cnt[i];
        cnt[i] = (uint32_t)run;
        run += v;
    }
    const uint64_t total = part[1023];
    __syncthreads();
    if (pair_offsets) {
        for (int i = tid; i < nf; i += 1024) pair_offsets[i] = cnt[D[i].chunk_start];
        if (tid == 0) pair_offsets[nf] = (int64_t)total;
    }
    if (tid == 0) {
        h->total_pairs = (int64_t)total;
        if ((int64_t)total > capacity) atomicOr(&h->status, ST_CAPACITY);
    }
}

// Ordered compaction: ascending vertex id within the chunk, chunks in order.
template <bool kFromLbl>
__global__ __launch_bounds__(kBlock) void k_pairs_write(const float *__restrict__ f, uint64_t *__restrict__ T,
                                                        const uint32_t *__restrict__ lbl,
                                                        const FieldDesc *__restrict__ D, const int64_t *__restrict__ cs,
                                                        int nf, const uint32_t *__restrict__ base, int64_t capacity,
                                                        uint32_t *__restrict__ birth, uint32_t *__restrict__ death,
                                                        float *__restrict__ bval, float *__restrict__ dval)
{
    __shared__ uint32_t wsum[kBlock / 64];
    const int64_t c = blockIdx.x;
    const FieldDesc d = D[find_field(cs, nf, c)];
    const int64_t lo = (c - d.chunk_start) * kChunk;
    const int64_t hi = min(lo + (int64_t)kChunk, d.n);
    const uint32_t off = (uint32_t)d.offset;
    const int wave = threadIdx.x >> 6;
    int64_t run = base[c];
    for (int64_t r0 = lo; r0 < hi; r0 += kBlock) {
        const int64_t j = r0 + threadIdx.x;
        bool p = false;
        uint32_t s_loc = 0;
        if (j < hi) {
            bool root;
            uint32_t err = 0;
            p = classify<kFromLbl>(T, lbl, off, (uint32_t)d.n, j, s_loc, root, err);
            if (kFromLbl && off != 0 && (p || root)) {
                // minima still hold global ids: make them local
                const uint32_t u = off + (uint32_t)j;
                const uint64_t t = T[u];
                T[u] = pack(lo32(t) - off, hi32(t) - off);
            }
        }
        const uint64_t m = __ballot(p);
        if ((threadIdx.x & 63) == 0) wsum[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t wb = 0, tot = 0;
        for (int w = 0; w < kBlock / 64; ++w) {
            wb += (w < wave) ? wsum[w] : 0u;
            tot += wsum[w];
        }
        if (p) {
            const int64_t pos = run + wb + (uint32_t)__popcll(m & lanemask_lt());
            if (pos < capacity) {
                birth[pos] = (uint32_t)j;
                death[pos] = s_loc;
                bval[pos] = f[off + (uint32_t)j];
                dval[pos] = f[off + s_loc];
            }
        }
        run += tot;
        __syncthreads();
    }
}

__global__ void k_fill0(float *__restrict__ g, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) g[i] = 0.0f;
}

struct BwdGroup {
    int64_t voff[kBwdGroup];  // vertex offset of each field of the group
    int64_t nv[kBwdGroup];    // vertices of each field of the group
    int32_t first, count;
};

// grad[birth] += gb (birth vertices are distinct and are never death
// vertices, so a plain update is race free); grad[death] += gd atomically.
__global__ __launch_bounds__(kBlock) void k_scatter(BwdGroup g, const int64_t *__restrict__ po, int64_t capacity,
                                                    const uint32_t *__restrict__ birth,
                                                    const uint32_t *__restrict__ death,
                                                    const float *__restrict__ gb, const float *__restrict__ gd,
                                                    float *__restrict__ grad)
{
    const int64_t k0 = po[g.first];
    const int64_t k1 = min(po[g.first + g.count], capacity);
    for (int64_t k = k0 + (int64_t)blockIdx.x * kBlock + threadIdx.x; k < k1; k += (int64_t)gridDim.x * kBlock) {
        int lo = 0, hi = g.count;  // po[first+lo] <= k < po[first+hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (po[g.first + mid] <= k) lo = mid; else hi = mid;
        }
        const int64_t vo = g.voff[lo];
        const uint32_t bk = birth[k], dk = death[k];
        if ((int64_t)bk >= g.nv[lo] || (int64_t)dk >= g.nv[lo]) continue;  // not an id of this field
        grad[vo + bk] += gb[k];
        unsafeAtomicAdd(grad + vo + dk, gd[k]);
    }
}

// ---------------------------------------------------------------------------
// host side

struct TileCfg { int tx, ty, tz; };

struct Layout {
    size_t descs, ts, cs, cnt, lbl, total;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Plan {
    std::vector<FieldDesc> d;
    int64_t n_total = 0, n_tiles = 0, n_chunks = 0;
    Layout lay{};
};

static bool parse_tile(const char *s, TileCfg &t, int dims)
{
    int a = 0, b = 1, c = 1;
    int got = sscanf(s, "%dx%dx%d", &a, &b, &c);
    if (got < dims) return false;
    t = {a, b, c};
    return true;
}

static bool tile_ok(TileCfg t, bool cx, bool cy, bool cz)
{
    if (t.tx < 1 || t.ty < 1 || t.tz < 1) return false;
    if ((int64_t)t.tx * t.ty * t.tz > kMaxTileVol) return false;
    const int64_t h = (int64_t)(t.tx + 2 * cx) * (t.ty + 2 * cy) * (t.tz + 2 * cz);
    return h <= kMaxHalo;
}

static std::mutex g_cfg_mu;
static TileCfg g_tile[3] = {{1024, 1, 1}, {64, 16, 1}, {32, 8, 4}};  // 1-D, 2-D, 3-D
static int g_remap = 1;
static uint32_t g_cap = 1u << 24;
static bool g_env_read = false;

static void read_env()
{
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    if (g_env_read) return;
    g_env_read = true;
    TileCfg t;
    if (const char *s = getenv("MT_TILE3D")) if (parse_tile(s, t, 3) && tile_ok(t, 1, 1, 1)) g_tile[2] = t;
    if (const char *s = getenv("MT_TILE2D")) if (parse_tile(s, t, 2) && tile_ok({t.tx, t.ty, 1}, 1, 1, 0)) g_tile[1] = {t.tx, t.ty, 1};
    if (const char *s = getenv("MT_TILE1D")) if (parse_tile(s, t, 1) && tile_ok({t.tx, 1, 1}, 1, 0, 0)) g_tile[0] = {t.tx, 1, 1};
    if (const char *s = getenv("MT_XCD_REMAP")) g_remap = atoi(s) != 0;
    if (const char *s = getenv("MT_MAX_STEPS")) {
        long v = atol(s);
        if (v >= 1 && v <= 0x7fffffffL) g_cap = (uint32_t)v;
    }
}

static int make_plan(const int64_t *dims, int32_t nf, Plan &p)
{
    if (!dims || nf < 1) return MT_ERR_INVALID_ARG;
    read_env();
    p.d.clear();
    p.d.reserve(nf);
    int64_t off = 0, tiles = 0, chunks = 0;
    for (int32_t i = 0; i < nf; ++i) {
        const int64_t nx = dims[3 * i], ny = dims[3 * i + 1], nz = dims[3 * i + 2];
        if (nx < 1 || ny < 1 || nz < 1) return MT_ERR_INVALID_ARG;
        if (nx >= (1LL << 31) || ny >= (1LL << 31) || nz >= (1LL << 31)) return MT_ERR_TOO_LARGE;
        if (nx * ny >= (1LL << 31) || nx * ny * nz >= (1LL << 31)) return MT_ERR_TOO_LARGE;
        const int64_t n = nx * ny * nz;
        const int cls = nz > 1 ? 2 : (ny > 1 ? 1 : 0);
        TileCfg t;
        {
            std::lock_guard<std::mutex> lk(g_cfg_mu);
            t = g_tile[cls];
        }
        FieldDesc d{};
        d.nx = (int32_t)nx; d.ny = (int32_t)ny; d.nz = (int32_t)nz;
        d.tx = t.tx; d.ty = t.ty; d.tz = t.tz;
        d.ntx = (int32_t)((nx + t.tx - 1) / t.tx);
        d.nty = (int32_t)((ny + t.ty - 1) / t.ty);
        d.ntz = (int32_t)((nz + t.tz - 1) / t.tz);
        d.offset = off;
        d.n = n;
        d.tile_start = tiles;
        d.chunk_start = chunks;
        p.d.push_back(d);
        off += n;
        tiles += (int64_t)d.ntx * d.nty * d.ntz;
        chunks += (n + kChunk - 1) / kChunk;
        if (off >= (1LL << 31)) return MT_ERR_TOO_LARGE;
    }
    p.n_total = off;
    p.n_tiles = tiles;
    p.n_chunks = chunks;
    size_t o = align256(sizeof(Header));
    p.lay.descs = o; o = align256(o + sizeof(FieldDesc) * nf);
    p.lay.ts = o; o = align256(o + sizeof(int64_t) * (nf + 1));
    p.lay.cs = o; o = align256(o + sizeof(int64_t) * (nf + 1));
    p.lay.cnt = o; o = align256(o + sizeof(uint32_t) * chunks);
    p.lay.lbl = o; o = align256(o + sizeof(uint32_t) * off);
    p.lay.total = o;
    return MT_OK;
}

struct Ptrs {
    Header *h;
    FieldDesc *D;
    int64_t *ts, *cs;
    uint32_t *cnt, *lbl;
};

static Ptrs ws_ptrs(const Plan &p, void *ws)
{
    char *b = (char *)ws;
    return Ptrs{(Header *)b, (FieldDesc *)(b + p.lay.descs), (int64_t *)(b + p.lay.ts), (int64_t *)(b + p.lay.cs),
                (uint32_t *)(b + p.lay.cnt), (uint32_t *)(b + p.lay.lbl)};
}

#define MT_LAUNCH_CHECK()                                    \
    do {                                                     \
        if (hipGetLastError() != hipSuccess) return MT_ERR_HIP; \
    } while (0)

static unsigned grid1d(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

static int enqueue_setup(const Plan &p, const Ptrs &w, uint32_t clear_status, bool zero_counts, hipStream_t st)
{
    const int nf = (int)p.d.size();
    for (int first = 0; first < nf; first += kSetupMax) {
        SetupArgs a{};
        a.first = first;
        a.count = std::min(kSetupMax, nf - first);
        a.nf = nf;
        a.clear_status = first == 0 ? clear_status : 0u;
        a.zero_counts = zero_counts && first == 0;
        a.total_tiles = p.n_tiles;
        a.total_chunks = p.n_chunks;
        for (int i = 0; i < a.count; ++i) a.d[i] = p.d[first + i];
        hipLaunchKernelGGL(k_setup, dim3(1), dim3(64), 0, st, a, w.D, w.ts, w.cs, w.h);
        MT_LAUNCH_CHECK();
    }
    return MT_OK;
}

static int enqueue_build(const Plan &p, const Ptrs &w, const float *f, uint64_t *T, hipStream_t st)
{
    const int nf = (int)p.d.size();
    uint32_t *status = &w.h->status;
    hipLaunchKernelGGL(k_descend, dim3((unsigned)p.n_tiles), dim3(kBlock), 0, st, f, w.lbl, T, w.D, w.ts, nf,
                       p.n_tiles, g_remap, status);
    MT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_resolve, dim3(grid1d(p.n_total)), dim3(kBlock), 0, st, w.lbl, p.n_total, g_cap, status);
    MT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_merge, dim3((unsigned)p.n_tiles), dim3(kBlock), 0, st, f, (const uint32_t *)w.lbl, T, w.D,
                       w.ts, nf, p.n_tiles, (uint32_t)p.n_total, g_remap, g_cap, status);
    MT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_repair_min, dim3(grid1d(p.n_total)), dim3(kBlock), 0, st, f, (const uint32_t *)w.lbl, T,
                       p.n_total, g_cap, status);
    MT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_repair_reg, dim3((unsigned)p.n_chunks), dim3(kBlock), 0, st, f, (const uint32_t *)w.lbl, T,
                       w.D, w.cs, nf, (uint32_t)p.n_total, g_cap, status);
    MT_LAUNCH_CHECK();
    return MT_OK;
}

template <bool kFromLbl>
static int enqueue_pairs(const Plan &p, const Ptrs &w, const float *f, uint64_t *T, int64_t capacity,
                         uint32_t *birth, uint32_t *death, float *bval, float *dval, int64_t *pair_offsets,
                         hipStream_t st)
{
    const int nf = (int)p.d.size();
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pairs_count<kFromLbl>), dim3((unsigned)p.n_chunks), dim3(kBlock), 0, st,
                       (const uint64_t *)T, (const uint32_t *)w.lbl, w.D, w.cs, nf, w.cnt, w.h);
    MT_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pairs_scan, dim3(1), dim3(1024), 0, st, w.cnt, p.n_chunks, w.D, nf, pair_offsets, capacity,
                       w.h);
    MT_LAUNCH_CHECK();
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_pairs_write<kFromLbl>), dim3((unsigned)p.n_chunks), dim3(kBlock), 0, st, f, T,
                       (const uint32_t *)w.lbl, w.D, w.cs, nf, (const uint32_t *)w.cnt, capacity, birth, death, bval,
                       dval);
    MT_LAUNCH_CHECK();
    return MT_OK;
}

static int status_to_code(uint32_t s)
{
    if (s & ST_NAN) return MT_ERR_NAN;
    if (s & ST_CORRUPT) return MT_ERR_INTERNAL;
    if (s & ST_LIVELOCK) return MT_ERR_LIVELOCK;
    if (s & ST_CAPACITY) return MT_ERR_CAPACITY;
    return MT_OK;
}

static int read_header(const void *ws, hipStream_t st, Header &h)
{
    if (hipMemcpyAsync(&h, ws, sizeof(Header), hipMemcpyDeviceToHost, st) != hipSuccess) return MT_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return MT_ERR_HIP;
    return MT_OK;
}

// Batch graph cache ----------------------------------------------------------

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static std::mutex g_graph_mu;
static std::unordered_map<std::string, GraphEntry> g_graphs;
static std::unordered_map<int, hipStream_t> g_capture_streams;

static hipStream_t capture_stream(int dev)
{
    auto it = g_capture_streams.find(dev);
    if (it != g_capture_streams.end()) return it->second;
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return nullptr;
    g_capture_streams[dev] = s;
    return s;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI

extern "C" {

const char *mt_status_string(int status)
{
    switch (status) {
    case MT_OK: return "MT_OK";
    case MT_ERR_INVALID_ARG: return "MT_ERR_INVALID_ARG";
    case MT_ERR_TOO_LARGE: return "MT_ERR_TOO_LARGE";
    case MT_ERR_NAN: return "MT_ERR_NAN";
    case MT_ERR_CAPACITY: return "MT_ERR_CAPACITY";
    case MT_ERR_LIVELOCK: return "MT_ERR_LIVELOCK";
    case MT_ERR_WORKSPACE: return "MT_ERR_WORKSPACE";
    case MT_ERR_HIP: return "MT_ERR_HIP";
    case MT_ERR_INTERNAL: return "MT_ERR_INTERNAL";
    default: return "MT_ERR_UNKNOWN";
    }
}

size_t mt_workspace_bytes(int64_t nx, int64_t ny, int64_t nz)
{
    const int64_t dims[3] = {nx, ny, nz};
    Plan p;
    if (make_plan(dims, 1, p) != MT_OK) return 0;
    return p.lay.total;
}

size_t mt_batch_workspace_bytes(const int64_t *dims, int32_t n_fields)
{
    Plan p;
    if (make_plan(dims, n_fields, p) != MT_OK) return 0;
    return p.lay.total;
}

int mt_build(const float *field, int64_t nx, int64_t ny, int64_t nz, uint32_t *triplets, void *workspace,
             size_t ws_bytes, void *stream)
{
    const int64_t dims[3] = {nx, ny, nz};
    Plan p;
    int rc = make_plan(dims, 1, p);
    if (rc != MT_OK) return rc;
    if (!field || !triplets || ((uintptr_t)triplets & 7u)) return MT_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace & 255u) || ws_bytes < p.lay.total) return MT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const Ptrs w = ws_ptrs(p, workspace);
    rc = enqueue_setup(p, w, ~0u, true, st);
    if (rc != MT_OK) return rc;
    return enqueue_build(p, w, field, (uint64_t *)triplets, st);
}

int mt_persistence_pairs(const float *field, const uint32_t *triplets, int64_t nx, int64_t ny, int64_t nz,
                         uint32_t *birth, uint32_t *death, float *birth_val, float *death_val, int64_t capacity,
                         int64_t *n_pairs, int64_t *n_roots, void *workspace, size_t ws_bytes, void *stream)
{
    const int64_t dims[3] = {nx, ny, nz};
    Plan p;
    int rc = make_plan(dims, 1, p);
    if (rc != MT_OK) return rc;
    if (!field || !triplets || ((uintptr_t)triplets & 7u) || !n_pairs || capacity < 0) return MT_ERR_INVALID_ARG;
    if (capacity > 0 && (!birth || !death || !birth_val || !death_val)) return MT_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace & 255u) || ws_bytes < p.lay.total) return MT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    const Ptrs w = ws_ptrs(p, workspace);
    rc = enqueue_setup(p, w, ST_CAPACITY | ST_CORRUPT, true, st);
    if (rc != MT_OK) return rc;
    rc = enqueue_pairs<false>(p, w, field, (uint64_t *)triplets, capacity, birth, death, birth_val, death_val,
                              nullptr, st);
    if (rc != MT_OK) return rc;
    Header h;
    rc = read_header(workspace, st, h);
    if (rc != MT_OK) return rc;
    *n_pairs = h.total_pairs;
    if (n_roots) *n_roots = h.roots;
    return status_to_code(h.status);
}

int mt_batch_build(const float *fields, const int64_t *dims, int32_t n_fields, uint32_t *triplets, uint32_t *birth,
                   uint32_t *death, float *birth_val, float *death_val, int64_t pair_capacity,
                   int64_t *pair_offsets, void *workspace, size_t ws_bytes, void *stream)
{
    Plan p;
    int rc = make_plan(dims, n_fields, p);
    if (rc != MT_OK) return rc;
    if (!fields || !triplets || ((uintptr_t)triplets & 7u) || !pair_offsets || pair_capacity < 0)
        return MT_ERR_INVALID_ARG;
    if (pair_capacity > 0 && (!birth || !death || !birth_val || !death_val)) return MT_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace & 255u) || ws_bytes < p.lay.total) return MT_ERR_WORKSPACE;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MT_ERR_HIP;
    std::string key;
    key.reserve(64 + 24 * n_fields);
    char buf[256];
    snprintf(buf, sizeof buf, "%d|%p|%p|%p|%p|%p|%p|%lld|%p|%p|%zu|%d|%u", dev, (const void *)fields,
             (void *)triplets, (void *)birth, (void *)death, (void *)birth_val, (void *)death_val,
             (long long)pair_capacity, (void *)pair_offsets, workspace, ws_bytes, g_remap, g_cap);
    key += buf;
    for (const FieldDesc &d : p.d) {
        snprintf(buf, sizeof buf, "|%d,%d,%d:%d,%d,%d", d.nx, d.ny, d.nz, d.tx, d.ty, d.tz);
        key += buf;
    }

    std::lock_guard<std::mutex> lk(g_graph_mu);
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        hipStream_t cs = capture_stream(dev);
        if (!cs) return MT_ERR_HIP;
        const Ptrs w = ws_ptrs(p, workspace);
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) return MT_ERR_HIP;
        int rc1 = enqueue_setup(p, w, ~0u, true, cs);
        if (rc1 == MT_OK) rc1 = enqueue_build(p, w, fields, (uint64_t *)triplets, cs);
        if (rc1 == MT_OK)
            rc1 = enqueue_pairs<true>(p, w, fields, (uint64_t *)triplets, pair_capacity, birth, death, birth_val,
                                      death_val, pair_offsets, cs);
        GraphEntry e;
        const hipError_t ec = hipStreamEndCapture(cs, &e.graph);
        if (rc1 != MT_OK || ec != hipSuccess) {
            if (e.graph) hipGraphDestroy(e.graph);
            return rc1 != MT_OK ? rc1 : MT_ERR_HIP;
        }
        if (hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess) {
            hipGraphDestroy(e.graph);
            return MT_ERR_HIP;
        }
        it = g_graphs.emplace(key, e).first;
    }
    if (hipGraphLaunch(it->second.exec, (hipStream_t)stream) != hipSuccess) return MT_ERR_HIP;
    return MT_OK;
}

int mt_sync_status(const void *workspace, void *stream, int64_t *n_pairs, int64_t *n_roots)
{
    if (!workspace) return MT_ERR_WORKSPACE;
    Header h;
    const int rc = read_header(workspace, (hipStream_t)stream, h);
    if (rc != MT_OK) return rc;
    if (n_pairs) *n_pairs = h.total_pairs;
    if (n_roots) *n_roots = h.roots;
    return status_to_code(h.status);
}

int mt_pairs_backward(const int64_t *dims, int32_t n_fields, const int64_t *pair_offsets, int64_t pair_capacity,
                      const uint32_t *birth, const uint32_t *death, const float *grad_birth,
                      const float *grad_death, float *grad_field, int accumulate, void *stream)
{
    if (!dims || n_fields < 1 || !pair_offsets || !grad_field || pair_capacity < 0) return MT_ERR_INVALID_ARG;
    if (pair_capacity > 0 && (!birth || !death || !grad_birth || !grad_death)) return MT_ERR_INVALID_ARG;
    std::vector<int64_t> voff(n_fields + 1);
    int64_t off = 0;
    for (int32_t i = 0; i < n_fields; ++i) {
        const int64_t nx = dims[3 * i], ny = dims[3 * i + 1], nz = dims[3 * i + 2];
        if (nx < 1 || ny < 1 || nz < 1) return MT_ERR_INVALID_ARG;
        if (nx >= (1LL << 31) || ny >= (1LL << 31) || nz >= (1LL << 31)) return MT_ERR_TOO_LARGE;
        if (nx * ny * nz >= (1LL << 31)) return MT_ERR_TOO_LARGE;
        voff[i] = off;
        off += nx * ny * nz;
        if (off >= (1LL << 31)) return MT_ERR_TOO_LARGE;
    }
    voff[n_fields] = off;
    hipStream_t st = (hipStream_t)stream;
    if (!accumulate) {
        hipLaunchKernelGGL(k_fill0, dim3(grid1d(off)), dim3(kBlock), 0, st, grad_field, off);
        MT_LAUNCH_CHECK();
    }
    if (pair_capacity == 0) return MT_OK;
    const unsigned blocks = (unsigned)std::min<int64_t>(2048, (pair_capacity + kBlock - 1) / kBlock);
    for (int32_t first = 0; first < n_fields; first += kBwdGroup) {
        BwdGroup g{};
        g.first = first;
        g.count = std::min<int32_t>(kBwdGroup, n_fields - first);
        for (int i = 0; i < g.count; ++i) {
            g.voff[i] = voff[first + i];
            g.nv[i] = voff[first + i + 1] - voff[first + i];
        }
        hipLaunchKernelGGL(k_scatter, dim3(blocks), dim3(kBlock), 0, st, g, pair_offsets, pair_capacity, birth,
                           death, grad_birth, grad_death, grad_field);
        MT_LAUNCH_CHECK();
    }
    return MT_OK;
}

void mt_release_caches(void)
{
    std::lock_guard<std::mutex> lk(g_graph_mu);
    for (auto &kv : g_graphs) {
        if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) hipGraphDestroy(kv.second.graph);
    }
    g_graphs.clear();
    for (auto &kv : g_capture_streams) hipStreamDestroy(kv.second);
    g_capture_streams.clear();
}

}  // extern "C"
