// mt_device.h -- device code of the triplet merge tree library (gfx950).
//
// Included once, by mt.hip.  The method is the triplet merge tree of "Fast
// Merge Tree Computation via SYCL" (arXiv 2301.10838): Sec. 2, Alg. 1-5, with
// the GPU layout of Sec. 3.2 (a triplet (u, s, v) is stored as T[u] = (s, v),
// two 32-bit ids packed into one 64-bit word, so one 64-bit compare-and-swap
// replaces it atomically).
//
// Pipeline of one build (every field of a batch at once):
//
//   k_local<S>      one workgroup per tile, everything in LDS: the merge tree
//                   of the tile's own subgraph.  Each vertex points at its
//                   lowest lower neighbour inside the tile, chains are
//                   followed to the tile-local minimum, every edge inside the
//                   tile joining two different local basins is merged
//                   (Alg. 3 with LDS compare-and-swap) and the local minima
//                   are repaired (Alg. 5).  The tile's local minima get
//                   consecutive "minimum numbers"; their triplets go to the
//                   global minima array and every vertex records the number
//                   of its local basin.
//   k_cross<S>      one workgroup per tile: Merge (Alg. 3 with 64-bit
//                   compare-and-swap in global memory) of every edge that
//                   leaves the tile through its +x, +y, +z faces, between the
//                   local minima of its two ends.
//   k_repair_min    Repair of every local minimum.
//   k_repair_reg    every vertex's output triplet: a local minimum copies its
//                   own, any other vertex u gets (u, u, representative of its
//                   local minimum at the level of u); pair counts per chunk.
//   k_pairs_*       pairs read out of T in ascending birth id.
//
// Why this computes the paper's tree.  Alg. 1 merges the edges in any order,
// and the triplet representation that is both normalized and minimal is
// unique (Sec. 2), so every schedule of merges followed by a repair ends in
// the same T.  (1) Pointing each vertex at its lowest lower neighbour is the
// state Merge reaches when those edges are merged one by one in decreasing
// order of their upper vertex.  (2) Following those pointers to the minimum
// z(u) they reach only shortens links that all lie below u, so (u, u, z(u))
// represents the same connectivity; an edge whose two ends reach the same
// minimum then joins vertices already connected below its upper end and needs
// no merge, and any other edge (a, b) is the fact "z(a) and z(b) are
// connected at the level of max(a, b)".  (3) Merging the edges inside each
// tile first (and repairing), then the edges between tiles, is one more
// schedule of the same merges.  Only minima ever carry a changing triplet.
//
// Minimum slots.  Minimum number m owns a 16-byte slot: w = (saddle id,
// target number) is the triplet, replaced by 64-bit compare-and-swap; k is
// the 64-bit order key of w's saddle, stored after every successful swap.  A
// reader uses k only if its id part matches the saddle it read in w, and
// otherwise reads the saddle's value from the field, so a stale k costs time,
// never correctness.  mkey[m] is the key of the minimum itself.
//
// Order.  Vertices compare by (value, id) with IEEE semantics: the float is
// mapped to an order-preserving uint32 with -0.0 folded onto +0.0, and the id
// is appended, so every comparison is one 64-bit integer compare.  Inside a
// tile the id is replaced by the position in the tile, which orders the same
// way (both grow with z, then y, then x).
//
// Safety.  Every id read back from memory is range-checked before it is used
// as an address; a failed check latches ST_CORRUPT instead of faulting, and
// every loop is bounded by a step cap that latches ST_LIVELOCK.

#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mtd {

constexpr int kBlock = 256;                  // threads per workgroup of the flat passes
constexpr int kChunk = 4096;                 // vertices per workgroup in flat passes
constexpr int kSetupMax = 12;                // field descriptors per k_setup launch
constexpr int kBwdGroup = 64;                // fields per backward launch
constexpr int kXFace = 256;                  // largest x face of a tile shape (TY * TZ)
// Cross-tile facts are binned by the top bits of their saddle key (sign and
// exponent of the value: coarse on purpose, since within a bin the facts
// keep roughly their queue order, i.e. stay grouped by tile, which keeps the
// slots that concurrent merges touch close; the lanes in flight span many
// such bins anyway).  Each bin's counter has kQCopies copies (chosen by the
// fact's queue position, so the counting and the scattering pass agree),
// which keeps the atomics on one bin apart.
constexpr int kMaxProbes = 32;               // pair-table probes per edge, at most (and the default)
constexpr int kQBinBits = 9;
constexpr int kQBins = 1 << kQBinBits;
constexpr int kQCopies = 16;
constexpr int kQChunkBits = 10;              // queue positions per copy turn
constexpr int kQCounters = kQBins * kQCopies;  // per XCD
__host__ __device__ constexpr uint32_t qcounter(uint32_t pos, uint64_t ks)
{
    return (((pos >> kQChunkBits) % kQCopies) << kQBinBits) | (uint32_t)(ks >> (64 - kQBinBits));
}

constexpr uint32_t ST_NAN = 1u, ST_LIVELOCK = 2u, ST_CAPACITY = 4u, ST_CORRUPT = 8u;

struct FieldDesc {
    int32_t nx, ny, nz;
    int32_t ntx, nty, ntz;   // tiles along each axis
    int32_t tpos;            // position of the field in tile order
    int32_t pad;
    int64_t offset;          // global id of the first vertex
    int64_t n;               // vertices
    int64_t tile_start;      // first tile (tile order)
    int64_t chunk_start;     // first chunk (field order)
};

// Event counts of a counting build (mt_set_counting).  The timed build is a
// separate instantiation of the same kernels with every count compiled out.
enum CtrId {
    C_GM_FACTS,       // cross-tile merges started (one per queued fact)
    C_GM_STEPS,       // iterations of the cross-tile merge loop
    C_GM_DESCENTS,    // of those, descent steps (a link followed)
    C_GM_CAS,         // 64-bit compare-and-swaps on the slots
    C_GM_CAS_FAIL,    // of those, failed
    C_GM_REMERGE,     // displaced triplets merged again
    C_GM_MAX_STEPS,   // most iterations of one cross-tile merge (a maximum)
    C_LDS_MERGES,     // merges inside a tile
    C_LDS_STEPS,      // iterations of the in-tile merge loop
    C_LDS_CAS,        // 64-bit LDS compare-and-swaps
    C_LDS_CAS_FAIL,   // of those, failed
    C_LDS_MAX_STEPS,  // most iterations of one in-tile merge (a maximum)
    C_TAB_INSERTS,    // edges offered to the in-tile pair table
    C_TAB_PROBES,     // atomic-min probes of those inserts
    C_TAB_DIRECT,     // edges without table room (overflow list), or without a table (merged at once)
    C_REG_CHASES,     // chase steps of the output pass
    C_GM_COMPRESS,    // path compressions in cross-tile descents
    C_MIN_CHASES,     // chase steps of the minimum repair
    // shader clock cycles of each barrier-separated phase of the tile pass,
    // summed over tiles (taken by the workgroup's first lane, so each phase
    // includes the wait for its slowest wave)
    C_PH_LOAD,        // field loads awaited, order keys into LDS
    C_PH_DESCENT,     // lowest lower neighbour of every vertex
    C_PH_NUMBER,      // local minima numbered, their records initialised
    C_PH_BASIN,       // descent chains followed to the local minimum
    C_PH_CLEAR,       // field loads issued and the pair table cleared (from the workgroup's start)
    C_PH_INSERT,      // edges between basins marked and offered to the table
    C_PH_COMPACT,     // occupied table entries compacted
    C_PH_MERGE,       // merges of the kept edges (Alg. 3 in LDS)
    C_PH_REPAIR,      // repair of the local minima (Alg. 5)
    C_PH_LABEL,       // minimum records written, vertices labelled
    C_TAB_REDO,       // tiles whose overflow list filled up (all their edges merged at once)
    C_REG_ROUNDS,     // rounds of the output pass's chase loop, per wave and vertex group
    kCtr
};
__host__ __device__ constexpr bool ctr_is_max(int i) { return i == C_GM_MAX_STEPS || i == C_LDS_MAX_STEPS; }

constexpr int kXStride = 32;  // one 128-byte line per XCD queue counter
struct Header {
    uint32_t status;
    uint32_t n_minima;       // minimum numbers handed out
    int64_t total_pairs;
    int64_t roots;
    int64_t reserved[1];
    // cross-tile facts queued for XCD x at n_cross[x * kXStride]: every
    // workgroup of an XCD reserves its queue room here, so the counters
    // stay on lines of their own
    alignas(128) uint32_t n_cross[8 * kXStride];
    alignas(128) unsigned long long ctr[kCtr];  // counting build only
};

// Per-lane event counts, flushed with one atomic per wave; empty when CNT is
// false.  flush() must be reached by every lane of the wave.
template <bool CNT>
struct Tally {
    uint32_t v[CNT ? kCtr : 1];
    __device__ Tally()
    {
        if constexpr (CNT)
            for (int i = 0; i < kCtr; ++i) v[i] = 0;
    }
    __device__ __forceinline__ void add(int id, uint32_t x = 1)
    {
        if constexpr (CNT) v[id] += x;
    }
    __device__ __forceinline__ void max(int id, uint32_t x)
    {
        if constexpr (CNT) v[id] = v[id] > x ? v[id] : x;
    }
    __device__ void flush(Header *h)
    {
        if constexpr (CNT) {
#pragma unroll
            for (int i = 0; i < kCtr; ++i) {
                unsigned long long x = v[i];
                for (int o = 32; o > 0; o >>= 1) {
                    const unsigned long long y = __shfl_xor(x, o);
                    x = ctr_is_max(i) ? (x > y ? x : y) : x + y;
                }
                if ((threadIdx.x & 63) == 0 && x) {
                    if (ctr_is_max(i)) atomicMax(&h->ctr[i], x);
                    else atomicAdd(&h->ctr[i], x);
                }
            }
        }
    }
};

// A fact "minima a and b are connected at the level of the saddle whose key
// is ks", queued for the cross-tile merge.
struct Fact {
    uint32_t a, b;
    uint64_t ks;
};

struct alignas(16) Slot {
    uint64_t w;  // (saddle id, target number): the triplet
    uint64_t k;  // order key of the saddle, valid if its low half equals w's saddle
};

// ---------------------------------------------------------------------------
// helpers

__device__ __forceinline__ uint32_t okey(float x)
{
    uint32_t b = __float_as_uint(x);
    b = (b == 0x80000000u) ? 0u : b;  // -0.0 == +0.0
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// flip = 0: the order of the values (merge tree, sublevel sets); flip = ~0:
// the reversed order (split tree, superlevel sets = the merge tree of -f),
// ids still breaking ties upward.
__device__ __forceinline__ uint64_t vkey(const float *__restrict__ f, uint32_t id, uint32_t flip)
{
    return ((uint64_t)(okey(f[id]) ^ flip) << 32) | id;
}

__device__ __forceinline__ uint32_t lo32(uint64_t t) { return (uint32_t)t; }
__device__ __forceinline__ uint32_t hi32(uint64_t t) { return (uint32_t)(t >> 32); }
__device__ __forceinline__ uint64_t pack(uint32_t s, uint32_t v) { return (uint64_t)s | ((uint64_t)v << 32); }

// Output id width.  Internally every id is a uint32 (a batch holds fewer than
// 2^32 - 1 vertices); the output either keeps that width (T[u] = one 64-bit
// word (s, v), the packing of Sec. 3.2, pair ids uint32) or widens it for
// callers that index with 64-bit integers (T[u] = two uint64 in one 16-byte
// word, pair ids uint64).
struct Out32 {
    using Id = uint32_t;
    using Word = uint64_t;
    __device__ static void store(Word *T, uint32_t u, uint32_t s, uint32_t v) { T[u] = pack(s, v); }
    __device__ static void load(const Word *T, uint32_t u, uint32_t &s, uint32_t &v)
    {
        const uint64_t t = T[u];
        s = lo32(t);
        v = hi32(t);
    }
};
struct Out64 {
    using Id = uint64_t;
    using Word = ulonglong2;
    __device__ static void store(Word *T, uint32_t u, uint32_t s, uint32_t v) { T[u] = make_ulonglong2(s, v); }
    __device__ static void load(const Word *T, uint32_t u, uint32_t &s, uint32_t &v)
    {
        const ulonglong2 t = T[u];
        // ids written by this library fit 32 bits; anything else fails the range checks
        s = t.x >> 32 ? 0xffffffffu : (uint32_t)t.x;
        v = t.y >> 32 ? 0xffffffffu : (uint32_t)t.y;
    }
};

// Untorn 64-bit read/write of a slot word.  The merge phase reads through the
// cache: a stale triplet is a fact that held earlier and still holds, and
// the compare-and-swap, which always sees the current word, hands back the
// fresh value when the read was stale.
template <typename T>
__device__ __forceinline__ T ld_relaxed(T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Both words of a slot.
struct SlotRead {
    uint64_t w, k;
};

// A slot that other lanes may be replacing in the same kernel (the cross-tile
// merge, the minimum repair): each word is read by its own relaxed atomic
// load, so it arrives whole; the two may come from different moments, which
// the id check on k absorbs.  Wavefront scope keeps the read cached: a stale
// word is a triplet that held earlier and still holds, and the
// compare-and-swap, which always sees the current word, hands back the fresh
// one when the read was stale.
__device__ __forceinline__ SlotRead ld_slot_live(Slot *__restrict__ S, uint32_t x)
{
    SlotRead r;
    r.w = ld_relaxed(&S[x].w);
    r.k = ld_relaxed(&S[x].k);
    return r;
}

// Key of the saddle of a slot read: the cached key if it belongs to that
// saddle, else the value read from the field.
__device__ __forceinline__ uint64_t saddle_key(const SlotRead &r, const float *__restrict__ f, uint32_t flip)
{
    const uint32_t s = lo32(r.w);
    return lo32(r.k) == s ? r.k : vkey(f, s, flip);
}

template <typename I>
__device__ __forceinline__ int search(const I *__restrict__ starts, int nf, int64_t t)
{
    int lo = 0, hi = nf;  // starts[lo] <= t < starts[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)starts[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous
// run of tiles so that neighbouring tiles (which share halo lines) share an L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G, int remap)
{
    if (!remap || G < 8) return b;
    const int64_t per = G / 8, rem = G % 8;
    const int64_t x = b % 8, j = b / 8;
    return x * per + (x < rem ? x : rem) + j;
}

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const int lane = threadIdx.x & 63;
    return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Position of the k-th set bit (k < popcount) of a 64-bit word, by halving.
__device__ __forceinline__ uint32_t select_bit(uint64_t m, uint32_t k)
{
    uint32_t pos = 0;
#pragma unroll
    for (int w = 32; w >= 1; w >>= 1) {
        const uint32_t c = (uint32_t)__popcll(m & ((1ull << w) - 1));
        if (k >= c) { k -= c; pos += w; m >>= w; }
    }
    return pos;
}

// Tile shape and workgroup size.
template <int X, int Y, int Z, int NTHREADS>
struct Shape {
    static constexpr int TX = X, TY = Y, TZ = Z, VOL = X * Y * Z, NT = NTHREADS;
    static_assert(VOL % NT == 0 && NT % 64 == 0 && VOL <= 4096, "tile volume");
    static_assert((X & (X - 1)) == 0 && (Y & (Y - 1)) == 0 && (Z & (Z - 1)) == 0, "powers of two");
};

struct TileCtx {
    FieldDesc d;
    int64_t t;   // global tile index
    int x0, y0, z0, ex, ey, ez;
    int64_t sxy;
};

template <class S>
__device__ __forceinline__ TileCtx tile_ctx(const FieldDesc *__restrict__ D, const int32_t *__restrict__ tfield,
                                            const int64_t *__restrict__ tstart, int nfc, int64_t t)
{
    TileCtx c;
    const int k = search(tstart, nfc, t);
    c.d = D[tfield[k]];
    c.t = t;
    const int64_t lt = t - c.d.tile_start;
    const int bx = (int)(lt % c.d.ntx);
    const int64_t r = lt / c.d.ntx;
    const int by = (int)(r % c.d.nty);
    const int bz = (int)(r / c.d.nty);
    c.x0 = bx * S::TX; c.y0 = by * S::TY; c.z0 = bz * S::TZ;
    c.ex = min(S::TX, c.d.nx - c.x0);
    c.ey = min(S::TY, c.d.ny - c.y0);
    c.ez = min(S::TZ, c.d.nz - c.z0);
    c.sxy = (int64_t)c.d.nx * c.d.ny;
    return c;
}

// ---------------------------------------------------------------------------
// setup

struct SetupArgs {
    FieldDesc d[kSetupMax];
    int32_t first, count, nf;
    uint32_t clear_status;  // status bits to clear
    int32_t zero_counts;
    int32_t pad;
    int64_t total_tiles, total_chunks;
};

__global__ void k_setup(SetupArgs a, FieldDesc *D, int32_t *tfield, int64_t *tstart, int64_t *cs, Header *h)
{
    const int i = threadIdx.x;
    if (i < a.count) {
        const FieldDesc d = a.d[i];
        D[a.first + i] = d;
        tfield[d.tpos] = a.first + i;
        tstart[d.tpos] = d.tile_start;
        cs[a.first + i] = d.chunk_start;
    }
    if (i == 0) {
        if (a.first + a.count == a.nf) {
            tstart[a.nf] = a.total_tiles;
            cs[a.nf] = a.total_chunks;
        }
        if (a.clear_status) h->status &= ~a.clear_status;
        if (a.zero_counts) {
            h->total_pairs = 0;
            h->roots = 0;
            h->n_minima = 0;
            for (int x = 0; x < 8; ++x) h->n_cross[x * kXStride] = 0;
            for (int c = 0; c < kCtr; ++c) h->ctr[c] = 0;
        }
    }
}

// ---------------------------------------------------------------------------
// 1. merge tree of each tile's subgraph, in LDS

// Tile order key of tile position p: (order key of the value << PB) | p, PB =
// log2 of the tile volume.  It orders tile vertices exactly as the global key
// does (positions grow with the id inside a tile).
template <int PB>
__device__ __forceinline__ uint64_t lkey(const uint32_t *hk, uint32_t p)
{
    return ((uint64_t)hk[p] << PB) | p;
}

// LDS triplet of local minimum i, one 64-bit word: (tile key of the saddle <<
// TB) | target (local minimum index).  A root is (own key, own index).  A
// descent step is one load and one compare, and the word is replaced by one
// 64-bit compare-and-swap.
template <int VOL>
struct LTrip {
    static constexpr int PB = __builtin_ctz(VOL);
    static constexpr int TB = 32 - PB;                 // target bits
    static constexpr uint64_t TM = (1ull << TB) - 1;
    static_assert(PB - 1 <= TB, "every local minimum index fits the target bits");
    __device__ static uint64_t make(uint64_t key, uint32_t t) { return (key << TB) | t; }
    __device__ static uint32_t tgt(uint64_t w) { return (uint32_t)(w & TM); }
    __device__ static uint64_t key(uint64_t w) { return w >> TB; }
};

__device__ __forceinline__ uint64_t lds_ld64(uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Merge (Alg. 3) of "local minima u and v are connected at the level whose
// tile key is ks".  Descents stop at roots; after a swap that replaced a root
// nothing was displaced; otherwise the displaced triplet is merged again from
// the lower minimum; a lost swap restarts with the value it saw.
template <int VOL, bool CNT>
__device__ void lds_merge(uint64_t *TL, const uint32_t *hk, const uint16_t *mh, uint32_t u, uint64_t ks,
                          uint32_t v, uint32_t cnt, uint32_t cap, uint32_t &err, Tally<CNT> &tc)
{
    using L = LTrip<VOL>;
    tc.add(C_LDS_MERGES);
    if (u >= cnt || v >= cnt) { err |= ST_CORRUPT; return; }
    uint64_t tu = lds_ld64(TL + u), tv = lds_ld64(TL + v);
    // A word's key lies below ks exactly when the word lies below ks << TB
    // (its target fills the low TB bits), so the descent tests compare whole
    // words; a replacement word (ks, u) is that bound with u in the low bits.
    uint64_t ksT = ks << L::TB;
    // (every exit returns from inside the loop: the timed build, in which
    // done() is empty, keeps the loop's exits apart)
    auto done = [&](uint32_t steps) {
        tc.add(C_LDS_STEPS, steps);
        tc.max(C_LDS_MAX_STEPS, steps);
    };
    for (uint32_t step = 0; step < cap; ++step) {
        const uint32_t u1 = L::tgt(tu), v1 = L::tgt(tv);
        if (u1 >= cnt || v1 >= cnt) { err |= ST_CORRUPT; done(step + 1); return; }
        // one descent step, u's before v's: a link below the merge's level
        const bool du = u1 != u && tu < ksT;
        const bool dv = v1 != v && tv < ksT;
        if (du || dv) {
            const uint32_t x = du ? u1 : v1;
            const uint64_t t = lds_ld64(TL + x);
            if (du) { u = x; tu = t; } else { v = x; tv = t; }
            continue;
        }
        if (u == v) { done(step + 1); return; }
        // the upper minimum is re-pointed: tile keys compared as (value key, position)
        const uint32_t pu = mh[u], pv = mh[v];
        const uint32_t ku = hk[pu], kv = hk[pv];
        if (kv < ku || (kv == ku && pv < pu)) {
            const uint32_t w = u; u = v; v = w;
            const uint64_t tw = tu; tu = tv; tv = tw;
        }
        uint64_t seen = tv;
        tc.add(C_LDS_CAS);
        if (__hip_atomic_compare_exchange_strong(TL + v, &seen, ksT | u, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
            if (L::tgt(tv) == v) { done(step + 1); return; }
            ksT = tv & ~L::TM;  // merge the displaced triplet again, at its own level
            v = L::tgt(tv);
            tv = lds_ld64(TL + v);
        } else {
            tc.add(C_LDS_CAS_FAIL);
            tv = seen;
        }
        tu = lds_ld64(TL + u);
    }
    done(cap);
    err |= ST_LIVELOCK;
}

// MODE 0: the timed kernel; 1: counting build (event counts); 2: phase
// clocks only (the tile pass's phases timed by the workgroup's first lane
// into LDS, added to the counters once per workgroup; no event counts, whose
// per-lane registers would slow the phases down).
template <class S, int MODE, bool LIMIT>
__global__ __launch_bounds__(S::NT, 8) void k_local(const float *__restrict__ f, uint32_t *__restrict__ lbl,
                                                 Slot *__restrict__ slot, uint64_t *__restrict__ mkey,
                                                 const FieldDesc *__restrict__ D, const int32_t *__restrict__ tfield,
                                                 const int64_t *__restrict__ tstart, int nfc, int64_t tile0,
                                                 int64_t ntiles, int remap, uint32_t mcap, uint32_t cap,
                                                 uint64_t *__restrict__ xface, uint32_t flip,
                                                 uint32_t probes, Header *__restrict__ h)
{
    constexpr int NT = S::NT, VOL = S::VOL, TX = S::TX, TY = S::TY;
    static_assert(S::TY * S::TZ <= kXFace, "x face record");
    constexpr int HALF = VOL / 2;   // local minima are pairwise non-adjacent: at most half the tile
    using L = LTrip<VOL>;
    constexpr int PB = L::PB;
    // Basin-pair table: one 64-bit word per entry holding the lowest edge of
    // the pair, (tile key of its upper end << 2ZB | lo | hi << ZB), so
    // claiming an entry and lowering its edge are one word each.
    constexpr int ZB = (32 - PB) / 2;            // bits of a minimum number in a tag
    constexpr uint32_t ZMAX = 1u << ZB;          // the table is used when the tile has at most ZMAX minima
    constexpr uint64_t TAGM = (1ull << (2 * ZB)) - 1;
    constexpr int H = VOL;
    static_assert((VOL & (VOL - 1)) == 0 && PB + 2 * ZB <= 32, "tag layout");
    __shared__ uint32_t hk[VOL];    // order key of every tile vertex
    __shared__ uint16_t zl[VOL];    // local minimum index of the vertex's local basin
    __shared__ uint64_t TL[HALF];   // triplets of the local minima
    __shared__ uint16_t mh[HALF];   // tile position of local minimum i
    __shared__ uint64_t htab[H];    // the pair table
    // The lowest-neighbour pointers are dead once the basins are known, and
    // the triplets' space is first written after that: the pointers live
    // there, so that the table can be cleared while the field loads.
    typedef int16_t __attribute__((may_alias)) i16a;
    i16a *const wl = (i16a *)TL;    // lowest lower neighbour in the tile (self at a local minimum)
    static_assert(sizeof(int16_t) * VOL <= sizeof(uint64_t) * HALF, "aliasing");
    __shared__ uint32_t wsum[VOL / 64];
    __shared__ uint32_t sb0, nwin, scnt, novf;
    // edges that found no table room, merged with the table's entries (a
    // count above kOvf sends the tile down the direct path instead)
    constexpr uint32_t kOvf = 64;
    __shared__ uint64_t ovf[kOvf];

    const int64_t tl = xcd_tile(blockIdx.x, gridDim.x, remap);
    if (tl >= ntiles) return;
    constexpr bool CNT = MODE == 1;
    Tally<CNT> tc;
    __shared__ uint32_t phc[MODE == 2 ? kCtr : 1];  // phase clocks of this workgroup
    uint64_t ph_t = 0;                              // clock at the end of the previous phase
    if constexpr (MODE == 2) {
        if (threadIdx.x == 0) {
            for (int i = 0; i < kCtr; ++i) phc[i] = 0;
            ph_t = clock64();
        }
    }
    auto phase = [&](int id) {
        if constexpr (MODE == 2) {
            if (threadIdx.x == 0) {
                const uint64_t t = clock64();
                phc[id] += (uint32_t)(t - ph_t);
                ph_t = t;
            }
        }
    };
    const TileCtx c = tile_ctx<S>(D, tfield, tstart, nfc, tile0 + tl);
    const uint32_t off = (uint32_t)c.d.offset;
    auto valid = [&](int lx, int ly, int lz) { return lx < c.ex && ly < c.ey && lz < c.ez; };
    // Ids in 32 bits: every id of the batch is below 2^32 - 2.
    const uint32_t nx = (uint32_t)c.d.nx, sxy = (uint32_t)c.sxy;
    const uint32_t base = off + (uint32_t)c.x0 + nx * (uint32_t)c.y0 + sxy * (uint32_t)c.z0;
    auto lid = [&](int lx, int ly, int lz) { return (uint32_t)lx + nx * (uint32_t)ly + sxy * (uint32_t)lz; };
    auto gid = [&](int p) {
        const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
        return base + lid(lx, ly, lz);
    };
    constexpr int PER = VOL / NT;  // vertices per lane

    {
        // all of a lane's loads in flight together; positions outside the
        // field read a clamped in-field address and are then discarded
        float fv[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int p = k * NT + threadIdx.x;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            fv[k] = f[base + lid(min(lx, c.ex - 1), min(ly, c.ey - 1), min(lz, c.ez - 1))];
        }
        // the pair table cleared while the loads are in flight
        for (int i = threadIdx.x; i < H; i += NT) htab[i] = ~0ull;
        phase(C_PH_CLEAR);
        bool nan = false;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int p = k * NT + threadIdx.x;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            const bool ok = valid(lx, ly, lz);
            nan |= ok && (fv[k] != fv[k]);
            hk[p] = ok ? okey(fv[k]) ^ flip : 0xffffffffu;  // outside the field: above every vertex
        }
        if (__ballot(nan) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&h->status, ST_NAN);
    }
    __syncthreads();
    phase(C_PH_LOAD);

    // lowest lower neighbour inside the tile; a position outside the field
    // points at itself, so that the basin pass can follow every pointer
    // without a test
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int p = k * NT + threadIdx.x;
        const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
        if (!valid(lx, ly, lz)) {
            wl[p] = (int16_t)p;
            continue;
        }
        // the six neighbours' keys read at once (an absent neighbour reads the
        // vertex itself); the lowest (value key, position) wins, in 32-bit
        // compares: the lower positions are taken in descending order and win
        // ties, the higher ones in ascending order and lose them
        const bool cmx = lx > 0, cmy = ly > 0, cmz = lz > 0;
        const bool cpx = lx + 1 < c.ex, cpy = ly + 1 < c.ey, cpz = lz + 1 < c.ez;
        const uint32_t h0 = hk[p];
        const uint32_t hmx = hk[cmx ? p - 1 : p], hmy = hk[cmy ? p - TX : p], hmz = hk[cmz ? p - TX * TY : p];
        const uint32_t hpx = hk[cpx ? p + 1 : p], hpy = hk[cpy ? p + TX : p], hpz = hk[cpz ? p + TX * TY : p];
        uint32_t bh = h0;
        int bp = p;
        if (cmx && hmx <= bh) { bh = hmx; bp = p - 1; }
        if (cmy && hmy <= bh) { bh = hmy; bp = p - TX; }
        if (cmz && hmz <= bh) { bh = hmz; bp = p - TX * TY; }
        if (cpx && hpx < bh) { bh = hpx; bp = p + 1; }
        if (cpy && hpy < bh) { bh = hpy; bp = p + TX; }
        if (cpz && hpz < bh) { bh = hpz; bp = p + TX * TY; }
        wl[p] = (int16_t)bp;
    }
    __syncthreads();
    phase(C_PH_DESCENT);

    // Number the local minima in tile order (position k * NT + thread):
    // per-wave ballots, one scan of the VOL / 64 wave counts by wave 0.
    constexpr int NW = NT / 64;
    static_assert(VOL / 64 <= 64, "one wave scans the counts");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // First minimum number of the tile, reserved by one global atomic whose
    // result is only published (sb0) before the slot writes, so no wave waits
    // for it in between.
    uint32_t gbase = 0;
    {
        bool is_min[PER];
        uint64_t mb[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int p = k * NT + threadIdx.x;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            is_min[k] = valid(lx, ly, lz) && wl[p] == p;
            mb[k] = __ballot(is_min[k]);
            if (lane == 0) wsum[k * NW + wave] = (uint32_t)__popcll(mb[k]);
        }
        __syncthreads();
        if (wave == 0) {
            const uint32_t own = lane < VOL / 64 ? wsum[lane] : 0u;
            uint32_t inc = own;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(inc, o);
                if (lane >= o) inc += t;
            }
            if (lane < VOL / 64) wsum[lane] = inc - own;
            if (lane == 63) {
                scnt = inc;
                // (the address is written per lane, offset 0 here, so the
                // compiler keeps the atomic as issued instead of turning it
                // into a wave-wide one whose result it must wait for at once)
                gbase = atomicAdd(&h->n_minima + (threadIdx.x - 63u), inc);
                nwin = 0;
                novf = 0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (!is_min[k]) continue;
            const int p = k * NT + threadIdx.x;
            const uint32_t r = wsum[k * NW + wave] + (uint32_t)__popcll(mb[k] & lanemask_lt());
            zl[p] = (uint16_t)r;
            mh[r] = (uint16_t)p;
        }
    }
    __syncthreads();  // the basin pass reads the minima's numbers
    phase(C_PH_NUMBER);
    const uint32_t cnt = scnt;

    // local basins: follow the pointers to the local minimum (keys fall
    // strictly along them, so at most VOL steps); a lane follows the chains
    // of all its vertices together so that their loads overlap, and every
    // read is issued with no test around it: a finished chain sits on its
    // minimum, and a position outside the field on itself, both pointing at
    // themselves
    {
        int xs[PER];
        uint32_t moved = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int p = k * NT + threadIdx.x;
            xs[k] = wl[p];
            moved |= (uint32_t)(xs[k] != p) << k;
        }
        bool more = moved != 0;
        for (int step = 0; more && step < VOL; ++step) {
            int ys[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) ys[k] = wl[xs[k]];
            more = false;
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                more |= ys[k] != xs[k];
                xs[k] = ys[k];
            }
        }
        // minima's numbers first, then the writes (they go to vertices that are
        // no minima, so no read sees them)
        uint16_t zz[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) zz[k] = zl[xs[k]];
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if ((moved >> k) & 1u) zl[k * NT + threadIdx.x] = zz[k];
    }
    __syncthreads();
    phase(C_PH_BASIN);

    // Edges inside the tile whose ends lie in different local basins.  Of all
    // edges joining the same two basins only the lowest (smallest upper end)
    // is merged: the connection it makes at its level implies the connection
    // every other one would make at a higher level.  The pair table keeps that
    // lowest edge; an edge that finds no table room goes to a short overflow
    // list merged with the table's entries (should that list fill up too,
    // every edge of the tile is merged directly once the table's merges are
    // done), and every edge of a tile with more minima than a tag can number
    // is merged directly.
    uint32_t err = 0;
    const bool tabled = (uint32_t)HALF <= ZMAX || cnt <= ZMAX;
    // The value keys of the local minima, for the table merges' test of
    // which minimum lies deeper, where a tile with a table (at most ZMAX
    // minima) leaves the triplets' upper half unused (shapes whose triplets
    // have no such half read them through the minima's positions).
    constexpr bool MKV = (uint32_t)HALF > ZMAX;
    static_assert(!MKV || 2 * (HALF - ZMAX) >= ZMAX, "room for the minima's value keys");
    uint32_t *const mkv = reinterpret_cast<uint32_t *>(TL + (MKV ? ZMAX : 0));
    // the local minima's triplets, roots at their own level (and their value keys)
    auto init_tl = [&]() {
        for (uint32_t i = threadIdx.x; i < cnt; i += NT) {
            const uint32_t mp = mh[i];
            TL[i] = L::make(lkey<PB>(hk, mp), i);
            if (MKV && tabled) mkv[i] = hk[mp];
        }
    };
    // One atomic min per probe: an empty entry is claimed; an entry of the
    // same pair keeps the lower edge; an entry of another pair keeps the
    // lower of the two words and the lane carries the other one on.  Entries
    // move but are never dropped, so every pair's lowest edge ends in the
    // table (or on the overflow list); a pair left with a second, higher
    // entry only costs a merge that changes nothing.  `probes` (at most 32 by
    // default) bounds the probes before the overflow list; a smaller value
    // only sends more edges down that path.
    // (The probe loops have a compile-time length and are unrolled: measurably
    // faster than a loop to a runtime bound.  With the default bound, the
    // maximum, the kernel is instantiated without any bound check (LIMIT
    // false); a smaller bound selects the instantiation that checks it.)
    auto insert = [&](uint64_t val) {
        tc.add(C_TAB_INSERTS);
        uint32_t si = ((uint32_t)(val & TAGM) * 0x9E3779B1u) >> (32 - PB);
        for (int probe = 0; probe < kMaxProbes; ++probe) {
            if constexpr (LIMIT) {
                if ((uint32_t)probe >= probes) break;
            }
            tc.add(C_TAB_PROBES);
            const uint64_t prev = __hip_atomic_fetch_min(htab + si, val, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
            if (prev == ~0ull || ((prev ^ val) & TAGM) == 0) return;
            val = prev < val ? val : prev;
            si = (si + 1) & (H - 1);
        }
        tc.add(C_TAB_DIRECT);
        const uint32_t o = atomicAdd(&novf, 1u);
        if (o < kOvf) ovf[o] = val;
    };
    // The edge from p in direction dir (0: +x, 1: +y, 2: +z) to q: its upper
    // end is the saddle, q unless p's value key is the larger (q follows p in
    // tile order; 32-bit work, the tile key is assembled once).  Into the
    // table, or merged at once (`direct`, and in a tile with more minima than
    // a tag numbers).
    auto offer = [&](int p, int dir, bool direct) {
        const int q = p + (dir == 0 ? 1 : dir == 1 ? TX : TX * TY);
        const uint32_t za = zl[p], zb = zl[q];
        const uint32_t ha = hk[p], hb = hk[q];
        const bool qup = hb >= ha;
        const uint32_t hs = qup ? hb : ha, ps = qup ? (uint32_t)q : (uint32_t)p;
        if (tabled && !direct) {
            // (tile key << 2 ZB) | lo | hi << ZB, the tile key being (hs << PB) | ps
            insert(((uint64_t)hs << (PB + 2 * ZB)) | (ps << (2 * ZB)) | min(za, zb) | (max(za, zb) << ZB));
        } else {
            if (!tabled) tc.add(C_TAB_DIRECT);  // (the edges of an overflowing tile were counted on the way in)
            lds_merge<VOL, CNT>(TL, hk, mh, za, ((uint64_t)hs << PB) | ps, zb, cnt, cap, err, tc);
        }
    };
    // Slot (k, dir) of a lane holds such an edge: vertex k of the lane and its
    // +dir neighbour lie in the tile and in different local basins.
    auto marked = [&](int k, int dir) {
        const int p = k * NT + threadIdx.x;
        const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
        if (!valid(lx, ly, lz)) return false;
        if (dir == 0) return lx + 1 < c.ex && zl[p + 1] != zl[p];
        if (dir == 1) return ly + 1 < c.ey && zl[p + TX] != zl[p];
        return lz + 1 < c.ez && zl[p + TX * TY] != zl[p];
    };
    // Each wave lists its marked slots in LDS (in the space of the minima's
    // triplets, which are only written once the table is complete) and its
    // lanes take the list's entries in turn: a wave runs as many rounds as
    // its edges over 64, not as many as its busiest lane has (about 6 against
    // 10 on a log-normal field).  Slots past the list's room stay with their
    // lanes, one per round.
    constexpr uint32_t kListCap = HALF * (uint32_t)(sizeof(uint64_t) / sizeof(uint16_t)) / NW;
    static_assert(PB + 2 <= 16 && PER * 3 <= 32, "list codes and slot marks");
    uint16_t *const elist = reinterpret_cast<uint16_t *>(TL) + wave * kListCap;
    const uint32_t lcap = tabled ? kListCap : 0u;  // untabled tiles merge at once and need the triplets
    uint32_t pend = 0, nlist = 0;                  // slots left to their lanes; listed slots (uniform)
#pragma unroll
    for (int k = 0; k < PER; ++k) {
#pragma unroll
        for (int dir = 0; dir < 3; ++dir) {
            const bool m = marked(k, dir);
            const uint64_t bm = __ballot(m);
            if (m) {
                const uint32_t pos = nlist + (uint32_t)__popcll(bm & lanemask_lt());
                if (pos < lcap) elist[pos] = (uint16_t)((k * NT + threadIdx.x) | (dir << PB));
                else pend |= 1u << (3 * k + dir);
            }
            nlist += (uint32_t)__popcll(bm);
        }
    }
    if (!tabled) init_tl();
    __syncthreads();
    const uint32_t nl = min(nlist, lcap);
    for (uint32_t i = lane; i < nl; i += 64) {
        const uint32_t code = elist[i];
        offer((int)(code & (VOL - 1)), (int)(code >> PB), false);
    }
    while (pend) {
        const int b = __builtin_ctz(pend);
        pend &= pend - 1;
        const int k = b / 3;
        offer(k * NT + threadIdx.x, b - 3 * k, false);
    }
    __syncthreads();
    phase(C_PH_INSERT);
    // Occupied entries, compacted to the front of the table so that every
    // lane of a wave has a merge: each lane holds its entries while the
    // table is rewritten.  The triplets take the lists' place.
    {
        if (tabled) init_tl();
        constexpr int PER = (H + NT - 1) / NT;
        uint64_t e[PER];
        uint32_t pos[PER];
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int i = k * NT + threadIdx.x;
            e[k] = i < H ? htab[i] : ~0ull;
            const bool occ = e[k] != ~0ull;
            const uint64_t m = __ballot(occ);
            uint32_t base = 0;
            if (lane == 0 && m) base = atomicAdd(&nwin, (uint32_t)__popcll(m));
            base = __shfl(base, 0);
            pos[k] = base + (uint32_t)__popcll(m & lanemask_lt());
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; ++k)
            if (e[k] != ~0ull) htab[pos[k]] = e[k];
    }
    __syncthreads();
    phase(C_PH_COMPACT);
    // The table's merges (Alg. 3), the same steps as lds_merge written as one
    // step per loop round: each wave takes an equal share of the entries, and
    // a lane whose merge has ended takes the wave's next entry at once.  The
    // wave then loops about as often as its lanes' steps add up to over 64,
    // not as often as the longest merge of every batch of 64 (merges take 7
    // steps on average and up to about 30).
    // The overflow list's edges follow the table's entries.
    const uint32_t nov = novf;
    {
        const uint32_t nw = nwin, ne = nw + min(nov, kOvf);
        const uint32_t share = (ne + NW - 1) / NW;
        uint32_t next = min(ne, (uint32_t)wave * share);
        const uint32_t end = min(ne, next + share);
        bool act = false;
        uint32_t u = 0, v = 0, steps = 0;
        uint64_t tu = 0, tv = 0, ksT = 0;
        for (;;) {
            const uint64_t idle = __ballot(!act);
            if (!act) {
                const uint32_t i = next + __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                if (i < end) {
                    const uint64_t e = i < nw ? htab[i] : ovf[i - nw];
                    const uint32_t tag = (uint32_t)(e & TAGM);
                    u = tag & (ZMAX - 1);
                    v = tag >> ZB;
                    ksT = (e >> (2 * ZB)) << L::TB;
                    tc.add(C_LDS_MERGES);
                    if (u >= cnt || v >= cnt) {
                        err |= ST_CORRUPT;
                    } else {
                        tu = lds_ld64(TL + u);
                        tv = lds_ld64(TL + v);
                        steps = 0;
                        act = true;
                    }
                }
            }
            next += (uint32_t)__popcll(idle);
            if (__ballot(act) == 0ull) break;
            if (!act) continue;
            ++steps;
            const uint32_t u1 = L::tgt(tu), v1 = L::tgt(tv);
            const bool du = u1 != u && tu < ksT;
            const bool dv = v1 != v && tv < ksT;
            if (u1 >= cnt || v1 >= cnt) {
                err |= ST_CORRUPT;
                act = false;
            } else if (du || dv) {
                const uint32_t x = du ? u1 : v1;
                const uint64_t t = lds_ld64(TL + x);
                if (du) { u = x; tu = t; } else { v = x; tv = t; }
            } else if (u == v) {
                act = false;
            } else {
                // tile keys compared as (value key, position): positions only on a tie
                bool swap;
                if constexpr (MKV) {
                    const uint32_t ku = mkv[u], kv = mkv[v];
                    swap = kv < ku;
                    if (kv == ku) swap = mh[v] < mh[u];
                } else {
                    const uint32_t pu = mh[u], pv = mh[v];
                    const uint32_t ku = hk[pu], kv = hk[pv];
                    swap = kv < ku || (kv == ku && pv < pu);
                }
                if (swap) {
                    const uint32_t w = u; u = v; v = w;
                    const uint64_t tw = tu; tu = tv; tv = tw;
                }
                uint64_t seen = tv;
                tc.add(C_LDS_CAS);
                if (__hip_atomic_compare_exchange_strong(TL + v, &seen, ksT | u, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) {
                    if (L::tgt(tv) == v) {
                        act = false;
                    } else {
                        ksT = tv & ~L::TM;
                        v = L::tgt(tv);
                        tv = lds_ld64(TL + v);
                    }
                } else {
                    tc.add(C_LDS_CAS_FAIL);
                    tv = seen;
                }
                if (act) tu = lds_ld64(TL + u);
            }
            if (act && steps == cap) {
                err |= ST_LIVELOCK;
                act = false;
            }
            if (!act) {
                tc.add(C_LDS_STEPS, steps);
                tc.max(C_LDS_MAX_STEPS, steps);
            }
        }
    }
    if (nov > kOvf) {  // (uniform) the overflow list ran out of room: every edge is merged at once
        if (threadIdx.x == 0) tc.add(C_TAB_REDO);
#pragma unroll
        for (int k = 0; k < PER; ++k)
#pragma unroll
            for (int dir = 0; dir < 3; ++dir)
                if (marked(k, dir)) offer(k * NT + threadIdx.x, dir, true);
    }
    __syncthreads();
    phase(C_PH_MERGE);

    // Repair (Alg. 5) of the local minima: target -> deepest local minimum
    // reached through links whose saddle is at or below the minimum's own.
    for (uint32_t i = threadIdx.x; i < cnt; i += NT) {
        const uint64_t t = lds_ld64(TL + i);
        uint32_t x = L::tgt(t);
        if (x == i) continue;
        const uint64_t above = t | L::TM;  // a word lies above it exactly when its key is above t's
        for (uint32_t step = 0; step < cap; ++step) {
            const uint64_t tx = lds_ld64(TL + x);
            const uint32_t v = L::tgt(tx);
            if (v >= cnt) { err |= ST_CORRUPT; break; }
            if (v == x || tx > above) break;
            x = v;
        }
        if (x != L::tgt(t))
            __hip_atomic_store(TL + i, (t & ~L::TM) | x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    if (threadIdx.x == 63) sb0 = gbase;
    __syncthreads();
    phase(C_PH_REPAIR);
    const uint32_t b0 = sb0;
    if (b0 + cnt > mcap || b0 + cnt < b0) {  // cannot happen: capacity bounds the minima
        if (threadIdx.x == 0) atomicOr(&h->status, ST_CORRUPT);
        return;
    }

    for (uint32_t i = threadIdx.x; i < cnt; i += NT) {
        const uint64_t t = TL[i];
        const uint32_t sp = (uint32_t)L::key(t) & (VOL - 1), mp = mh[i];
        const uint32_t sg = gid((int)sp);
        slot[b0 + i].w = pack(sg, b0 + L::tgt(t));
        slot[b0 + i].k = ((uint64_t)(uint32_t)(L::key(t) >> PB) << 32) | sg;
        mkey[b0 + i] = ((uint64_t)hk[mp] << 32) | gid((int)mp);
    }
    // Every vertex is labelled with the representative of its local basin
    // at its own level (the deepest vertex it is connected to inside the tile
    // at that level).  Later merges and chases start there: the links below
    // the vertex's level are already followed.
    // (the PER chases of a lane advance together, so their loads overlap)
    {
        uint32_t xs[PER], act = 0;
        uint64_t lv[PER];  // a triplet word above this has its saddle above the vertex's level
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int p = k * NT + threadIdx.x;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            xs[k] = zl[p];
            lv[k] = (lkey<PB>(hk, p) << L::TB) | L::TM;
            if (!valid(lx, ly, lz)) { xs[k] = 0; continue; }
            if (xs[k] >= cnt) { err |= ST_CORRUPT; xs[k] = 0; continue; }
            act |= 1u << k;
        }
        const uint32_t live = act;
        for (uint32_t step = 0; act != 0; ++step) {
            if (step == cap) { err |= ST_LIVELOCK; break; }
            uint64_t t[PER];
#pragma unroll
            for (int k = 0; k < PER; ++k) t[k] = TL[xs[k]];  // in range: checked or 0
#pragma unroll
            for (int k = 0; k < PER; ++k) {
                if (!((act >> k) & 1u)) continue;
                const uint32_t v = L::tgt(t[k]);
                if (v >= cnt) { err |= ST_CORRUPT; act &= ~(1u << k); continue; }
                if (v == xs[k] || t[k] > lv[k]) act &= ~(1u << k);
                else xs[k] = v;
            }
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (!((live >> k) & 1u)) continue;
            const int p = k * NT + threadIdx.x;
            const int lx = p % TX, ly = (p / TX) % TY, lz = p / (TX * TY);
            lbl[gid(p)] = b0 + xs[k];
            // the first and last x columns also go to the tile's face record
            // (order key << 32 | label), read contiguously by the cross pass
            if (lx == 0 || lx == TX - 1)
                xface[((size_t)c.t * 2 + (lx != 0)) * kXFace + ly + TY * lz] =
                    ((uint64_t)hk[p] << 32) | (b0 + xs[k]);
        }
    }
    phase(C_PH_LABEL);
    if constexpr (MODE == 2) {
        if (threadIdx.x == 0)
            for (int i = C_PH_LOAD; i <= C_PH_LABEL; ++i) atomicAdd(&h->ctr[i], (unsigned long long)phc[i]);
    }
    if (err) atomicOr(&h->status, err);
    tc.flush(h);
}

// ---------------------------------------------------------------------------
// 2. Merge (Alg. 3) across tiles, on the minimum slots

// Path compression in long descents.  When a descent has followed x -> y (at
// saddle sx) and is about to follow y -> z at a saddle sy not above sx, x is
// re-pointed at z at its own saddle, (sx, y) -> (sx, z), by compare-and-swap:
// x and z are connected at the level of sx through y and z lies below y, so
// this is one step of Repair's chase (Alg. 4) written back early, and a swap
// that finds x changed does nothing.  Merged in ascending saddle order only
// approximately (the facts are binned by their top key bits), a monotone path
// through many tiles otherwise builds chains that every later merge walks to
// the end: quadratic in the path length.  Merges that stay short (the common
// case) never pay the extra swap.
constexpr uint32_t kCompressAfter = 8;

struct Link {  // the link a descent followed last: x -> hi32(w) at the saddle with key k
    uint32_t x = 0xffffffffu;
    uint64_t w = 0, k = 0;
};

template <bool CNT>
__device__ __forceinline__ void compress(Slot *__restrict__ S, const Link &l, uint32_t y, uint64_t ky, uint32_t z,
                                         uint32_t desc, Tally<CNT> &tc)
{
    if (desc <= kCompressAfter || l.x == 0xffffffffu || hi32(l.w) != y || ky > l.k) return;
    uint64_t e = l.w;
    if (__hip_atomic_compare_exchange_strong(&S[l.x].w, &e, pack(lo32(l.w), z), __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        tc.add(C_GM_COMPRESS);
}

template <bool CNT>
__device__ void gmerge(Slot *__restrict__ S, const uint64_t *__restrict__ mkey, const float *__restrict__ f,
                       uint32_t flip, uint32_t M, uint32_t n, uint32_t u, uint32_t s, uint64_t ks, uint32_t v,
                       uint32_t cap, uint32_t &err, Tally<CNT> &tc)
{
    tc.add(C_GM_FACTS);
    SlotRead tu = ld_slot_live(S, u);
    SlotRead tv = ld_slot_live(S, v);
    Link lu, lv;
    uint32_t step = 0, desc = 0;
    for (; step < cap; ++step) {
        const uint32_t u1 = hi32(tu.w), su = lo32(tu.w), v1 = hi32(tv.w), sv = lo32(tv.w);
        if (u1 >= M || v1 >= M || su >= n || sv >= n) { err |= ST_CORRUPT; break; }
        if (u1 != u) {
            const uint64_t ku = saddle_key(tu, f, flip);
            if (ku < ks) {
                tc.add(C_GM_DESCENTS);
                compress(S, lu, u, ku, u1, ++desc, tc);
                lu.x = u; lu.w = tu.w; lu.k = ku;
                u = u1; tu = ld_slot_live(S, u); continue;
            }
        }
        if (v1 != v) {
            const uint64_t kv = saddle_key(tv, f, flip);
            if (kv < ks) {
                tc.add(C_GM_DESCENTS);
                compress(S, lv, v, kv, v1, ++desc, tc);
                lv.x = v; lv.w = tv.w; lv.k = kv;
                v = v1; tv = ld_slot_live(S, v); continue;
            }
        }
        if (u == v) break;
        if (mkey[v] < mkey[u]) {  // the upper minimum is re-pointed
            const uint32_t w = u; u = v; v = w;
            const SlotRead tw = tu; tu = tv; tv = tw;
            const Link lw = lu; lu = lv; lv = lw;
        }
        uint64_t seen = tv.w;
        tc.add(C_GM_CAS);
        if (__hip_atomic_compare_exchange_strong(&S[v].w, &seen, pack(s, u), __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
            st_relaxed(&S[v].k, ks);
            if (hi32(tv.w) == v) break;  // v was a root
            tc.add(C_GM_REMERGE);
            const uint64_t kv = saddle_key(tv, f, flip);  // merge the displaced triplet again
            s = lo32(tv.w);
            ks = kv;
            v = hi32(tv.w);
            tv = ld_slot_live(S, v);
            lv.x = 0xffffffffu;
        } else {
            tc.add(C_GM_CAS_FAIL);
            tv.w = seen;
            tv.k = ld_relaxed(&S[v].k);
        }
        tu = ld_slot_live(S, u);
    }
    tc.add(C_GM_STEPS, step + (step < cap));
    tc.max(C_GM_MAX_STEPS, step + (step < cap));
    if (step == cap) err |= ST_LIVELOCK;
}

// Per-workgroup aggregation of bin-counter increments: lanes add into a
// small LDS table keyed by counter index (the returned rank is the lane's
// place among the workgroup's facts of that counter); flush adds each
// distinct counter's total to the global counters once.  A counter that finds
// no table room is counted in global memory directly (rank ~0u).
template <int LH>
struct CounterAgg {
    uint32_t key[LH], cnt[LH], base[LH];
    __device__ void clear(int tid, int nt)
    {
        for (int i = tid; i < LH; i += nt) { key[i] = 0xffffffffu; cnt[i] = 0u; }
    }
    // returns the rank of this increment within its counter, or ~0u if not tabled
    __device__ uint32_t add(uint32_t k, uint32_t &slot)
    {
        uint32_t si = (k * 0x9E3779B1u) >> (32 - __builtin_ctz(LH));
        for (int probe = 0; probe < 16; ++probe) {
            uint32_t prev = 0xffffffffu;
            __hip_atomic_compare_exchange_strong(key + si, &prev, k, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
            if (prev == 0xffffffffu || prev == k) {
                slot = si;
                return atomicAdd(cnt + si, 1u);
            }
            si = (si + 1) & (LH - 1);
        }
        return 0xffffffffu;
    }
};

constexpr int pow2_at_least(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Per tile: the edges leaving through its +x, +y, +z faces.  A local basin
// lies inside one tile, so all edges joining the same two local basins cross
// the same face and meet in this workgroup; only the lowest of them (smallest
// upper end) is kept, the others add nothing above its level.  The kept facts
// are appended to the queue of the XCD this workgroup runs on (one atomic per
// workgroup) and merged by k_merge_q, where every lane has a merge to do and
// each XCD works on the facts of its own tiles (so its L2 holds their slots).
// Workgroup size of the cross pass: at most 256 threads (a tile's faces hold
// at most 3 x 256 edges).  With its small tables that lets eight workgroups
// share a CU, which overlap each other's queue reservations.
template <class S>
constexpr int cross_threads() { return S::NT < 256 ? S::NT : 256; }

template <class S>
__global__ __launch_bounds__(cross_threads<S>()) void k_cross(const float *__restrict__ f, const uint32_t *__restrict__ lbl,
                                                 Fact *__restrict__ queue, uint32_t qsub,
                                                 const FieldDesc *__restrict__ D, const int32_t *__restrict__ tfield,
                                                 const int64_t *__restrict__ tstart, int nfc, int64_t tile0,
                                                 int64_t ntiles, int remap, uint32_t *__restrict__ qhist,
                                                 const uint64_t *__restrict__ xface, uint32_t flip,
                                                 uint32_t probes, Header *__restrict__ h)
{
    constexpr int TX = S::TX, TY = S::TY, TZ = S::TZ, NT = cross_threads<S>();
    // faces that can have a neighbour: a 2-D shape has no z face, a 1-D one no y face
    constexpr int FX = TY * TZ, FY = TY > 1 ? TX * TZ : 0, FZ = TZ > 1 ? TX * TY : 0;
    constexpr int E = FX + FY + FZ;
    // pair table: one entry per face edge at most (at least 2, so the hash keeps a bit)
    constexpr int H = pow2_at_least(E) < 2 ? 2 : pow2_at_least(E) < 2048 ? pow2_at_least(E) : 2048;
    __shared__ uint64_t hpair[H];  // (lower number | higher number << 32)
    __shared__ uint64_t hbest[H];  // lowest upper-end key of an edge joining that pair
    __shared__ uint32_t wsum[NT / 64];
    __shared__ uint32_t sbase;
    __shared__ CounterAgg<256> agg;
    const int64_t tl = xcd_tile(blockIdx.x, gridDim.x, remap);
    if (tl >= ntiles) return;
    const TileCtx c = tile_ctx<S>(D, tfield, tstart, nfc, tile0 + tl);
    const uint32_t off = (uint32_t)c.d.offset;
    const bool hx = c.x0 + TX < c.d.nx, hy = c.y0 + TY < c.d.ny, hz = c.z0 + TZ < c.d.nz;
    agg.clear(threadIdx.x, NT);
    const uint32_t M = h->n_minima;
    for (int i = threadIdx.x; i < H; i += NT) {
        hpair[i] = ~0ull;
        hbest[i] = ~0ull;
    }
    __syncthreads();
    uint32_t err = 0;
    // facts that find no table room are queued as they are (at most one per edge)
    constexpr int kOverflow = (E + NT - 1) / NT;
    Fact over[kOverflow];
    uint32_t ovf = 0;  // bit r: over[r] holds a fact
#pragma unroll
    for (int r = 0; r < kOverflow; ++r) {  // a static index keeps over[] in registers
        const int e = r * NT + (int)threadIdx.x;
        if (e >= E) continue;
        int lx, ly, lz;
        int64_t step;
        bool ok;
        if (e < FX) {
            ly = e % TY; lz = e / TY; lx = TX - 1; step = 1; ok = hx;
        } else if (e < FX + FY) {
            const int q = e - FX;
            lx = q % TX; lz = q / TX; ly = TY - 1; step = c.d.nx; ok = hy;
        } else {
            const int q = e - FX - FY;
            lx = q % TX; ly = q / TX; lz = TZ - 1; step = c.sxy; ok = hz;
        }
        if (!ok || lx >= c.ex || ly >= c.ey || lz >= c.ez) continue;
        const uint32_t a = off + (uint32_t)((c.x0 + lx) + (int64_t)c.d.nx * (c.y0 + ly) + c.sxy * (c.z0 + lz));
        const uint32_t b = a + (uint32_t)step;
        uint32_t za, zb;
        uint64_t ka, kb;
        if (e < FX) {  // x face: this tile's last column and the next tile's first, from the face records
            const uint64_t ra = xface[((size_t)c.t * 2 + 1) * kXFace + e];
            const uint64_t rb = xface[((size_t)(c.t + 1) * 2) * kXFace + e];
            za = lo32(ra); zb = lo32(rb);
            ka = (ra & 0xffffffff00000000ull) | a;
            kb = (rb & 0xffffffff00000000ull) | b;
        } else {
            za = lbl[a]; zb = lbl[b];
            ka = vkey(f, a, flip); kb = vkey(f, b, flip);
        }
        if (za >= M || zb >= M) { err |= ST_CORRUPT; continue; }
        const uint64_t ks = kb < ka ? ka : kb;  // the upper end is the saddle
        const uint64_t key = (uint64_t)min(za, zb) | ((uint64_t)max(za, zb) << 32);
        uint32_t si = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> (64 - __builtin_ctz(H)));
        bool placed = false;
        for (uint32_t probe = 0; probe < probes; ++probe) {
            uint64_t prev = ~0ull;
            __hip_atomic_compare_exchange_strong(hpair + si, &prev, key, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
            if (prev == ~0ull || prev == key) {
                atomicMin((unsigned long long *)(hbest + si), (unsigned long long)ks);
                placed = true;
                break;
            }
            si = (si + 1) & (H - 1);
        }
        if (!placed) {
            over[r] = Fact{za, zb, ks};
            ovf |= 1u << r;
        }
    }
    const int nover = __builtin_popcount(ovf);
    __syncthreads();

    // count this workgroup's facts, reserve queue room with one atomic
    uint32_t mine = nover;
    for (int i = threadIdx.x; i < H; i += NT) mine += hpair[i] != ~0ull;
    uint32_t incl = mine;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o);
        if ((threadIdx.x & 63) >= o) incl += v;
    }
    if ((threadIdx.x & 63) == 63) wsum[threadIdx.x >> 6] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < NT / 64; ++w) tot += wsum[w];
        sbase = tot ? atomicAdd(&h->n_cross[(blockIdx.x % 8) * kXStride], tot) : 0u;
    }
    __syncthreads();
    uint32_t pos = sbase + incl - mine;
    for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) pos += wsum[w];
    Fact *__restrict__ mq = queue + (size_t)(blockIdx.x % 8) * qsub;
    uint32_t *__restrict__ hist = qhist + (size_t)(blockIdx.x % 8) * kQCounters;
    auto put = [&](const Fact &q) {
        if (pos < qsub) {
            mq[pos] = q;
            const uint32_t k = qcounter(pos, q.ks);
            uint32_t slot;
            if (agg.add(k, slot) == 0xffffffffu) atomicAdd(hist + k, 1u);
        } else {
            err |= ST_CORRUPT;  // cannot happen: each queue holds every face edge of its tiles
        }
        ++pos;
    };
#pragma unroll
    for (int r = 0; r < kOverflow; ++r)
        if ((ovf >> r) & 1u) put(over[r]);
    for (int i = threadIdx.x; i < H; i += NT) {
        const uint64_t key = hpair[i];
        if (key != ~0ull) put(Fact{lo32(key), hi32(key), hbest[i]});
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += NT)
        if (agg.cnt[i]) atomicAdd(hist + agg.key[i], agg.cnt[i]);
    if (err) atomicOr(&h->status, err);
}

// Cross-tile facts in ascending order of their saddle key's top bits (a
// counting sort per XCD queue).  Any order of the merges gives the same tree;
// in this one most merges find the higher minimum still a root at their level,
// so few links are displaced and few swaps collide.
__global__ void k_zero32(uint32_t *__restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Exclusive scan of each XCD's counters in (bin, copy) order, in two
// launches over kQScanBlocks workgroups per XCD: block totals first, then
// each block scans its bins from the sum of the blocks before it.  Lane t of
// a block owns QB bins with all their copies.
constexpr int kQScanBlocks = 2;
constexpr int kQScanThreads = 256;
constexpr int kQBinsPerBlock = kQBins / kQScanBlocks;
static_assert(kQBinsPerBlock % kQScanThreads == 0, "whole bins per lane");

__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t *wsum)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t t = 0;
    for (int w = 0; w < kQScanThreads / 64; ++w) t += wsum[w];
    return t;
}

// grid (kQScanBlocks, 8): total of every block's counters
__global__ __launch_bounds__(kQScanThreads) void k_qtotals(const uint32_t *__restrict__ qhist,
                                                          uint32_t *__restrict__ qtot)
{
    constexpr int QB = kQBinsPerBlock / kQScanThreads;
    __shared__ uint32_t wsum[kQScanThreads / 64];
    const uint32_t *__restrict__ hist = qhist + (size_t)blockIdx.y * kQCounters + blockIdx.x * kQBinsPerBlock;
    uint32_t run = 0;
    for (int c = 0; c < kQCopies; ++c)
#pragma unroll
        for (int b = 0; b < QB; ++b) run += hist[(c << kQBinBits) + b * kQScanThreads + threadIdx.x];
    const uint32_t t = block_sum(run, wsum);
    if (threadIdx.x == 0) qtot[blockIdx.y * kQScanBlocks + blockIdx.x] = t;
}

// grid (kQScanBlocks, 8): counters -> exclusive prefix in (bin, copy) order
__global__ __launch_bounds__(kQScanThreads) void k_qscan(uint32_t *__restrict__ qhist,
                                                        const uint32_t *__restrict__ qtot)
{
    constexpr int QB = kQBinsPerBlock / kQScanThreads;
    __shared__ uint32_t wsum[kQScanThreads / 64];
    uint32_t *__restrict__ hist = qhist + (size_t)blockIdx.y * kQCounters + blockIdx.x * kQBinsPerBlock;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    uint32_t base = 0;
    for (int j = 0; j < (int)blockIdx.x; ++j) base += qtot[blockIdx.y * kQScanBlocks + j];
    // lane t owns bins t * QB .. t * QB + QB - 1 of the block
    uint32_t run = 0;
#pragma unroll
    for (int b = 0; b < QB; ++b)
        for (int c = 0; c < kQCopies; ++c) run += hist[(c << kQBinBits) + t * QB + b];
    uint32_t inc = run;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t e = base + inc - run;
    for (int w = 0; w < wave; ++w) e += wsum[w];
#pragma unroll
    for (int b = 0; b < QB; ++b)
        for (int c = 0; c < kQCopies; ++c) {
            uint32_t *const q = hist + (c << kQBinBits) + t * QB + b;
            const uint32_t v = *q;
            *q = e;
            e += v;
        }
}

// Each fact to its counter's next free place; workgroup b serves XCD b % 8
// and takes kBlock consecutive facts at a time, reserving one range per
// distinct counter.
__global__ __launch_bounds__(kBlock) void k_qscatter(const Fact *__restrict__ queue, Fact *__restrict__ qbin,
                                                     uint32_t qsub, uint32_t *__restrict__ qhist,
                                                     const Header *__restrict__ h)
{
    __shared__ CounterAgg<2 * kBlock> agg;
    const uint32_t x = blockIdx.x % 8, per = gridDim.x / 8;
    const uint32_t Q = min(h->n_cross[x * kXStride], qsub);
    const Fact *__restrict__ src = queue + (size_t)x * qsub;
    Fact *__restrict__ dst = qbin + (size_t)x * qsub;
    uint32_t *__restrict__ hist = qhist + (size_t)x * kQCounters;
    for (uint32_t i0 = (blockIdx.x / 8) * kBlock; i0 < Q; i0 += per * kBlock) {  // uniform per workgroup
        agg.clear(threadIdx.x, kBlock);
        __syncthreads();
        const uint32_t i = i0 + threadIdx.x;
        Fact q{};
        uint32_t k = 0, slot = 0, rank = 0;
        if (i < Q) {
            q = src[i];
            k = qcounter(i, q.ks);
            rank = agg.add(k, slot);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < 2 * kBlock; e += kBlock)
            if (agg.cnt[e]) agg.base[e] = atomicAdd(hist + agg.key[e], agg.cnt[e]);
        __syncthreads();
        if (i < Q) {
            const uint32_t at = rank != 0xffffffffu ? agg.base[slot] + rank : atomicAdd(hist + k, 1u);
            if (at < Q) dst[at] = q;  // always: the counters count exactly the queued facts
        }
        __syncthreads();
    }
}

// Merge of the queued cross-tile facts, one per lane; workgroup b serves the
// queue of XCD b % 8 (the grid is a multiple of 8 workgroups).
template <bool CNT>
__global__ __launch_bounds__(kBlock) void k_merge_q(const float *__restrict__ f, const Fact *__restrict__ queue,
                                                    uint32_t qsub, Slot *__restrict__ slot,
                                                    const uint64_t *__restrict__ mkey, uint32_t n, uint32_t cap,
                                                    uint32_t flip, Header *__restrict__ h)
{
    Tally<CNT> tc;
    const uint32_t M = h->n_minima;
    const uint32_t x = blockIdx.x % 8, per = gridDim.x / 8;
    const uint32_t Q = min(h->n_cross[x * kXStride], qsub);
    const Fact *__restrict__ mq = queue + (size_t)x * qsub;
    uint32_t err = 0;
    for (int64_t i = (int64_t)(blockIdx.x / 8) * kBlock + threadIdx.x; i < Q; i += (int64_t)per * kBlock) {
        const Fact q = mq[i];
        if (q.a >= M || q.b >= M || lo32(q.ks) >= n) { err |= ST_CORRUPT; continue; }
        gmerge<CNT>(slot, mkey, f, flip, M, n, q.a, lo32(q.ks), q.ks, q.b, cap, err, tc);
    }
    if (err) atomicOr(&h->status, err);
    tc.flush(h);
}

// ---------------------------------------------------------------------------
// 3. Repair (Alg. 4, 5)

// The id half of minimum m's key word (ids are the low 32 bits): one 4-byte load.
__device__ __forceinline__ uint32_t mkey_id(const uint64_t *__restrict__ mkey, uint32_t m)
{
    return reinterpret_cast<const uint32_t *>(mkey)[2 * (size_t)m];
}

// Representative: follow the slots from x while the saddle is at or below
// `level` and x is no root; the last minimum reached.
template <bool CNT>
__device__ __forceinline__ uint32_t chase(Slot *__restrict__ S, const float *__restrict__ f, uint32_t flip,
                                          uint32_t M, uint32_t n, uint32_t x, uint64_t level, uint32_t cap,
                                          uint32_t &err, Tally<CNT> &tc)
{
    for (uint32_t step = 0; step < cap; ++step) {
        tc.add(C_MIN_CHASES);
        const SlotRead t = ld_slot_live(S, x);
        const uint32_t v = hi32(t.w), s = lo32(t.w);
        if (v >= M || s >= n) { err |= ST_CORRUPT; return x; }
        if (v == x) return x;
        if (saddle_key(t, f, flip) > level) return x;
        x = v;
    }
    err |= ST_LIVELOCK;
    return x;
}

// Every minimum that is no root gets its repaired triplet, and its slot's
// key word is rewritten as (value key of the saddle << 32) | the minimum's
// own id, which is the form the output pass reads: the last slot of a chase
// then names the vertex the chase ends at.  Chases of other lanes that meet
// a rewritten word find its id half no longer equal to the saddle's id and
// read the saddle's value from the field instead (a root's word, (own key),
// is already in that form and stays).
template <bool CNT>
__global__ __launch_bounds__(kBlock) void k_repair_min(const float *__restrict__ f, Slot *__restrict__ S,
                                                       const uint64_t *__restrict__ mkey, uint32_t n,
                                                       uint32_t cap, uint32_t flip, Header *__restrict__ h)
{
    const uint32_t M = h->n_minima;
    uint32_t err = 0;
    Tally<CNT> tc;
    for (int64_t mm = (int64_t)blockIdx.x * kBlock + threadIdx.x; mm < M; mm += (int64_t)gridDim.x * kBlock) {
        const uint32_t m = (uint32_t)mm;
        const SlotRead t = ld_slot_live(S, m);
        const uint32_t v = hi32(t.w), s = lo32(t.w);
        if (v == m) continue;
        if (v >= M || s >= n) { err |= ST_CORRUPT; continue; }
        const uint64_t ks = saddle_key(t, f, flip);
        const uint32_t r = chase<CNT>(S, f, flip, M, n, v, ks, cap, err, tc);
        if (r != v) st_relaxed(&S[m].w, pack(s, r));
        st_relaxed(&S[m].k, (uint64_t)((ks & 0xffffffff00000000ull) | mkey_id(mkey, m)));
    }
    if (err) atomicOr(&h->status, err);
    tc.flush(h);
}

// Value of an order key's value part (inverse of okey, flip undone).  The
// key folds -0.0 onto +0.0, so a key of +0.0 does not say which zero the
// field holds: callers read the field for that one key.
__device__ __forceinline__ uint32_t key_bits(uint32_t k, uint32_t flip)
{
    k ^= flip;
    return (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
}
constexpr uint32_t kKeyZero = 0x80000000u;  // okey(+0.0) == okey(-0.0)

// Staged pair readout.  The output pass already knows every pair (a local
// minimum u whose repaired triplet has s != u) together with both values
// (f[u] from its level key, f[s] from the saddle key), so it writes them
// out, and the readout only has to move them to their place in ascending
// birth order instead of reading T again.  Chunk c's vertices fall into 64
// buckets of 64 consecutive ids, bucket (group g, vertex slot i, wave w) =
// g * 16 + i * 4 + w; each wave appends its pairs, in bucket order, to a
// list of its own of kStageCap entries {birth, death, f[birth], f[death]}
// (field-local ids), and records each bucket's count.  A wave with more
// pairs than that keeps only the count, and the readout then takes the
// chunk from T instead.
constexpr int kStageCap = 256;                               // entries per wave and chunk
constexpr int kBuckets = kChunk / 64;                        // 64 buckets of 64 vertices
constexpr int kStagePerChunk = (kBlock / 64) * kStageCap;    // entries per chunk

// Output triplets in vertex order, field-local ids.  A local minimum copies
// its own (repaired) triplet; any other vertex u gets (u, u, representative
// of its local minimum at the level of u).  Also counts pairs and roots per
// chunk, and stages the pairs when `stage` is not null.  Slots are read-only
// here, so plain loads, and repaired: a slot's key word holds (value key of
// the saddle, the minimum's own id), so the last slot a chase reads names the
// vertex the chase ends at.  Each lane carries RV vertices at once, so the
// dependent loads of their chases (label -> slot -> slot ...) overlap.
constexpr int RV = 4;
static_assert(kChunk == kBlock * RV * 4 && (kBlock / 64) * RV * 4 == kBuckets, "bucket layout");
template <bool CNT, class O>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_repair_reg(const float *__restrict__ f, const uint32_t *__restrict__ lbl,
                                                       const Slot *__restrict__ S,
                                                       typename O::Word *__restrict__ T, uint32_t *__restrict__ pcnt,
                                                       uint4 *__restrict__ stage, uint8_t *__restrict__ bcnt,
                                                       const FieldDesc *__restrict__ D, const int64_t *__restrict__ cs,
                                                       int nf, uint32_t n, uint32_t cap, uint32_t flip,
                                                       Header *__restrict__ h)
{
    __shared__ uint32_t sp[kBlock / 64];
    const int64_t c = blockIdx.x;
    // (the wave index is uniform: kept in a scalar register, like everything per wave below)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    uint32_t wcnt = 0;  // pairs of the wave's vertices in this chunk (staged ones: the first kStageCap)
    const FieldDesc d = D[search(cs, nf, c)];
    const int64_t lo = (c - d.chunk_start) * kChunk;
    const int64_t hi = min(lo + (int64_t)kChunk, d.n);
    const uint32_t off = (uint32_t)d.offset;
    const uint32_t M = h->n_minima;
    uint32_t err = 0;
    Tally<CNT> tc;
    static_assert(kChunk % (kBlock * RV) == 0, "whole groups per chunk");
    for (int64_t g0 = lo; g0 < hi; g0 += kBlock * RV) {
        const int gi = (int)((g0 - lo) / (kBlock * RV));
        uint32_t u[RV], z[RV], x[RV], s[RV];
        uint64_t level[RV], tw[RV], tk[RV];
        // id of the vertex the target names: the low half of the key word of
        // the last slot read (the repaired slots hold (saddle value, own id))
        uint32_t tid[RV];
        // bit i: vertex i is written / chasing / stops after one slot read /
        // gets target tid[i] (else itself: a root)
        uint32_t live = 0, act = 0, once = 0, need = 0;
#pragma unroll
        for (int i = 0; i < RV; ++i) {
            const int64_t j = g0 + i * kBlock + threadIdx.x;
            const bool in = j < hi;
            live |= (uint32_t)in << i;
            u[i] = off + (uint32_t)(in ? j : lo);
            z[i] = lbl[u[i]];
            level[i] = vkey(f, u[i], flip);
        }
#pragma unroll
        for (int i = 0; i < RV; ++i) {
            if (z[i] >= M) {
                if ((live >> i) & 1u) err |= ST_CORRUPT;
                z[i] = 0;
                live &= ~(1u << i);
            }
            tw[i] = S[z[i]].w;
            tk[i] = S[z[i]].k;
        }
#pragma unroll
        for (int i = 0; i < RV; ++i) {
            x[i] = z[i];
            s[i] = u[i];
            tid[i] = lo32(tk[i]);  // the local minimum z's own id
            const uint32_t s0 = lo32(tw[i]), v0 = hi32(tw[i]);
            bool pf = false;  // u is a pair birth (a live local minimum with s != u)
            uint32_t dk = 0;  // then: the value key of its saddle
            if (v0 >= M || s0 >= n) {
                if ((live >> i) & 1u) err |= ST_CORRUPT;
                live &= ~(1u << i);
            } else {
                const uint64_t sk = ((uint64_t)hi32(tk[i]) << 32) | s0;
                if (tid[i] == u[i]) {  // u is a local minimum: its own repaired triplet
                    s[i] = s0;
                    if ((live >> i) & 1u) {
                        // a root: one per connected component, so counted by a rare atomic
                        if (v0 == z[i]) atomicAdd((unsigned long long *)&h->roots, 1ull);
                        pf = s0 != u[i];
                        dk = hi32(sk);
                    }
                    if (v0 != z[i]) {  // its target's id: one slot read
                        x[i] = v0;
                        act |= 1u << i;
                        once |= 1u << i;
                        need |= 1u << i;
                    }
                } else if (v0 == z[i] || sk > level[i]) {
                    need |= 1u << i;  // target z itself
                } else {                    // (u, u, representative of z at the level of u)
                    x[i] = v0;
                    act |= 1u << i;
                    need |= 1u << i;
                }
            }
            const uint64_t m = __ballot(pf);
            if (stage) {  // (uniform) the pair onto the wave's list, in bucket (gi, i, wave)
                // rank among the wave's pairs: the pairs of lower lanes, counted by mbcnt
                const uint32_t r = wcnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (pf && r < (uint32_t)kStageCap) {
                    const uint32_t bk = hi32(level[i]);
                    const uint32_t bb = bk == (kKeyZero ^ flip) ? __float_as_uint(f[u[i]]) : key_bits(bk, flip);
                    const uint32_t db = dk == (kKeyZero ^ flip) ? __float_as_uint(f[s0]) : key_bits(dk, flip);
                    stage[((size_t)c * (kBlock / 64) + wave) * kStageCap + r] =
                        make_uint4(u[i] - off, s0 - off, bb, db);
                }
                if (lane == 0) bcnt[(size_t)c * kBuckets + gi * 16 + i * 4 + wave] = (uint8_t)__popcll(m);
            }
            wcnt += (uint32_t)__popcll(m);
        }
        for (uint32_t step = 0; act != 0; ++step) {
            if (step == cap) { err |= ST_LIVELOCK; break; }
            tc.add(C_REG_CHASES, (uint32_t)__builtin_popcount(act));
            if constexpr (CNT) tc.add(C_REG_ROUNDS, (__ballot(1) & lanemask_lt()) == 0ull);  // first active lane
            // all RV loads issued together, no branch around them: a vertex
            // whose chase has ended reads slot 0 (one shared line per wave)
#pragma unroll
            for (int i = 0; i < RV; ++i) {
                const uint32_t xi = ((act >> i) & 1u) ? x[i] : 0u;
                tw[i] = S[xi].w;
                tk[i] = S[xi].k;
            }
#pragma unroll
            for (int i = 0; i < RV; ++i) {
                if (!((act >> i) & 1u)) continue;
                const uint32_t v = hi32(tw[i]), sv = lo32(tw[i]);
                if (v >= M || sv >= n) {
                    err |= ST_CORRUPT;
                    act &= ~(1u << i);
                    need &= ~(1u << i);
                    live &= ~(1u << i);
                    continue;
                }
                tid[i] = lo32(tk[i]);
                const uint64_t sk = ((uint64_t)hi32(tk[i]) << 32) | sv;
                if (((once >> i) & 1u) || v == x[i] || sk > level[i]) act &= ~(1u << i);
                else x[i] = v;
            }
        }
#pragma unroll
        for (int i = 0; i < RV; ++i) {
            if (!((live >> i) & 1u)) continue;
            const uint32_t t = ((need >> i) & 1u) ? tid[i] : u[i];  // the target's id
            if (t >= n) { err |= ST_CORRUPT; continue; }
            O::store(T, u[i], s[i] - off, t - off);
        }
    }
    if (lane == 0) sp[wave] = wcnt;
    // buckets of groups past the end of the field hold no pair
    if (stage)
        for (int g = (int)((hi - lo + kBlock * RV - 1) / (kBlock * RV)); g < kChunk / (kBlock * RV); ++g)
            if (lane < RV) bcnt[(size_t)c * kBuckets + g * 16 + lane * 4 + wave] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (int w = 0; w < kBlock / 64; ++w) a += sp[w];
        pcnt[c] = a;
    }
    if (err) atomicOr(&h->status, err);
    tc.flush(h);
}

// ---------------------------------------------------------------------------
// 5. Pairs: one per branch (Sec. 1), i.e. every u with T[u] = (s, v), s != u.

// Ids read from T are checked to lie in the field; a bad one is no pair and
// latches ST_CORRUPT.
template <class O>
__device__ __forceinline__ bool classify(const typename O::Word *__restrict__ T, uint32_t off, uint32_t nloc,
                                         int64_t j, uint32_t &s_out, bool &root, uint32_t &err)
{
    uint32_t s, v;
    O::load(T, off + (uint32_t)j, s, v);
    root = false;
    if (s >= nloc || v >= nloc) { err |= ST_CORRUPT; return false; }
    if (s == (uint32_t)j) { root = (v == (uint32_t)j); return false; }
    s_out = s;
    return true;
}

template <class O>
__global__ __launch_bounds__(kBlock) void k_pairs_count(const typename O::Word *__restrict__ T,
                                                        const FieldDesc *__restrict__ D, const int64_t *__restrict__ cs,
                                                        int nf, uint32_t *__restrict__ cnt, Header *__restrict__ h)
{
    __shared__ uint32_t sp[kBlock / 64], sr[kBlock / 64];
    const int64_t c = blockIdx.x;
    const FieldDesc d = D[search(cs, nf, c)];
    const int64_t lo = (c - d.chunk_start) * kChunk;
    const int64_t hi = min(lo + (int64_t)kChunk, d.n);
    uint32_t np = 0, nr = 0, err = 0;
    for (int64_t j = lo + threadIdx.x; j < hi; j += kBlock) {
        uint32_t s;
        bool root;
        np += classify<O>(T, (uint32_t)d.offset, (uint32_t)d.n, j, s, root, err) ? 1u : 0u;
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

// Exclusive scan of the chunk counts (one workgroup of 1024), the total, and
// the per-field pair offsets.  Thread t owns a contiguous run of `per` counts
// (a multiple of 4, so its 16-byte words are aligned), read with all words in
// flight; the run sums are scanned with wave shuffles and one LDS round.
__global__ __launch_bounds__(1024) void k_pairs_scan(uint32_t *__restrict__ cnt, int64_t n_chunks,
                                                     const FieldDesc *__restrict__ D, int nf,
                                                     int64_t *__restrict__ pair_offsets, int64_t capacity,
                                                     Header *__restrict__ h)
{
    constexpr int NT = 1024, V = 8;  // 16-byte words per thread and round
    __shared__ uint64_t wtot[NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t per = (((n_chunks + NT - 1) / NT) + 3) & ~(int64_t)3;
    const int64_t a = min((int64_t)tid * per, n_chunks), b = min(a + per, n_chunks);
    auto word = [&](int64_t i) -> uint4 {  // counts i .. i+3, zero past b
        if (i + 4 <= b) return *(const uint4 *)(cnt + i);
        uint4 q = make_uint4(0, 0, 0, 0);
        if (i < b) q.x = cnt[i];
        if (i + 1 < b) q.y = cnt[i + 1];
        if (i + 2 < b) q.z = cnt[i + 2];
        return q;
    };
    uint64_t s = 0;
    for (int64_t i0 = a; i0 < b; i0 += 4 * V) {
        uint4 q[V];
#pragma unroll
        for (int v = 0; v < V; ++v) q[v] = word(i0 + 4 * v);
#pragma unroll
        for (int v = 0; v < V; ++v) s += (uint64_t)q[v].x + q[v].y + q[v].z + q[v].w;
    }
    uint64_t inc = s;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    uint64_t run = inc - s, total = 0;
    for (int w = 0; w < NT / 64; ++w) {
        const uint64_t t = wtot[w];
        run += w < wave ? t : 0;
        total += t;
    }
    for (int64_t i0 = a; i0 < b; i0 += 4 * V) {
        uint4 q[V];
#pragma unroll
        for (int v = 0; v < V; ++v) q[v] = word(i0 + 4 * v);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int64_t i = i0 + 4 * v;
            uint4 o;
            o.x = (uint32_t)run; run += q[v].x;
            o.y = (uint32_t)run; run += q[v].y;
            o.z = (uint32_t)run; run += q[v].z;
            o.w = (uint32_t)run; run += q[v].w;
            if (i + 4 <= b) {
                *(uint4 *)(cnt + i) = o;
            } else {
                if (i < b) cnt[i] = o.x;
                if (i + 1 < b) cnt[i + 1] = o.y;
                if (i + 2 < b) cnt[i + 2] = o.z;
            }
        }
    }
    __syncthreads();
    if (pair_offsets) {
        for (int i = tid; i < nf; i += NT) pair_offsets[i] = cnt[D[i].chunk_start];
        if (tid == 0) pair_offsets[nf] = (int64_t)total;
    }
    if (tid == 0) {
        h->total_pairs = (int64_t)total;
        if ((int64_t)total > capacity) atomicOr(&h->status, ST_CAPACITY);
    }
}

// Ordered compaction: ascending vertex id within the chunk, chunks in order.
// Wave w owns the w-th quarter of the chunk.  It reads its triplets (all
// loads in flight, coalesced), keeps one ballot word of pair births per 64
// vertices (word r in lane r) and parks the death ids in LDS; one barrier
// shares the wave totals.  Then lane k of a pass takes the wave's k-th pair
// (its word by the word counts' prefix, its bit by halving), so the value
// gathers and the stores run on dense lanes, 64 consecutive pairs a pass.
//
// When the output pass staged the chunk's pairs (stage not null, no wave of
// the chunk past kStageCap), the pairs are instead copied from the wave lists:
// entry e of wave w's list lies in bucket (g, i, w) where the list's bucket
// prefix puts it, and its place in the chunk is the number of the chunk's
// pairs in earlier buckets plus its rank inside its bucket.
template <class O>
__global__ __launch_bounds__(kBlock) void k_pairs_write(const float *__restrict__ f,
                                                        const typename O::Word *__restrict__ T,
                                                        const FieldDesc *__restrict__ D, const int64_t *__restrict__ cs,
                                                        int nf, const uint32_t *__restrict__ base, int64_t capacity,
                                                        typename O::Id *__restrict__ birth,
                                                        typename O::Id *__restrict__ death,
                                                        float *__restrict__ bval, float *__restrict__ dval,
                                                        const uint4 *__restrict__ stage,
                                                        const uint8_t *__restrict__ bcnt)
{
    constexpr int WSPAN = kChunk / (kBlock / 64);  // vertices per wave
    constexpr int NWD = WSPAN / 64;                // ballot words per wave
    static_assert(NWD <= 64 && (NWD & (NWD - 1)) == 0, "one word per lane");
    __shared__ uint32_t sdeath[kChunk];
    __shared__ uint32_t wsum[kBlock / 64];
    __shared__ uint32_t bpre[kBuckets];  // pairs of the chunk in earlier buckets
    __shared__ uint32_t sover;
    const int64_t c = blockIdx.x;
    const FieldDesc d = D[search(cs, nf, c)];
    const int64_t lo = (c - d.chunk_start) * kChunk;
    const int64_t hi = min(lo + (int64_t)kChunk, d.n);
    const uint32_t off = (uint32_t)d.offset, nloc = (uint32_t)d.n;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (stage) {
        constexpr int NB = RV * 4;  // buckets of one wave: (g, i) = lane / RV, lane % RV
        if (wave == 0) {
            const uint32_t own = bcnt[(size_t)c * kBuckets + lane];
            uint32_t inc = own;
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t t = __shfl_up(inc, o);
                if (lane >= o) inc += t;
            }
            bpre[lane] = inc - own;
            if (lane == 0) sover = 0;
        }
        __syncthreads();
        // wave w's buckets, in its list order: lane k < NB holds bucket (k / RV) * 16 + (k % RV) * 4 + w
        const int kb = (lane / RV) * 16 + (lane % RV) * 4 + wave;
        const uint32_t own = lane < NB ? bcnt[(size_t)c * kBuckets + kb] : 0u;
        uint32_t inc = own;
#pragma unroll
        for (int o = 1; o < NB; o <<= 1) {
            const uint32_t t = __shfl_up(inc, o);
            if (lane >= o) inc += t;
        }
        const uint32_t total = __shfl(inc, NB - 1);
        if (lane == 0 && total > (uint32_t)kStageCap) atomicOr(&sover, 1u);
        __syncthreads();
        if (!sover) {
            const uint4 *__restrict__ list = stage + ((size_t)c * (kBlock / 64) + wave) * kStageCap;
            const int64_t b0 = base[c];
            for (uint32_t e = lane; e < ((total + 63u) & ~63u); e += 64) {
                // the list bucket k holding entry e: the first whose inclusive prefix exceeds e
                uint32_t k = 0;
#pragma unroll
                for (int st = NB / 2; st >= 1; st >>= 1) {
                    const uint32_t pre = __shfl(inc, (int)(k + st - 1));
                    if (pre <= e) k += st;
                }
                const uint32_t before = __shfl(inc, (int)k) - __shfl(own, (int)k);
                const uint32_t b = (k / RV) * 16 + (k % RV) * 4 + wave;
                if (e >= total) continue;
                const uint4 q = list[e];
                const int64_t pos = b0 + bpre[b] + (e - before);
                if (pos < capacity) {
                    birth[pos] = q.x;
                    death[pos] = q.y;
                    bval[pos] = __uint_as_float(q.z);
                    dval[pos] = __uint_as_float(q.w);
                }
            }
            return;
        }
    }
    const int64_t w0 = lo + (int64_t)wave * WSPAN;
    uint32_t sl[NWD], err = 0;
    bool pf[NWD];
#pragma unroll
    for (int r = 0; r < NWD; ++r) {
        const int64_t j = w0 + r * 64 + lane;
        pf[r] = false;
        sl[r] = 0;
        if (j < hi) {
            bool root;
            pf[r] = classify<O>(T, off, nloc, j, sl[r], root, err);
        }
    }
    uint64_t wd = 0;  // lane r < NWD: the ballot word of vertices w0 + 64 r + [0, 64)
#pragma unroll
    for (int r = 0; r < NWD; ++r) {
        const uint64_t m = __ballot(pf[r]);
        if (lane == r) wd = m;
        if (pf[r]) sdeath[wave * WSPAN + r * 64 + lane] = sl[r];
    }
    const uint32_t cnt = (uint32_t)__popcll(wd);
    uint32_t inc = cnt;  // inclusive prefix of the word counts over lanes < NWD
#pragma unroll
    for (int o = 1; o < NWD; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    const uint32_t total = __shfl(inc, NWD - 1);
    if (lane == 0) wsum[wave] = total;
    __syncthreads();
    int64_t run = base[c];
    for (int w = 0; w < wave; ++w) run += wsum[w];
    for (uint32_t k0 = 0; k0 < total; k0 += 64) {
        const uint32_t k = k0 + lane;
        // the word holding pair k: the first word whose inclusive prefix exceeds k
        uint32_t w = 0;
#pragma unroll
        for (int st = NWD / 2; st >= 1; st >>= 1) {
            const uint32_t pre = __shfl(inc, (int)(w + st - 1));
            if (pre <= k) w += st;
        }
        const uint32_t before = __shfl(inc, (int)w) - __shfl(cnt, (int)w);
        const uint64_t m = __shfl(wd, (int)w);
        if (k >= total) continue;
        const uint32_t q = w * 64 + select_bit(m, k - before);  // position in the wave's quarter
        const uint32_t j = (uint32_t)w0 + q;
        const uint32_t sv = sdeath[wave * WSPAN + q];
        const int64_t pos = run + k;
        if (pos < capacity) {
            birth[pos] = j;
            death[pos] = sv;
            bval[pos] = f[off + j];
            dval[pos] = f[off + sv];
        }
    }
}

// ---------------------------------------------------------------------------
// Vertex ranks: the (value, id) order of Sec. 2 as integer keys, the first
// step of a rank-keyed build (order keys, one radix sort, positions back).

__global__ __launch_bounds__(kBlock) void k_rank_keys(const float *__restrict__ f, uint32_t n, uint32_t flip,
                                                      uint64_t *__restrict__ keys, Header *__restrict__ h)
{
    bool nan = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const uint32_t u = (uint32_t)i;
        const float x = f[u];
        nan |= x != x;
        keys[u] = vkey(f, u, flip);
    }
    if (__ballot(nan) != 0ull && (threadIdx.x & 63) == 0) atomicOr(&h->status, ST_NAN);
}

__global__ __launch_bounds__(kBlock) void k_rank_scatter(const uint64_t *__restrict__ sorted, uint32_t n,
                                                         uint32_t *__restrict__ rank)
{
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
        const uint32_t u = lo32(sorted[i]);
        if (u < n) rank[u] = (uint32_t)i;
    }
}

// ---------------------------------------------------------------------------
// 6. Adjoint of the pair readout

// Zero fill of the gradient: 16-byte stores where the buffer is 16-byte
// aligned, single floats for the head before that and the tail after it.
__global__ __launch_bounds__(kBlock) void k_fill0(float *__restrict__ g, int64_t n)
{
    const int64_t head = min(n, (int64_t)((16 - ((uintptr_t)g & 15)) & 15) / 4);
    const int64_t nv = (n - head) / 4;  // whole 16-byte words after the head
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x, stride = (int64_t)gridDim.x * kBlock;
    if (t < head) g[t] = 0.0f;
    float4 *__restrict__ v = (float4 *)(g + head);
    for (int64_t i = t; i < nv; i += stride) v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int64_t r = t + head + 4 * nv;
    if (r < n) g[r] = 0.0f;  // (the tail is shorter than 4, and t < 4 covers it)
}

struct BwdGroup {
    int64_t voff[kBwdGroup];  // vertex offset of each field of the group
    int64_t nv[kBwdGroup];    // vertices of each field of the group
    int32_t first, count;
};

// grad[birth] += gb (birth vertices are distinct and are never death
// vertices, so a plain update is race free); grad[death] += gd atomically.
// The group's pair offsets are read once per workgroup into LDS, so finding
// the field of a pair is a search in LDS.
__global__ __launch_bounds__(kBlock) void k_scatter(BwdGroup g, const int64_t *__restrict__ po, int64_t capacity,
                                                    const uint32_t *__restrict__ birth,
                                                    const uint32_t *__restrict__ death,
                                                    const float *__restrict__ gb, const float *__restrict__ gd,
                                                    float *__restrict__ grad)
{
    __shared__ int64_t spo[kBwdGroup + 1];
    for (int i = threadIdx.x; i <= g.count; i += kBlock) spo[i] = po[g.first + i];
    __syncthreads();
    const int64_t k0 = spo[0];
    const int64_t k1 = min(spo[g.count], capacity);
    for (int64_t k = k0 + (int64_t)blockIdx.x * kBlock + threadIdx.x; k < k1; k += (int64_t)gridDim.x * kBlock) {
        int lo = 0, hi = g.count;  // spo[lo] <= k < spo[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (spo[mid] <= k) lo = mid; else hi = mid;
        }
        // a zero upstream gradient adds nothing: its scattered read-modify-write is skipped (a loss
        // that selects pairs, like a persistence threshold, leaves most of them at zero)
        const float b_g = gb[k], d_g = gd[k];
        if (b_g == 0.0f && d_g == 0.0f) continue;
        const int64_t vo = g.voff[lo];
        const uint32_t bk = birth[k], dk = death[k];
        if ((int64_t)bk >= g.nv[lo] || (int64_t)dk >= g.nv[lo]) continue;  // not an id of this field
        if (b_g != 0.0f) grad[vo + bk] += b_g;
        if (d_g != 0.0f) unsafeAtomicAdd(grad + vo + dk, d_g);
    }
}

}  // namespace mtd
