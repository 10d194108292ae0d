// mt.hip -- host side and C ABI of the triplet merge tree library (gfx950).
//
// The kernels live in mt_device.h (see its header comment for the pipeline
// and for why it computes the unique triplet merge tree of Sec. 2 of "Fast
// Merge Tree Computation via SYCL", arXiv 2301.10838).  This file turns the
// C-ABI calls of include/mt.h into launches: it validates arguments, lays out
// the caller's workspace, picks the tile shape of each class of fields
// (3-D, 2-D, 1-D), enqueues the kernels on the caller's stream, captures the
// batched form into a cached hipGraph, and offers per-kernel event timing.

#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_map>
#include <type_traits>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "mt.h"
#include "mt_device.h"

using namespace mtd;

namespace {

// Tile shapes compiled in (x, y, z, workgroup threads).  Class 0: 3-D fields
// (nz > 1), 1: 2-D (nz == 1, ny > 1), 2: 1-D.  Each class uses one shape per
// launch.
struct ShapeInfo {
    int tx, ty, tz, nt, cls;
};
constexpr ShapeInfo kShapes[] = {
    {16, 8, 8, 256, 0},   {32, 8, 4, 256, 0},   {8, 8, 8, 256, 0},     {16, 16, 4, 256, 0},
    {16, 16, 16, 1024, 0}, {32, 16, 8, 1024, 0}, {64, 16, 1, 256, 1},  {32, 32, 1, 256, 1},
    {64, 64, 1, 1024, 1}, {128, 32, 1, 1024, 1}, {1024, 1, 1, 256, 2}, {4096, 1, 1, 1024, 2},
    {16, 16, 8, 512, 0},  {64, 32, 1, 512, 1},   {2048, 1, 1, 512, 2},
};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);

template <class F>
static void with_shape(int id, F &&fn)
{
    switch (id) {
    case 0: fn(Shape<16, 8, 8, 256>{}); break;
    case 1: fn(Shape<32, 8, 4, 256>{}); break;
    case 2: fn(Shape<8, 8, 8, 256>{}); break;
    case 3: fn(Shape<16, 16, 4, 256>{}); break;
    case 4: fn(Shape<16, 16, 16, 1024>{}); break;
    case 5: fn(Shape<32, 16, 8, 1024>{}); break;
    case 6: fn(Shape<64, 16, 1, 256>{}); break;
    case 7: fn(Shape<32, 32, 1, 256>{}); break;
    case 8: fn(Shape<64, 64, 1, 1024>{}); break;
    case 9: fn(Shape<128, 32, 1, 1024>{}); break;
    case 10: fn(Shape<1024, 1, 1, 256>{}); break;
    case 11: fn(Shape<4096, 1, 1, 1024>{}); break;
    case 12: fn(Shape<16, 16, 8, 512>{}); break;
    case 13: fn(Shape<64, 32, 1, 512>{}); break;
    default: fn(Shape<2048, 1, 1, 512>{}); break;
    }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t D, tfield, tstart, cs, pcnt, lbl, slot, mkey, queue, qbin, qhist, qtot, xface, stage, bcnt, total;
};

struct ClassLaunch {
    int shape = 0;
    int cb = 0;   // first entry of the class in tile order
    int nfc = 0;  // fields in the class
    int64_t tile0 = 0, ntiles = 0;
};

struct Plan {
    std::vector<FieldDesc> d;  // field order
    int64_t n_total = 0, n_tiles = 0, n_chunks = 0, m_cap = 0, q_cap = 0;
    ClassLaunch cls[3];
    Layout lay{};
    // configuration in force when the plan was made
    int remap = 1;
    int mgroups = 2048;  // workgroups per XCD of the fact scatter and the cross-tile merge
    uint32_t cap = 0, probes = 0;
    int count = 0;
};

// Configuration (tile shape per class, XCD remap, step cap, pair-table probes).
static std::mutex g_cfg_mu;
static int g_shape[3] = {4, 6, 10};  // 16x16x16, 64x16, 1024
static int g_remap = 1;
constexpr int kDefaultMergeGroups = 2048;
static int g_mgroups = kDefaultMergeGroups;
constexpr uint32_t kDefaultCap = 1u << 24;
constexpr uint32_t kDefaultProbes = kMaxProbes;
static uint32_t g_cap = kDefaultCap;
static uint32_t g_probes = kDefaultProbes;
static int g_count = 0;  // counting build (event counters) instead of the timed one
static bool g_env_read = false;

static int find_shape(int cls, int tx, int ty, int tz)
{
    for (int i = 0; i < kNumShapes; ++i)
        if (kShapes[i].cls == cls && kShapes[i].tx == tx && kShapes[i].ty == ty && kShapes[i].tz == tz) return i;
    return -1;
}

static void read_env_locked()
{
    if (g_env_read) return;
    g_env_read = true;
    const char *names[3] = {"MT_TILE3D", "MT_TILE2D", "MT_TILE1D"};
    for (int c = 0; c < 3; ++c) {
        const char *s = getenv(names[c]);
        if (!s) continue;
        int a = 1, b = 1, z = 1;
        if (sscanf(s, "%dx%dx%d", &a, &b, &z) < 1) continue;
        const int id = find_shape(c, a, b, z);
        if (id >= 0) g_shape[c] = id;
    }
    if (const char *s = getenv("MT_XCD_REMAP")) g_remap = atoi(s) != 0;
    if (const char *s = getenv("MT_MAX_STEPS")) {
        const long v = atol(s);
        if (v >= 1 && v <= 0x7fffffffL) g_cap = (uint32_t)v;
    }
}

static int field_class(int64_t ny, int64_t nz) { return nz > 1 ? 0 : (ny > 1 ? 1 : 2); }

// Ids are uint32 inside every kernel: a field, or a whole batch, holds at most
// 2^32 - 2 vertices, so 0xffffffff and 0xfffffffe are never ids.  One
// dimension must fit a signed 32-bit integer (the tile descriptors).
constexpr int64_t kMaxVertices = 0xfffffffeLL;
constexpr int64_t kMaxDim = (1LL << 31) - 1;

static int make_plan(const int64_t *dims, int32_t nf, Plan &p, const int *shape_override = nullptr)
{
    if (!dims || nf < 1) return MT_ERR_INVALID_ARG;
    int shape[3];
    {
        std::lock_guard<std::mutex> lk(g_cfg_mu);
        read_env_locked();
        for (int c = 0; c < 3; ++c) shape[c] = shape_override ? shape_override[c] : g_shape[c];
        p.remap = g_remap;
        p.mgroups = g_mgroups;
        p.cap = g_cap;
        p.probes = g_probes;
        p.count = g_count;
    }
    p.d.assign(nf, FieldDesc{});
    p.q_cap = 0;
    int64_t off = 0, chunks = 0, mcap = 0;
    for (int32_t i = 0; i < nf; ++i) {
        const int64_t nx = dims[3 * i], ny = dims[3 * i + 1], nz = dims[3 * i + 2];
        if (nx < 1 || ny < 1 || nz < 1) return MT_ERR_INVALID_ARG;
        if (nx > kMaxDim || ny > kMaxDim || nz > kMaxDim) return MT_ERR_TOO_LARGE;
        if (nx * ny > kMaxVertices || nx * ny * nz > kMaxVertices) return MT_ERR_TOO_LARGE;
        const int64_t n = nx * ny * nz;
        FieldDesc &d = p.d[i];
        d.nx = (int32_t)nx; d.ny = (int32_t)ny; d.nz = (int32_t)nz;
        d.offset = off;
        d.n = n;
        d.chunk_start = chunks;
        off += n;
        chunks += (n + kChunk - 1) / kChunk;
        mcap += (n + 1) / 2;  // local minima of a tile are pairwise non-adjacent: at most
                              // half of each tile, rounded up (the tile term is added below)
        if (off > kMaxVertices) return MT_ERR_TOO_LARGE;
    }
    // tile order: 3-D fields, then 2-D, then 1-D, each in field order
    int64_t tiles = 0;
    int pos = 0;
    for (int c = 0; c < 3; ++c) {
        ClassLaunch &cl = p.cls[c];
        cl.shape = shape[c];
        cl.cb = pos;
        cl.tile0 = tiles;
        const ShapeInfo &sh = kShapes[shape[c]];
        // face edges a tile of this shape can own (+x always, +y and +z when the shape spans them)
        const int64_t faces = (int64_t)sh.ty * sh.tz + (sh.ty > 1 ? (int64_t)sh.tx * sh.tz : 0) +
                              (sh.tz > 1 ? (int64_t)sh.tx * sh.ty : 0);
        for (int32_t i = 0; i < nf; ++i) {
            FieldDesc &d = p.d[i];
            if (field_class(d.ny, d.nz) != c) continue;
            d.ntx = (int32_t)((d.nx + sh.tx - 1) / sh.tx);
            d.nty = (int32_t)((d.ny + sh.ty - 1) / sh.ty);
            d.ntz = (int32_t)((d.nz + sh.tz - 1) / sh.tz);
            d.tpos = pos++;
            d.tile_start = tiles;
            tiles += (int64_t)d.ntx * d.nty * d.ntz;
        }
        cl.nfc = pos - cl.cb;
        cl.ntiles = tiles - cl.tile0;
        // one queue per XCD; a workgroup of this class launch serves at most
        // ceil(ntiles / 8) tiles of each queue
        p.q_cap += (cl.ntiles + 7) / 8 * faces;
    }
    mcap += tiles;
    if (mcap > kMaxVertices || p.q_cap >= (1LL << 31)) return MT_ERR_TOO_LARGE;
    p.n_total = off;
    p.n_tiles = tiles;
    p.n_chunks = chunks;
    p.m_cap = mcap;
    Layout &L = p.lay;
    size_t o = align256(sizeof(Header));
    L.D = o; o = align256(o + sizeof(FieldDesc) * nf);
    L.tfield = o; o = align256(o + sizeof(int32_t) * nf);
    L.tstart = o; o = align256(o + sizeof(int64_t) * (nf + 1));
    L.cs = o; o = align256(o + sizeof(int64_t) * (nf + 1));
    L.pcnt = o; o = align256(o + sizeof(uint32_t) * chunks);
    L.lbl = o; o = align256(o + sizeof(uint32_t) * off);
    L.slot = o; o = align256(o + sizeof(Slot) * mcap);
    L.mkey = o; o = align256(o + sizeof(uint64_t) * mcap);
    L.queue = o; o = align256(o + sizeof(Fact) * p.q_cap * 8);
    L.qbin = o; o = align256(o + sizeof(Fact) * p.q_cap * 8);
    L.qhist = o; o = align256(o + sizeof(uint32_t) * kQCounters * 8);
    L.qtot = o; o = align256(o + sizeof(uint32_t) * kQScanBlocks * 8);
    L.xface = o; o = align256(o + sizeof(uint64_t) * 2 * kXFace * p.n_tiles);
    L.stage = o; o = align256(o + sizeof(uint4) * (size_t)kStagePerChunk * chunks);
    L.bcnt = o; o = align256(o + (size_t)kBuckets * chunks);
    L.total = o;
    return MT_OK;
}

struct Ptrs {
    Header *h;
    FieldDesc *D;
    int32_t *tfield;
    int64_t *tstart, *cs;
    uint32_t *pcnt, *lbl;
    Slot *slot;
    uint64_t *mkey;
    Fact *queue, *qbin;
    uint32_t *qhist, *qtot;
    uint64_t *xface;
    uint4 *stage;
    uint8_t *bcnt;
};

static Ptrs ws_ptrs(const Plan &p, void *ws)
{
    char *b = (char *)ws;
    const Layout &L = p.lay;
    Ptrs w;
    w.h = (Header *)b;
    w.D = (FieldDesc *)(b + L.D);
    w.tfield = (int32_t *)(b + L.tfield);
    w.tstart = (int64_t *)(b + L.tstart);
    w.cs = (int64_t *)(b + L.cs);
    w.pcnt = (uint32_t *)(b + L.pcnt);
    w.lbl = (uint32_t *)(b + L.lbl);
    w.slot = (Slot *)(b + L.slot);
    w.mkey = (uint64_t *)(b + L.mkey);
    w.queue = (Fact *)(b + L.queue);
    w.qbin = (Fact *)(b + L.qbin);
    w.qhist = (uint32_t *)(b + L.qhist);
    w.qtot = (uint32_t *)(b + L.qtot);
    w.xface = (uint64_t *)(b + L.xface);
    w.stage = (uint4 *)(b + L.stage);
    w.bcnt = (uint8_t *)(b + L.bcnt);
    return w;
}

// Per-kernel timing with HIP events (off unless mt_profile_begin was called).
// Launches made while a stream is being captured into a graph are not timed.
static std::mutex g_prof_mu;
static bool g_prof_on = false;
struct PendingEv {
    const char *name;
    hipEvent_t a, b;
};
static std::vector<PendingEv> g_pending;
static std::vector<hipEvent_t> g_pool;
static std::vector<std::string> g_prof_names;
static std::vector<double> g_prof_ms;
static std::vector<int64_t> g_prof_n;

static hipEvent_t pool_get()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

struct ProfScope {
    const char *name;
    hipStream_t st;
    hipEvent_t a = nullptr;
    ProfScope(const char *n, hipStream_t s) : name(n), st(s)
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        a = pool_get();
        if (a && hipEventRecord(a, st) != hipSuccess) {
            g_pool.push_back(a);
            a = nullptr;
        }
    }
    ~ProfScope()
    {
        if (!a) return;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        hipEvent_t b = pool_get();
        if (b && hipEventRecord(b, st) == hipSuccess) {
            g_pending.push_back({name, a, b});
        } else {
            g_pool.push_back(a);
            if (b) g_pool.push_back(b);
        }
    }
};

#define MT_LAUNCH(name, kernel, grid, block, st, ...)                               \
    do {                                                                            \
        ProfScope ps_(name, st);                                                    \
        hipLaunchKernelGGL(kernel, grid, block, 0, st, __VA_ARGS__);                \
        if (hipGetLastError() != hipSuccess) return MT_ERR_HIP;                     \
    } while (0)

static unsigned grid1d(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kBlock - 1) / kBlock); }

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
        MT_LAUNCH("k_setup", k_setup, dim3(1), dim3(64), st, a, w.D, w.tfield, w.tstart, w.cs, w.h);
    }
    return MT_OK;
}

template <class S, int MODE, bool LIMIT>
static int launch_local_as(const Plan &p, const ClassLaunch &cl, const Ptrs &w, const float *f, uint32_t flip,
                           hipStream_t st)
{
    auto *const kern = &k_local<S, MODE, LIMIT>;
    MT_LAUNCH("k_local", kern, dim3((unsigned)cl.ntiles), dim3(S::NT), st, f, w.lbl,
              w.slot, w.mkey, (const FieldDesc *)w.D, (const int32_t *)w.tfield + cl.cb,
              (const int64_t *)w.tstart + cl.cb, cl.nfc, cl.tile0, cl.ntiles, p.remap, (uint32_t)p.m_cap, p.cap,
              w.xface, flip, p.probes, w.h);
    return MT_OK;
}

template <class S>
static int launch_local(const Plan &p, const ClassLaunch &cl, const Ptrs &w, const float *f, uint32_t flip,
                        hipStream_t st)
{
    // a table-probe bound below the maximum only matters to tests of the
    // fallback paths: the counting build always checks it, and of the
    // timed kernel an instantiation of its own does
    if (p.count == 1) return launch_local_as<S, 1, true>(p, cl, w, f, flip, st);
    if (p.probes < (uint32_t)kMaxProbes) return launch_local_as<S, 0, true>(p, cl, w, f, flip, st);
    if (p.count == 2) return launch_local_as<S, 2, false>(p, cl, w, f, flip, st);
    return launch_local_as<S, 0, false>(p, cl, w, f, flip, st);
}

template <class S>
static int launch_cross(const Plan &p, const ClassLaunch &cl, const Ptrs &w, const float *f, uint32_t flip,
                        hipStream_t st)
{
    MT_LAUNCH("k_cross", HIP_KERNEL_NAME(k_cross<S>), dim3((unsigned)cl.ntiles), dim3(cross_threads<S>()), st, f,
              (const uint32_t *)w.lbl, w.queue, (uint32_t)p.q_cap, (const FieldDesc *)w.D,
              (const int32_t *)w.tfield + cl.cb, (const int64_t *)w.tstart + cl.cb, cl.nfc, cl.tile0, cl.ntiles,
              p.remap, w.qhist, (const uint64_t *)w.xface, flip, p.probes, w.h);
    return MT_OK;
}

// The merge tree: triplets T (field-local ids; uint32 pairs, or uint64 pairs
// when wide) and, per chunk, pair counts; with stage_pairs also the pairs
// themselves, staged per chunk for the readout that follows.
static int enqueue_build(const Plan &p, const Ptrs &w, const float *f, void *T, uint32_t flip, hipStream_t st,
                         bool wide = false, bool stage_pairs = false)
{
    const int nf = (int)p.d.size();
    const uint32_t n = (uint32_t)p.n_total;
    MT_LAUNCH("k_zero32", k_zero32, dim3(kQCounters * 8 / kBlock), dim3(kBlock), st, w.qhist,
              (int64_t)kQCounters * 8);
    for (int c = 0; c < 3; ++c) {
        const ClassLaunch &cl = p.cls[c];
        if (cl.ntiles == 0) continue;
        int rc = MT_OK;
        with_shape(cl.shape, [&](auto s) { rc = launch_local<decltype(s)>(p, cl, w, f, flip, st); });
        if (rc != MT_OK) return rc;
    }
    for (int c = 0; c < 3; ++c) {
        const ClassLaunch &cl = p.cls[c];
        if (cl.ntiles == 0) continue;
        int rc = MT_OK;
        with_shape(cl.shape, [&](auto s) { rc = launch_cross<decltype(s)>(p, cl, w, f, flip, st); });
        if (rc != MT_OK) return rc;
    }
    // facts into ascending order of their saddle's key bin, per XCD queue
    const unsigned gq =
        8 * (unsigned)std::min<int64_t>(p.mgroups, std::max<int64_t>(1, (p.q_cap + kBlock - 1) / kBlock));
    MT_LAUNCH("k_qtotals", k_qtotals, dim3(kQScanBlocks, 8), dim3(kQScanThreads), st, (const uint32_t *)w.qhist,
              w.qtot);
    MT_LAUNCH("k_qscan", k_qscan, dim3(kQScanBlocks, 8), dim3(kQScanThreads), st, w.qhist,
              (const uint32_t *)w.qtot);
    MT_LAUNCH("k_qscatter", k_qscatter, dim3(gq), dim3(kBlock), st, (const Fact *)w.queue, w.qbin,
              (uint32_t)p.q_cap, w.qhist, w.h);
    if (p.count == 1)
        MT_LAUNCH("k_merge_q", k_merge_q<true>, dim3(gq), dim3(kBlock), st, f, (const Fact *)w.qbin,
                  (uint32_t)p.q_cap, w.slot, (const uint64_t *)w.mkey, n, p.cap, flip, w.h);
    else
        MT_LAUNCH("k_merge_q", k_merge_q<false>, dim3(gq), dim3(kBlock), st, f, (const Fact *)w.qbin,
                  (uint32_t)p.q_cap, w.slot, (const uint64_t *)w.mkey, n, p.cap, flip, w.h);
    const unsigned gm = (unsigned)std::min<int64_t>(8192, std::max<int64_t>(1, (p.m_cap + kBlock - 1) / kBlock));
    if (p.count == 1)
        MT_LAUNCH("k_repair_min", k_repair_min<true>, dim3(gm), dim3(kBlock), st, f, w.slot,
                  (const uint64_t *)w.mkey, n, p.cap, flip, w.h);
    else
        MT_LAUNCH("k_repair_min", k_repair_min<false>, dim3(gm), dim3(kBlock), st, f, w.slot,
                  (const uint64_t *)w.mkey, n, p.cap, flip, w.h);
    auto reg = [&](auto cnt, auto out) {
        using O = decltype(out);
        auto *const kern = &k_repair_reg<decltype(cnt)::value, O>;
        MT_LAUNCH("k_repair_reg", kern, dim3((unsigned)p.n_chunks), dim3(kBlock), st, f, (const uint32_t *)w.lbl,
                  w.slot, (typename O::Word *)T, w.pcnt,
                  stage_pairs ? w.stage : nullptr, stage_pairs ? w.bcnt : nullptr, (const FieldDesc *)w.D,
                  (const int64_t *)w.cs, nf, n, p.cap, flip, w.h);
        return MT_OK;
    };
    using CT = std::true_type;
    using CF = std::false_type;
    if (wide) return p.count == 1 ? reg(CT{}, Out64{}) : reg(CF{}, Out64{});
    return p.count == 1 ? reg(CT{}, Out32{}) : reg(CF{}, Out32{});
}

template <class O>
static int enqueue_pairs_as(const Plan &p, const Ptrs &w, bool after_build, const float *f, const void *Tv,
                            int64_t capacity, void *birth, void *death, float *bval, float *dval,
                            int64_t *pair_offsets, hipStream_t st)
{
    const int nf = (int)p.d.size();
    const typename O::Word *T = (const typename O::Word *)Tv;
    if (!after_build) {
        auto *const kc = &k_pairs_count<O>;
        MT_LAUNCH("k_pairs_count", kc, dim3((unsigned)p.n_chunks), dim3(kBlock), st, T, (const FieldDesc *)w.D,
                  (const int64_t *)w.cs, nf, w.pcnt, w.h);
    }
    MT_LAUNCH("k_pairs_scan", k_pairs_scan, dim3(1), dim3(1024), st, w.pcnt, p.n_chunks, (const FieldDesc *)w.D, nf,
              pair_offsets, capacity, w.h);
    auto *const kw = &k_pairs_write<O>;
    MT_LAUNCH("k_pairs_write", kw, dim3((unsigned)p.n_chunks), dim3(kBlock), st, f, T, (const FieldDesc *)w.D,
              (const int64_t *)w.cs, nf, (const uint32_t *)w.pcnt, capacity, (typename O::Id *)birth,
              (typename O::Id *)death, bval, dval, after_build ? (const uint4 *)w.stage : nullptr,
              after_build ? (const uint8_t *)w.bcnt : nullptr);
    return MT_OK;
}

// Pairs of T: counts (unless the build just counted them: its output pass
// leaves the pair count of every chunk in the workspace), scan, ordered write.
static int enqueue_pairs(const Plan &p, const Ptrs &w, bool after_build, const float *f, const void *T,
                         int64_t capacity, void *birth, void *death, float *bval, float *dval,
                         int64_t *pair_offsets, hipStream_t st, bool wide = false)
{
    return wide ? enqueue_pairs_as<Out64>(p, w, after_build, f, T, capacity, birth, death, bval, dval, pair_offsets, st)
                : enqueue_pairs_as<Out32>(p, w, after_build, f, T, capacity, birth, death, bval, dval, pair_offsets, st);
}

// Any difference between two triplet arrays latches ST_CORRUPT (autotuner check).
__global__ void k_compare(const uint64_t *__restrict__ a, const uint64_t *__restrict__ b, int64_t n,
                          uint32_t *__restrict__ status)
{
    bool diff = false;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
        diff |= a[i] != b[i];
    if (__ballot(diff) != 0ull && (threadIdx.x & 63) == 0) atomicOr(status, ST_CORRUPT);
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

static int check_ws(const Plan &p, const void *ws, size_t bytes)
{
    if (!ws || ((uintptr_t)ws & 255u) || bytes < p.lay.total) return MT_ERR_WORKSPACE;
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

static uint32_t kind_flip(int kind) { return kind == MT_TREE_SPLIT ? 0xffffffffu : 0u; }

int mt_build(const float *field, int64_t nx, int64_t ny, int64_t nz, uint32_t *triplets, void *workspace,
             size_t ws_bytes, void *stream)
{
    return mt_build_tree(field, nx, ny, nz, MT_TREE_MERGE, triplets, workspace, ws_bytes, stream);
}

int mt_build_tree(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind, uint32_t *triplets,
                  void *workspace, size_t ws_bytes, void *stream)
{
    if (kind != MT_TREE_MERGE && kind != MT_TREE_SPLIT) return MT_ERR_INVALID_ARG;
    const int64_t dims[3] = {nx, ny, nz};
    Plan p;
    int rc = make_plan(dims, 1, p);
    if (rc != MT_OK) return rc;
    if (!field || !triplets || ((uintptr_t)triplets & 7u)) return MT_ERR_INVALID_ARG;
    if ((rc = check_ws(p, workspace, ws_bytes)) != MT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const Ptrs w = ws_ptrs(p, workspace);
    rc = enqueue_setup(p, w, ~0u, true, st);
    if (rc != MT_OK) return rc;
    return enqueue_build(p, w, field, (uint64_t *)triplets, kind_flip(kind), st);
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
    if ((rc = check_ws(p, workspace, ws_bytes)) != MT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const Ptrs w = ws_ptrs(p, workspace);
    rc = enqueue_setup(p, w, ST_CAPACITY | ST_CORRUPT, true, st);
    if (rc != MT_OK) return rc;
    rc = enqueue_pairs(p, w, false, field, (const uint64_t *)triplets, capacity, birth, death, birth_val, death_val,
                       nullptr, st);
    if (rc != MT_OK) return rc;
    Header h;
    rc = read_header(workspace, st, h);
    if (rc != MT_OK) return rc;
    *n_pairs = h.total_pairs;
    if (n_roots) *n_roots = h.roots;
    return status_to_code(h.status);
}

static int build_pairs(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind, void *triplets,
                       void *birth, void *death, float *birth_val, float *death_val, int64_t capacity,
                       int64_t *n_pairs, int64_t *n_roots, void *workspace, size_t ws_bytes, void *stream, bool wide)
{
    if (kind != MT_TREE_MERGE && kind != MT_TREE_SPLIT) return MT_ERR_INVALID_ARG;
    const int64_t dims[3] = {nx, ny, nz};
    Plan p;
    int rc = make_plan(dims, 1, p);
    if (rc != MT_OK) return rc;
    const uintptr_t talign = wide ? 15u : 7u;
    if (!field || !triplets || ((uintptr_t)triplets & talign) || !n_pairs || capacity < 0) return MT_ERR_INVALID_ARG;
    if (capacity > 0 && (!birth || !death || !birth_val || !death_val)) return MT_ERR_INVALID_ARG;
    if ((rc = check_ws(p, workspace, ws_bytes)) != MT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    const Ptrs w = ws_ptrs(p, workspace);
    if ((rc = enqueue_setup(p, w, ~0u, true, st)) != MT_OK) return rc;
    if ((rc = enqueue_build(p, w, field, triplets, kind_flip(kind), st, wide, true)) != MT_OK) return rc;
    rc = enqueue_pairs(p, w, true, field, triplets, capacity, birth, death, birth_val, death_val, nullptr, st, wide);
    if (rc != MT_OK) return rc;
    Header h;
    if ((rc = read_header(workspace, st, h)) != MT_OK) return rc;
    *n_pairs = h.total_pairs;
    if (n_roots) *n_roots = h.roots;
    return status_to_code(h.status);
}

int mt_build_pairs(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind, uint32_t *triplets,
                   uint32_t *birth, uint32_t *death, float *birth_val, float *death_val, int64_t capacity,
                   int64_t *n_pairs, int64_t *n_roots, void *workspace, size_t ws_bytes, void *stream)
{
    return build_pairs(field, nx, ny, nz, kind, triplets, birth, death, birth_val, death_val, capacity, n_pairs,
                       n_roots, workspace, ws_bytes, stream, false);
}

int mt_build_pairs64(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind, uint64_t *triplets,
                     uint64_t *birth, uint64_t *death, float *birth_val, float *death_val, int64_t capacity,
                     int64_t *n_pairs, int64_t *n_roots, void *workspace, size_t ws_bytes, void *stream)
{
    return build_pairs(field, nx, ny, nz, kind, triplets, birth, death, birth_val, death_val, capacity, n_pairs,
                       n_roots, workspace, ws_bytes, stream, true);
}

}  // extern "C"

// Allocation-free variant of mt_build_pairs ---------------------------------
//
// Its workspace is this fixed device array instead of a caller's buffer.  The
// array's name is a host-side handle only: host code never passes it to a
// kernel or a copy.  Its device address, which differs per GPU, is looked up
// once per device with hipGetSymbolAddress (with that device current) and
// kept in g_scratch; every launch and copy uses that address.  Each GPU the
// library runs on holds its copy of the array until the process ends.
namespace {
static __device__ __align__(256) unsigned char scratch[MT_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;                       // held for the whole call
static std::unordered_map<int, void *> g_scratch;     // device -> address of `scratch`

static int scratch_address(int dev, void **out)
{
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) {
        *out = it->second;
        return MT_OK;
    }
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return MT_ERR_HIP;
    g_scratch.emplace(dev, ptr);
    *out = ptr;
    return MT_OK;
}
}  // namespace

extern "C" {

size_t mt_noalloc_scratch_bytes(void) { return MT_NOALLOC_SCRATCH_BYTES; }

int mt_build_pairs_noalloc(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind, uint32_t *triplets,
                           uint32_t *birth, uint32_t *death, float *birth_val, float *death_val, int64_t capacity,
                           int64_t *n_pairs, int64_t *n_roots, void *stream)
{
    const int64_t dims[3] = {nx, ny, nz};
    Plan p;
    const int rc = make_plan(dims, 1, p);
    if (rc != MT_OK) return rc;
    if (p.lay.total > (size_t)MT_NOALLOC_SCRATCH_BYTES) return MT_ERR_TOO_LARGE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MT_ERR_HIP;
    // One call at a time per process: the call synchronizes its stream before
    // it returns, so holding the lock keeps every use of the array apart.
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    void *ws = nullptr;
    if (scratch_address(dev, &ws) != MT_OK) return MT_ERR_HIP;
    return build_pairs(field, nx, ny, nz, kind, triplets, birth, death, birth_val, death_val, capacity, n_pairs,
                       n_roots, ws, (size_t)MT_NOALLOC_SCRATCH_BYTES, stream, false);
}

int mt_batch_build(const float *fields, const int64_t *dims, int32_t n_fields, uint32_t *triplets, uint32_t *birth,
                   uint32_t *death, float *birth_val, float *death_val, int64_t pair_capacity,
                   int64_t *pair_offsets, void *workspace, size_t ws_bytes, void *stream)
{
    return mt_batch_build_tree(fields, dims, n_fields, MT_TREE_MERGE, triplets, birth, death, birth_val, death_val,
                               pair_capacity, pair_offsets, workspace, ws_bytes, stream);
}

int mt_batch_build_tree(const float *fields, const int64_t *dims, int32_t n_fields, int kind, uint32_t *triplets,
                        uint32_t *birth, uint32_t *death, float *birth_val, float *death_val,
                        int64_t pair_capacity, int64_t *pair_offsets, void *workspace, size_t ws_bytes,
                        void *stream)
{
    if (kind != MT_TREE_MERGE && kind != MT_TREE_SPLIT) return MT_ERR_INVALID_ARG;
    Plan p;
    int rc = make_plan(dims, n_fields, p);
    if (rc != MT_OK) return rc;
    if (!fields || !triplets || ((uintptr_t)triplets & 7u) || !pair_offsets || pair_capacity < 0)
        return MT_ERR_INVALID_ARG;
    if (pair_capacity > 0 && (!birth || !death || !birth_val || !death_val)) return MT_ERR_INVALID_ARG;
    if ((rc = check_ws(p, workspace, ws_bytes)) != MT_OK) return rc;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MT_ERR_HIP;
    std::string key;
    key.reserve(96 + 24 * n_fields);
    char buf[320];
    snprintf(buf, sizeof buf, "%d|%d|%p|%p|%p|%p|%p|%p|%lld|%p|%p|%zu|%d|%d|%u|%u|%d|%d,%d,%d", dev, kind,
             (const void *)fields, (void *)triplets, (void *)birth, (void *)death, (void *)birth_val,
             (void *)death_val, (long long)pair_capacity, (void *)pair_offsets, workspace, ws_bytes, p.remap,
             p.mgroups, p.cap,
             p.probes, p.count, p.cls[0].shape, p.cls[1].shape, p.cls[2].shape);
    key += buf;
    for (const FieldDesc &d : p.d) {
        snprintf(buf, sizeof buf, "|%d,%d,%d", d.nx, d.ny, d.nz);
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
        if (rc1 == MT_OK) rc1 = enqueue_build(p, w, fields, (uint64_t *)triplets, kind_flip(kind), cs, false, true);
        if (rc1 == MT_OK)
            rc1 = enqueue_pairs(p, w, true, fields, (const uint64_t *)triplets, pair_capacity, birth, death,
                                birth_val, death_val, pair_offsets, cs);
        GraphEntry e;
        const hipError_t ec = hipStreamEndCapture(cs, &e.graph);
        if (rc1 != MT_OK || ec != hipSuccess) {
            if (e.graph) (void)hipGraphDestroy(e.graph);
            return rc1 != MT_OK ? rc1 : MT_ERR_HIP;
        }
        if (hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(e.graph);
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

// Vertex ranks --------------------------------------------------------------

namespace {
struct RankLayout {
    size_t keys = 0, sorted = 0, tmp = 0, tmp_bytes = 0, total = 0;
};

int rank_layout(int64_t nx, int64_t ny, int64_t nz, RankLayout &L)
{
    if (nx < 1 || ny < 1 || nz < 1) return MT_ERR_INVALID_ARG;
    if (nx > kMaxDim || ny > kMaxDim || nz > kMaxDim || nx * ny > kMaxVertices || nx * ny * nz > kMaxVertices)
        return MT_ERR_TOO_LARGE;
    const size_t n = (size_t)(nx * ny * nz);
    size_t tmp = 0;  // a size query: nothing is launched
    if (rocprim::radix_sort_keys(nullptr, tmp, (const uint64_t *)nullptr, (uint64_t *)nullptr, n, 0, 64) !=
        hipSuccess)
        return MT_ERR_HIP;
    size_t o = align256(sizeof(Header));
    L.keys = o; o = align256(o + sizeof(uint64_t) * n);
    L.sorted = o; o = align256(o + sizeof(uint64_t) * n);
    L.tmp = o; L.tmp_bytes = tmp; o = align256(o + std::max<size_t>(tmp, 1));
    L.total = o;
    return MT_OK;
}
}  // namespace

size_t mt_rank_workspace_bytes(int64_t nx, int64_t ny, int64_t nz)
{
    RankLayout L;
    return rank_layout(nx, ny, nz, L) == MT_OK ? L.total : 0;
}

int mt_vertex_ranks(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind, uint32_t *ranks,
                    void *workspace, size_t ws_bytes, void *stream)
{
    if (kind != MT_TREE_MERGE && kind != MT_TREE_SPLIT) return MT_ERR_INVALID_ARG;
    RankLayout L;
    const int rc = rank_layout(nx, ny, nz, L);
    if (rc != MT_OK) return rc;
    if (!field || !ranks) return MT_ERR_INVALID_ARG;
    if (!workspace || ((uintptr_t)workspace & 255u) || ws_bytes < L.total) return MT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    char *b = (char *)workspace;
    Header *h = (Header *)b;
    const uint32_t n = (uint32_t)(nx * ny * nz);
    uint64_t *keys = (uint64_t *)(b + L.keys), *sorted = (uint64_t *)(b + L.sorted);
    const unsigned g = (unsigned)std::min<int64_t>(8192, ((int64_t)n + kBlock - 1) / kBlock);
    MT_LAUNCH("k_zero32", k_zero32, dim3(grid1d((int64_t)(sizeof(Header) / 4))), dim3(kBlock), st, (uint32_t *)h,
              (int64_t)(sizeof(Header) / 4));
    MT_LAUNCH("k_rank_keys", k_rank_keys, dim3(g), dim3(kBlock), st, field, n, kind_flip(kind), keys, h);
    {
        ProfScope ps_("radix_sort", st);
        size_t tb = L.tmp_bytes;
        if (rocprim::radix_sort_keys((void *)(b + L.tmp), tb, (const uint64_t *)keys, sorted, (size_t)n, 0, 64,
                                     st) != hipSuccess)
            return MT_ERR_HIP;
    }
    MT_LAUNCH("k_rank_scatter", k_rank_scatter, dim3(g), dim3(kBlock), st, (const uint64_t *)sorted, n, ranks);
    return MT_OK;
}

int mt_tile_shape_count(void) { return kNumShapes; }

int mt_tile_shape_info(int id, int *tx, int *ty, int *tz, int *threads, int *dims_class)
{
    if (id < 0 || id >= kNumShapes) return MT_ERR_INVALID_ARG;
    const ShapeInfo &s = kShapes[id];
    if (tx) *tx = s.tx;
    if (ty) *ty = s.ty;
    if (tz) *tz = s.tz;
    if (threads) *threads = s.nt;
    if (dims_class) *dims_class = s.cls;
    return MT_OK;
}

int mt_set_tile_shape(int dims_class, int id)
{
    if (dims_class < 0 || dims_class > 2 || id < 0 || id >= kNumShapes || kShapes[id].cls != dims_class)
        return MT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    g_shape[dims_class] = id;
    return MT_OK;
}

int mt_get_tile_shape(int dims_class)
{
    if (dims_class < 0 || dims_class > 2) return MT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    return g_shape[dims_class];
}

int mt_set_max_steps(int64_t steps)
{
    if (steps < 0 || steps > 0x7fffffffLL) return MT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    g_cap = steps == 0 ? kDefaultCap : (uint32_t)steps;
    return MT_OK;
}

int64_t mt_get_max_steps(void)
{
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    return g_cap;
}

int mt_set_table_probes(int probes)
{
    if (probes < -1 || probes > kMaxProbes) return MT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    g_probes = probes < 0 ? kDefaultProbes : (uint32_t)probes;
    return MT_OK;
}

int mt_get_table_probes(void)
{
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    return (int)g_probes;
}

int mt_set_counting(int on)
{
    if (on < 0 || on > 2) return MT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    g_count = on;
    return MT_OK;
}

int mt_get_counting(void)
{
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    return g_count;
}

int mt_read_counters(const void *workspace, void *stream, uint64_t *counts, int n)
{
    if (!workspace) return MT_ERR_WORKSPACE;
    if (!counts || n < 1) return MT_ERR_INVALID_ARG;
    Header h;
    const int rc = read_header(workspace, (hipStream_t)stream, h);
    if (rc != MT_OK) return rc;
    const int m = std::min(n, (int)kCtr);
    for (int i = 0; i < m; ++i) counts[i] = h.ctr[i];
    for (int i = m; i < n; ++i) counts[i] = 0;
    return m;
}

int mt_workspace_reset(void *workspace, size_t ws_bytes, void *stream)
{
    if (!workspace || ((uintptr_t)workspace & 255u) || ws_bytes < sizeof(Header)) return MT_ERR_WORKSPACE;
    hipStream_t st = (hipStream_t)stream;
    constexpr int64_t words = (int64_t)(sizeof(Header) / sizeof(uint32_t));
    MT_LAUNCH("k_zero32", k_zero32, dim3(grid1d(words)), dim3(kBlock), st, (uint32_t *)workspace, words);
    return MT_OK;
}

size_t mt_autotune_workspace_bytes(const int64_t *dims, int32_t n_fields)
{
    size_t best = 0;
    for (int a = 0; a < kNumShapes; ++a) {
        if (kShapes[a].cls != 0) continue;
        for (int b = 0; b < kNumShapes; ++b) {
            if (kShapes[b].cls != 1) continue;
            for (int c = 0; c < kNumShapes; ++c) {
                if (kShapes[c].cls != 2) continue;
                const int sh[3] = {a, b, c};
                Plan p;
                if (make_plan(dims, n_fields, p, sh) != MT_OK) return 0;
                best = std::max(best, p.lay.total);
            }
        }
    }
    return best;
}

}  // extern "C"

namespace {
// One autotuner candidate: `reps` timed builds (after one warm-up) with plan
// p into `out`; when `ref` is not null the triplets must equal ref's bit for
// bit (else MT_ERR_INTERNAL, latched by k_compare).  Synchronizes.
int time_candidate(const Plan &p, void *workspace, const float *fields, uint64_t *out, const uint64_t *ref,
                   int reps, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double &ms_per_build)
{
    const Ptrs w = ws_ptrs(p, workspace);
    int rc = MT_OK;
    for (int r = -1; r < reps && rc == MT_OK; ++r) {  // r = -1: warm-up
        if (r == 0 && hipEventRecord(e0, st) != hipSuccess) rc = MT_ERR_HIP;
        if (rc == MT_OK) rc = enqueue_setup(p, w, ~0u, true, st);
        if (rc == MT_OK) rc = enqueue_build(p, w, fields, out, 0u, st);
    }
    if (rc != MT_OK) return rc;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return MT_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return MT_ERR_HIP;
    if (ref) {
        hipLaunchKernelGGL(k_compare, dim3(1024), dim3(kBlock), 0, st, ref, (const uint64_t *)out, p.n_total,
                           &w.h->status);
        if (hipGetLastError() != hipSuccess) return MT_ERR_HIP;
    }
    Header h;
    if ((rc = read_header(workspace, st, h)) != MT_OK) return rc;
    if ((rc = status_to_code(h.status)) != MT_OK) return rc;
    ms_per_build = (double)ms / reps;
    return MT_OK;
}

// Candidates of the schedule tuner: XCD-aware tile order on or off, and the
// workgroups per XCD of the fact scatter and cross-tile merge.
constexpr int kSchedRemap[] = {1, 0};
constexpr int kSchedGroups[] = {256, 1024, 2048, 8192};
}  // namespace

extern "C" {

int mt_autotune(const float *fields, const int64_t *dims, int32_t n_fields, uint32_t *triplets,
                uint32_t *triplets_check, void *workspace, size_t ws_bytes, int reps, void *stream,
                double *best_ms)
{
    if (!fields || !triplets || !triplets_check || reps < 1) return MT_ERR_INVALID_ARG;
    if (((uintptr_t)triplets & 7u) || ((uintptr_t)triplets_check & 7u)) return MT_ERR_INVALID_ARG;
    Plan p0;
    int rc = make_plan(dims, n_fields, p0);
    if (rc != MT_OK) return rc;
    if ((rc = check_ws(p0, workspace, ws_bytes)) != MT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MT_ERR_HIP;
    int shape[3];
    for (int c = 0; c < 3; ++c) shape[c] = mt_get_tile_shape(c);
    bool have_ref = false;
    rc = MT_OK;
    for (int c = 0; c < 3 && rc == MT_OK; ++c) {
        if (best_ms) best_ms[c] = -1.0;
        if (p0.cls[c].ntiles == 0) continue;
        int best_id = shape[c];
        double best_t = 1e300;
        for (int id = 0; id < kNumShapes && rc == MT_OK; ++id) {
            if (kShapes[id].cls != c) continue;
            int sh[3] = {shape[0], shape[1], shape[2]};
            sh[c] = id;
            Plan p;
            if ((rc = make_plan(dims, n_fields, p, sh)) != MT_OK) break;
            if (p.lay.total > ws_bytes) continue;  // does not fit the caller's workspace
            double t = 0.0;
            // the first candidate writes the reference, every later one is compared with it
            rc = time_candidate(p, workspace, fields, (uint64_t *)(have_ref ? triplets_check : triplets),
                                have_ref ? (const uint64_t *)triplets : nullptr, reps, st, e0, e1, t);
            if (rc != MT_OK) break;
            have_ref = true;
            if (t < best_t) {
                best_t = t;
                best_id = id;
            }
        }
        if (rc == MT_OK) {
            shape[c] = best_id;
            mt_set_tile_shape(c, best_id);
            if (best_ms) best_ms[c] = best_t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

int mt_set_schedule(int xcd_remap, int merge_groups)
{
    if (xcd_remap < -1 || xcd_remap > 1 || merge_groups < 0 || merge_groups > 65536) return MT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    g_remap = xcd_remap < 0 ? 1 : xcd_remap;
    g_mgroups = merge_groups == 0 ? kDefaultMergeGroups : merge_groups;
    return MT_OK;
}

int mt_get_schedule(int *xcd_remap, int *merge_groups)
{
    std::lock_guard<std::mutex> lk(g_cfg_mu);
    read_env_locked();
    if (xcd_remap) *xcd_remap = g_remap;
    if (merge_groups) *merge_groups = g_mgroups;
    return MT_OK;
}

int mt_autotune_schedule(const float *fields, const int64_t *dims, int32_t n_fields, uint32_t *triplets,
                         uint32_t *triplets_check, void *workspace, size_t ws_bytes, int reps, void *stream,
                         double *best_ms)
{
    if (!fields || !triplets || !triplets_check || reps < 1) return MT_ERR_INVALID_ARG;
    if (((uintptr_t)triplets & 7u) || ((uintptr_t)triplets_check & 7u)) return MT_ERR_INVALID_ARG;
    Plan p;
    int rc = make_plan(dims, n_fields, p);
    if (rc != MT_OK) return rc;
    if ((rc = check_ws(p, workspace, ws_bytes)) != MT_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return MT_ERR_HIP;
    int best_r = p.remap, best_g = p.mgroups;
    double best_t = 1e300;
    bool have_ref = false;
    for (int r : kSchedRemap) {
        for (int g : kSchedGroups) {
            p.remap = r;
            p.mgroups = g;
            double t = 0.0;
            rc = time_candidate(p, workspace, fields, (uint64_t *)(have_ref ? triplets_check : triplets),
                                have_ref ? (const uint64_t *)triplets : nullptr, reps, st, e0, e1, t);
            if (rc != MT_OK) break;
            have_ref = true;
            if (t < best_t) {
                best_t = t;
                best_r = r;
                best_g = g;
            }
        }
        if (rc != MT_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != MT_OK) return rc;
    if (best_ms) *best_ms = best_t;
    return mt_set_schedule(best_r, best_g);
}

int mt_build_stats(const void *workspace, void *stream, int64_t *n_local_minima, int64_t *n_cross_facts)
{
    if (!workspace) return MT_ERR_WORKSPACE;
    if (!n_local_minima) return MT_ERR_INVALID_ARG;
    Header h;
    const int rc = read_header(workspace, (hipStream_t)stream, h);
    if (rc != MT_OK) return rc;
    *n_local_minima = h.n_minima;
    if (n_cross_facts) {
        int64_t t = 0;
        for (int x = 0; x < 8; ++x) t += h.n_cross[x * kXStride];
        *n_cross_facts = t;
    }
    return MT_OK;
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
        if (nx > kMaxDim || ny > kMaxDim || nz > kMaxDim) return MT_ERR_TOO_LARGE;
        if (nx * ny > kMaxVertices || nx * ny * nz > kMaxVertices) return MT_ERR_TOO_LARGE;
        voff[i] = off;
        off += nx * ny * nz;
        if (off > kMaxVertices) return MT_ERR_TOO_LARGE;
    }
    voff[n_fields] = off;
    hipStream_t st = (hipStream_t)stream;
    if (!accumulate)
        MT_LAUNCH("k_fill0", k_fill0, dim3((unsigned)std::min<int64_t>(8192, grid1d((off + 3) / 4))), dim3(kBlock), st,
                  grad_field, off);
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
        MT_LAUNCH("k_scatter", k_scatter, dim3(blocks), dim3(kBlock), st, g, pair_offsets, pair_capacity, birth,
                  death, grad_birth, grad_death, grad_field);
    }
    return MT_OK;
}

int mt_profile_begin(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = true;
    g_prof_names.clear();
    g_prof_ms.clear();
    g_prof_n.clear();
    return MT_OK;
}

int mt_profile_end(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = false;
    int rc = MT_OK;
    for (const PendingEv &e : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(e.b) != hipSuccess || hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) {
            rc = MT_ERR_HIP;
        } else {
            size_t i = 0;
            while (i < g_prof_names.size() && g_prof_names[i] != e.name) ++i;
            if (i == g_prof_names.size()) {
                g_prof_names.emplace_back(e.name);
                g_prof_ms.push_back(0.0);
                g_prof_n.push_back(0);
            }
            g_prof_ms[i] += ms;
            g_prof_n[i] += 1;
        }
        g_pool.push_back(e.a);
        g_pool.push_back(e.b);
    }
    g_pending.clear();
    return rc;
}

int mt_profile_count(void)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return (int)g_prof_names.size();
}

int mt_profile_get(int i, char *name, size_t name_len, double *total_ms, int64_t *launches)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (i < 0 || (size_t)i >= g_prof_names.size() || !name || name_len == 0) return MT_ERR_INVALID_ARG;
    snprintf(name, name_len, "%s", g_prof_names[i].c_str());
    if (total_ms) *total_ms = g_prof_ms[i];
    if (launches) *launches = g_prof_n[i];
    return MT_OK;
}

void mt_release_caches(void)
{
    {
        std::lock_guard<std::mutex> lk(g_graph_mu);
        for (auto &kv : g_graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        }
        g_graphs.clear();
        for (auto &kv : g_capture_streams) (void)hipStreamDestroy(kv.second);
        g_capture_streams.clear();
    }
    std::lock_guard<std::mutex> lp(g_prof_mu);
    for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
    g_pool.clear();
}

}  // extern "C"
