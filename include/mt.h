/*
 * mt.h -- C ABI of the MI355X triplet merge tree library (libmt.so).
 *
 * The library computes, on one AMD MI355X (gfx950), the merge tree of a
 * float32 scalar field on a 1-D, 2-D or 3-D regular grid in the triplet
 * representation of "Fast Merge Tree Computation via SYCL" (arXiv 2301.10838),
 * Sec. 2, "Triplet merge trees": every vertex u owns exactly one triplet
 * (u, s, v), stored as T[u] = (s, v), meaning that the branch born at u joins
 * the branch of the deeper vertex v at the saddle s; (u, u, u) marks the
 * global minimum of a connected component and (u, u, v) a vertex of degree
 * two.  The stored representation is the unique normalized and minimal one
 * (v is the deepest vertex of u's component of the sublevel set at the level
 * of s), which is what makes results comparable bit for bit.  It also reads
 * out the zero-dimensional persistence pairs, one per branch (Sec. 1), and
 * scatters gradients of a loss on those pairs back onto the field.
 *
 * Conventions shared by every call:
 *  - A field of nx*ny*nz values is C-contiguous [nz][ny][nx]; vertex id
 *    u = x + nx*(y + ny*z).  A 2-D field has nz = 1, a 1-D field ny = nz = 1.
 *    Edges join axis neighbours (6, 4 or 2 per vertex), the grid graph the
 *    paper builds by connecting neighbouring grid points (Sec. 1).
 *  - Vertices are ordered by value, ties by id: u precedes w iff
 *    f[u] < f[w] or (f[u] == f[w] and u < w), with the IEEE comparison
 *    (-0.0 == +0.0).  The paper's definitions use strict inequalities on
 *    distinct values; the id tie-break is this library's reading for repeats.
 *  - Ids are unsigned 32-bit inside the library (Sec. 3.2 packs a pair into
 *    one 64-bit word, replaced by one 64-bit compare-and-swap); a field, or a
 *    whole batch, may hold up to 2^32 - 2 vertices, each dimension below
 *    2^31.  Ids of 2^31 and more read as negative in signed 32-bit views;
 *    mt_build_pairs64 writes the same results with 64-bit ids.
 *  - T is uint32[N][2] = (s, v): one 8-byte-aligned 64-bit word per vertex,
 *    s in the low half.  Ids in every output are local to their field.
 *  - Pointers marked (device) are device memory on the current HIP device,
 *    allocated by the caller (hipMalloc, a torch tensor, ...); the caller owns
 *    every buffer.  The library allocates no memory per call; it keeps only
 *    cached graph plans, released by mt_release_caches.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued asynchronously unless the call says it synchronizes.
 *  - Every call returns an mt_status.  Host-side argument checks run before
 *    anything is enqueued.  Conditions found on the device (NaN input, a
 *    step cap exceeded, too small a pair capacity) are latched in a status
 *    word inside the workspace and returned by the next synchronizing call
 *    on that workspace (mt_persistence_pairs, mt_sync_status).
 */
#ifndef MT_H
#define MT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MT_OK = 0,
    MT_ERR_INVALID_ARG = -1, /* bad dims, null or misaligned pointer, bad count */
    MT_ERR_TOO_LARGE = -2,   /* more than 2^32 - 2 vertices, or a dimension of 2^31 or more */
    MT_ERR_NAN = -3,         /* the field holds a NaN: no order exists */
    MT_ERR_CAPACITY = -4,    /* more pairs than the output capacity */
    MT_ERR_LIVELOCK = -5,    /* a merge or chase exceeded its step cap */
    MT_ERR_WORKSPACE = -6,   /* workspace null or smaller than required */
    MT_ERR_HIP = -7,         /* a HIP runtime call failed */
    MT_ERR_INTERNAL = -8     /* a kernel met an out-of-range id (broken invariant); output invalid */
} mt_status;

/* Which tree: the merge (join) tree of sublevel sets, vertices ordered by
 * (value, id) -- the paper's definition (Sec. 2) -- or the split tree of
 * superlevel sets, the setting the paper's experiments report (Sec. 4): the
 * merge tree of -f, vertices ordered by (-value, id).  For the split tree the
 * triplets, pairs and minima below read "maxima"; pair values stay bit copies
 * of f. */
enum {
    MT_TREE_MERGE = 0,
    MT_TREE_SPLIT = 1
};

/* Human-readable name of a status code (static string). */
const char *mt_status_string(int status);

/* Bytes of device workspace one field of nx*ny*nz vertices needs; 0 if the
 * dims are invalid. */
size_t mt_workspace_bytes(int64_t nx, int64_t ny, int64_t nz);

/* Bytes of device workspace a batch needs.  dims (host) is int64[n_fields][3]
 * = (nx, ny, nz) per field.  0 if any entry is invalid. */
size_t mt_batch_workspace_bytes(const int64_t *dims, int32_t n_fields);

/*
 * mt_build -- merge tree of one field (paper Alg. 1, ComputeMergeTree).
 *
 * field     (device) float[nx*ny*nz], read only.
 * triplets  (device) uint32[N][2], written: T[u] = (s, v) as described above.
 * workspace (device) at least mt_workspace_bytes(nx, ny, nz) bytes, 256-byte
 *           aligned; scratch for the call, and it carries the latched device
 *           status to a following mt_persistence_pairs on the same workspace.
 *
 * Steps, all on `stream`, asynchronous:
 *  1. every vertex points at its lowest lower neighbour (or at itself when it
 *     is a local minimum, which is the initial triplet (u, u, u) of Alg. 1);
 *     this is the state Alg. 3 reaches by merging those edges in decreasing
 *     order of their upper vertex;
 *  2. those chains are compressed to the minimum each vertex descends to;
 *  3. every grid edge whose ends descend to different minima is merged with
 *     the lock-free path merge of Alg. 3 (64-bit compare-and-swap, Alg. 2);
 *     the others are already implied and need no merge;
 *  4. repair (Alg. 4, 5) restores minimality, minima first, then every other
 *     vertex.
 * Errors: MT_ERR_INVALID_ARG, MT_ERR_TOO_LARGE, MT_ERR_WORKSPACE, MT_ERR_HIP
 * synchronously; MT_ERR_NAN / MT_ERR_LIVELOCK latched in the workspace.
 */
int mt_build(const float *field, int64_t nx, int64_t ny, int64_t nz,
             uint32_t *triplets, void *workspace, size_t ws_bytes, void *stream);

/*
 * mt_build_tree -- mt_build for either tree: kind = MT_TREE_MERGE (the same
 * as mt_build) or MT_TREE_SPLIT (the merge tree of -f, Sec. 4); any other
 * kind is MT_ERR_INVALID_ARG.  Arguments, ownership and errors as mt_build.
 */
int mt_build_tree(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind,
                  uint32_t *triplets, void *workspace, size_t ws_bytes, void *stream);

/*
 * mt_persistence_pairs -- zero-dimensional persistence pairs of a merge tree
 * (Sec. 1: one point (f(a), f(b)) per branch from minimum a to saddle b).
 *
 * Reads only `field` and `triplets` (device): a pair is every u with
 * T[u] = (s, v), s != u, emitted in ascending birth id u with death id s and
 * values f[u], f[s] (bit copies).  Triplets (u, u, u) are the essential
 * branches, one per connected component; they are counted in *n_roots.
 *
 * birth, death (device) uint32[capacity]; birth_val, death_val (device)
 * float[capacity].  capacity >= ceil(N/2) always suffices.
 * n_pairs (host, required) receives the number of pairs, also when it exceeds
 * capacity (then only the first `capacity` are written and the call returns
 * MT_ERR_CAPACITY).  n_roots (host) may be NULL.
 * workspace: as for mt_build; pass the one mt_build used so its latched
 * status (NaN, livelock) is reported here.  Any other workspace must first be
 * cleared with mt_workspace_reset, or its leftover bytes may read as a
 * latched error.
 * Synchronizes `stream` once, to return the counts and the status.
 */
int mt_persistence_pairs(const float *field, const uint32_t *triplets,
                         int64_t nx, int64_t ny, int64_t nz,
                         uint32_t *birth, uint32_t *death, float *birth_val, float *death_val,
                         int64_t capacity, int64_t *n_pairs, int64_t *n_roots,
                         void *workspace, size_t ws_bytes, void *stream);

/*
 * mt_build_pairs -- mt_build_tree followed by mt_persistence_pairs in one
 * call (Alg. 1, then the pairs of Sec. 1), with the same results.  The
 * build's output pass already counts the pairs of every chunk of vertices,
 * so the readout skips its own counting pass over T.
 *
 * kind: as in mt_build_tree.  field, triplets: as in mt_build.  birth,
 * death, birth_val, death_val, capacity, n_pairs, n_roots: as in
 * mt_persistence_pairs.  workspace: mt_workspace_bytes(nx, ny, nz) bytes.
 * Errors: the synchronous ones of both calls; the status latched by the
 * build or the readout (MT_ERR_NAN, MT_ERR_LIVELOCK, MT_ERR_CAPACITY) is
 * returned.  Synchronizes `stream` once, at the end.
 */
int mt_build_pairs(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind,
                   uint32_t *triplets, uint32_t *birth, uint32_t *death,
                   float *birth_val, float *death_val, int64_t capacity,
                   int64_t *n_pairs, int64_t *n_roots,
                   void *workspace, size_t ws_bytes, void *stream);

/*
 * mt_build_pairs64 -- mt_build_pairs with 64-bit ids in every output, for
 * callers that index with 64-bit integers (a field may hold up to 2^32 - 2
 * vertices, past the signed 32-bit range).  Sec. 5 names wider ids as future
 * work; inside, the ids stay the unsigned 32-bit ones of Sec. 3.2's packed
 * compare-and-swap word, and only the output is widened, so the triplets and
 * pairs equal mt_build_pairs' value for value.
 *
 * triplets (device) uint64[N][2] = (s, v), 16-byte aligned.
 * birth, death (device) uint64[capacity].  Every other argument, the
 * ownership, the errors and the single synchronization are those of
 * mt_build_pairs.
 */
int mt_build_pairs64(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind,
                     uint64_t *triplets, uint64_t *birth, uint64_t *death,
                     float *birth_val, float *death_val, int64_t capacity,
                     int64_t *n_pairs, int64_t *n_roots,
                     void *workspace, size_t ws_bytes, void *stream);

/*
 * mt_build_pairs_noalloc -- mt_build_pairs without a workspace argument, for
 * callers that cannot allocate device memory (code that must not call
 * hipMalloc, tight serving loops, harnesses that forbid allocation).  Not in
 * the paper.
 *
 * The call's scratch is a fixed array of MT_NOALLOC_SCRATCH_BYTES (64 MiB)
 * inside the library's device code, one per GPU, held from the library's
 * first use on that GPU until the process ends.  The call itself allocates
 * nothing: no hipMalloc, no hipFree, no allocating library routine.  Fields
 * whose workspace (mt_workspace_bytes) exceeds that size -- about 2.2 M
 * vertices of a 3-D field, e.g. 130^3; 128^3 needs 54 MiB -- are rejected
 * with MT_ERR_TOO_LARGE before anything is enqueued.
 *
 * Arguments, outputs, results and errors are those of mt_build_pairs (32-bit
 * ids); the triplets and pairs are identical to its.  The current HIP device
 * must be the device of `stream` and of every buffer.  Synchronizes `stream`
 * once, at the end.  Every call on one GPU uses that GPU's one array, which
 * keeps the last call's contents (each call clears what it needs cleared).
 * Calls that overlapped on one GPU would race on the array, so the library
 * serializes the calls of one process with a lock held until the call's
 * stream has synchronized.
 */
#define MT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mt_build_pairs_noalloc(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind,
                           uint32_t *triplets, uint32_t *birth, uint32_t *death,
                           float *birth_val, float *death_val, int64_t capacity,
                           int64_t *n_pairs, int64_t *n_roots, void *stream);

/* MT_NOALLOC_SCRATCH_BYTES, as compiled into the library. */
size_t mt_noalloc_scratch_bytes(void);

/*
 * mt_batch_build -- merge trees and pairs of many fields of uneven sizes in
 * one graph launch.  This batching is not in the paper; each field gets
 * exactly the triplets and pairs that mt_build + mt_persistence_pairs give it.
 *
 * fields    (device) the fields concatenated in order, float[sum N_i].
 * dims      (host) int64[n_fields][3] = (nx, ny, nz) per field.
 * triplets  (device) uint32[sum N_i][2], concatenated like `fields`; ids are
 *           local to their field.
 * birth, death, birth_val, death_val (device) [pair_capacity]: pairs of all
 *           fields concatenated in field order, each field's in ascending
 *           birth id, ids local to their field.
 * pair_offsets (device) int64[n_fields + 1]: pairs of field i occupy
 *           [pair_offsets[i], pair_offsets[i+1]); pair_offsets[n_fields] is
 *           the total (it may exceed pair_capacity: MT_ERR_CAPACITY is then
 *           latched and nothing past capacity is written).
 * workspace (device) mt_batch_workspace_bytes(dims, n_fields) bytes.
 * Asynchronous: the whole sequence is captured once per distinct argument
 * set into a hipGraph and replayed with one hipGraphLaunch on `stream`.
 * Read the latched status (and the total) with mt_sync_status.
 */
int mt_batch_build(const float *fields, const int64_t *dims, int32_t n_fields,
                   uint32_t *triplets, uint32_t *birth, uint32_t *death,
                   float *birth_val, float *death_val, int64_t pair_capacity,
                   int64_t *pair_offsets, void *workspace, size_t ws_bytes, void *stream);

/*
 * mt_batch_build_tree -- mt_batch_build for either tree (kind as in
 * mt_build_tree, the same for every field of the batch).  The kind is part of
 * the cached graph's key.
 */
int mt_batch_build_tree(const float *fields, const int64_t *dims, int32_t n_fields, int kind,
                        uint32_t *triplets, uint32_t *birth, uint32_t *death,
                        float *birth_val, float *death_val, int64_t pair_capacity,
                        int64_t *pair_offsets, void *workspace, size_t ws_bytes, void *stream);

/*
 * mt_vertex_ranks -- every vertex's position in the order of Sec. 2 (value,
 * then id; kind as in mt_build_tree: MT_TREE_SPLIT ranks -f): ranks[u] = the
 * number of vertices that precede u.  The first step of a rank-keyed build
 * (one global sort, after which every order test is an integer compare); it
 * is exported so that its cost can be measured against the value-keyed build.
 *
 * field (device) float[nx*ny*nz], read only.  ranks (device) uint32[N],
 * written.  workspace (device) at least mt_rank_workspace_bytes(nx, ny, nz)
 * bytes, 256-byte aligned (order keys, their sorted copy, sort scratch).
 * Steps on `stream`, asynchronous: order keys (value key << 32 | id), one
 * radix sort of the 64-bit keys, positions scattered back.
 * Errors: MT_ERR_INVALID_ARG, MT_ERR_TOO_LARGE, MT_ERR_WORKSPACE, MT_ERR_HIP
 * synchronously; MT_ERR_NAN latched (read it with mt_sync_status).
 */
int mt_vertex_ranks(const float *field, int64_t nx, int64_t ny, int64_t nz, int kind,
                    uint32_t *ranks, void *workspace, size_t ws_bytes, void *stream);

/* Bytes of device workspace mt_vertex_ranks needs; 0 if the dims are invalid. */
size_t mt_rank_workspace_bytes(int64_t nx, int64_t ny, int64_t nz);

/*
 * mt_sync_status -- synchronize `stream` and return the status latched in
 * `workspace` by the work enqueued before (MT_OK if none).  n_pairs and
 * n_roots (host, may be NULL) receive the totals of the last pairs readout
 * on that workspace.
 */
int mt_sync_status(const void *workspace, void *stream, int64_t *n_pairs, int64_t *n_roots);

/*
 * mt_build_stats -- synchronize `stream` and report, for the last build on
 * `workspace`, the number of tile-local minima the build kept a merge record
 * for and (if n_cross_facts is not NULL) the number of cross-tile merge facts
 * it queued after de-duplication (internal sizes, reported for measurement).
 */
int mt_build_stats(const void *workspace, void *stream, int64_t *n_local_minima, int64_t *n_cross_facts);

/*
 * mt_pairs_backward -- adjoint of the pair readout.  A pair's birth value is
 * f at its birth vertex and its death value is f at its death vertex, so for
 * upstream gradients gb, gd:  grad[birth_k] += gb_k,  grad[death_k] += gd_k.
 * (Not in the paper; it serves losses on persistence pairs, the use the
 * paper's introduction motivates.)
 *
 * dims (host) int64[n_fields][3]; pair_offsets (device) int64[n_fields + 1]
 * as written by mt_batch_build (for one field: {0, P}); birth, death (device)
 * uint32, field-local ids; grad_birth, grad_death (device) float, one per
 * pair; grad_field (device) float[sum N_i].  accumulate = 0 overwrites
 * grad_field with the result, 1 adds to it.  Birth vertices never repeat;
 * death vertices can (several branches may die at one saddle) and are summed
 * with float atomics, so the rounding order of such sums is not fixed.
 * Pairs whose two upstream gradients are zero are skipped, and so is either
 * update of zero (adding a zero changes no value, only possibly the sign of
 * a zero already there).
 * pair_capacity bounds the number of pairs read.  Asynchronous.
 */
int mt_pairs_backward(const int64_t *dims, int32_t n_fields, const int64_t *pair_offsets,
                      int64_t pair_capacity, const uint32_t *birth, const uint32_t *death,
                      const float *grad_birth, const float *grad_death, float *grad_field,
                      int accumulate, void *stream);

/*
 * Per-kernel timing with HIP events, for measurement.  mt_profile_begin
 * clears the counters and turns timing on: every kernel the library launches
 * afterwards (outside graph capture) is bracketed by two events on its launch
 * stream.  mt_profile_end waits for those events, accumulates the elapsed
 * time per kernel name and turns timing off.  mt_profile_get(i, ...) returns
 * the i-th kernel name (copied into name[name_len]), its summed time in ms
 * and its launch count; i runs over [0, mt_profile_count()).
 */
int mt_profile_begin(void);
int mt_profile_end(void);
int mt_profile_count(void);
int mt_profile_get(int i, char *name, size_t name_len, double *total_ms, int64_t *launches);

/*
 * Tile shapes and their autotuner.  The stencil passes cut every field into
 * tiles of one of a few compiled shapes, chosen per dims class (0: 3-D
 * fields, nz > 1; 1: 2-D, nz == 1 < ny; 2: 1-D).  The output never depends on
 * the shape; the speed does.
 *
 * mt_tile_shape_count / mt_tile_shape_info enumerate the compiled shapes
 * (tile extents, workgroup threads, dims class).  mt_set_tile_shape selects
 * shape `id` for its class (process-wide; later calls and newly captured
 * batch graphs use it); mt_get_tile_shape returns the current id.
 *
 * mt_autotune runs the build of the given batch (host dims, device fields as
 * for mt_batch_build) once per candidate shape of every class present,
 * `reps` timed repetitions each with HIP events on `stream`, checks that
 * every candidate writes bit-identical triplets (else MT_ERR_INTERNAL), and
 * selects the fastest shape per class.  triplets and triplets_check are two
 * device buffers of uint32[N][2]; workspace must hold
 * mt_autotune_workspace_bytes(dims, n_fields) bytes (candidates that need
 * more than ws_bytes are skipped).  best_ms (host, may be NULL) receives the
 * best time per class, -1 for classes not present.  Synchronizes.
 */
int mt_tile_shape_count(void);
int mt_tile_shape_info(int id, int *tx, int *ty, int *tz, int *threads, int *dims_class);
int mt_set_tile_shape(int dims_class, int id);
int mt_get_tile_shape(int dims_class);
size_t mt_autotune_workspace_bytes(const int64_t *dims, int32_t n_fields);
int mt_autotune(const float *fields, const int64_t *dims, int32_t n_fields, uint32_t *triplets,
                uint32_t *triplets_check, void *workspace, size_t ws_bytes, int reps, void *stream,
                double *best_ms);

/*
 * Launch schedule and its tuner.  Two settings change how the work is laid
 * onto the chip but never the output: the XCD-aware tile order (consecutive
 * tiles to one XCD, so neighbouring tiles share an L2; on by default) and
 * the workgroups per XCD of the fact scatter and the cross-tile merge (2048
 * by default).  Both are process-wide, read when a call plans its launches,
 * and part of the batch graph cache key.
 *
 * mt_set_schedule: xcd_remap 1 on, 0 off, -1 the default; merge_groups
 * 1..65536, 0 the default; anything else MT_ERR_INVALID_ARG.
 * mt_get_schedule writes the settings in force (either pointer may be NULL).
 * mt_autotune_schedule times the build of the given batch (arguments as for
 * mt_autotune; workspace of mt_batch_workspace_bytes(dims, n_fields) bytes)
 * under every pairing of remap {on, off} with merge_groups {256, 1024, 2048,
 * 8192}, with the current tile shapes, checks that every candidate writes
 * bit-identical triplets (else MT_ERR_INTERNAL), selects the fastest and
 * writes its time per build to *best_ms (host, may be NULL).  Synchronizes.
 */
int mt_set_schedule(int xcd_remap, int merge_groups);
int mt_get_schedule(int *xcd_remap, int *merge_groups);
int mt_autotune_schedule(const float *fields, const int64_t *dims, int32_t n_fields, uint32_t *triplets,
                         uint32_t *triplets_check, void *workspace, size_t ws_bytes, int reps, void *stream,
                         double *best_ms);

/*
 * Bounds of the build's loops, for tests of its failure handling and for
 * tuning.  Both settings are process-wide and are read when a call plans its
 * launches (a batch graph captured under one setting keeps it; the setting is
 * part of the graph cache key).
 *
 * mt_set_max_steps -- step cap of every merge, descent and chase loop
 * (Alg. 3, 4, 5 each loop until a condition holds; every kernel bounds them
 * so that a broken invariant cannot spin forever).  A loop that reaches the
 * cap stops and latches MT_ERR_LIVELOCK; the triplets are then invalid.
 * steps = 0 restores the default (2^24); 1 <= steps < 2^31 sets it; anything
 * else is MT_ERR_INVALID_ARG.  The default is never reached by a valid input:
 * a merge step moves strictly down a chain of at most N triplets.
 * mt_get_max_steps returns the cap in force.
 *
 * mt_set_table_probes -- probes each edge may spend in the LDS tables that
 * keep only the lowest edge between two basins (inside a tile, and across a
 * tile face) before it takes the path that needs no table: inside the tile
 * a short overflow list merged with the table's entries (and, should that
 * list fill up, every edge of the tile merged directly), across tiles queued
 * as it is.  All paths give the same triplets; the tables only save merges.  probes = -1 restores the default
 * (32, also the largest value); 0 <= probes <= 32 sets it (0 sends every
 * edge down the direct path); anything else is MT_ERR_INVALID_ARG.
 * mt_get_table_probes returns it.
 */
int mt_set_max_steps(int64_t steps);
int64_t mt_get_max_steps(void);
int mt_set_table_probes(int probes);
int mt_get_table_probes(void);

/*
 * Counting build, for measurement.  mt_set_counting(1) makes every later
 * call (and newly captured batch graph: the flag is part of its cache key)
 * launch the counting instantiation of the merge kernels, which tally events
 * per lane and add them to counters in the workspace head with one atomic per
 * wave; mt_set_counting(2) launches instead a tile pass that only clocks its
 * phases (counters 18-27; the per-lane event tallies would slow the phases
 * they time), with the timed instantiation of every other kernel;
 * mt_set_counting(0) (the default) goes back to the timed kernels, in which
 * every count is compiled out.  The triplets are the same in every mode.
 * mt_get_counting returns the mode; any other value is MT_ERR_INVALID_ARG.
 *
 * mt_read_counters synchronizes `stream` and copies the counters of the last
 * build on `workspace` into counts (host, uint64[n]); it returns how many it
 * wrote (at most 30; the rest of counts is zeroed) or an error.  In order:
 *   0 cross-tile merges started (one per queued fact)
 *   1 iterations of the cross-tile merge loop (Alg. 3)
 *   2 of those, descent steps
 *   3 64-bit compare-and-swaps on the minimum slots (Alg. 2)
 *   4 of those, failed
 *   5 displaced triplets merged again
 *   6 most iterations of a single cross-tile merge
 *   7 merges inside a tile (Alg. 3 in LDS)
 *   8 iterations of the in-tile merge loop
 *   9 64-bit LDS compare-and-swaps
 *  10 of those, failed
 *  11 most iterations of a single in-tile merge
 *  12 in-tile edges offered to the table of basin pairs
 *  13 table probes (one LDS atomic minimum each)
 *  14 in-tile edges that found no room in the table (they go to a short
 *     overflow list) or had no table (merged at once)
 *  15 chase steps of the output pass (Alg. 4 for every regular vertex)
 *  16 path compressions in long cross-tile descents (a link re-pointed past
 *     the next one when that one's saddle is not higher, one Repair step)
 *  17 chase steps of the minimum repair (Alg. 5 for every local minimum)
 *  18-27 (mode 2 only) shader clock cycles of the tile pass's phases,
 *     summed over tiles, each taken by the workgroup's first lane from one
 *     barrier to the next
 *     (so a phase includes the wait for its slowest wave): field loads
 *     awaited and order keys written; lowest lower neighbours; numbering of
 *     the local minima; descent chains to the local minima; field loads
 *     issued and the pair table cleared (from the workgroup's start, ahead
 *     of the first barrier); edges offered to the table; compaction of the
 *     table; the in-tile merges; repair of the local minima; minimum records
 *     and vertex labels
 *  28 tiles whose overflow list filled up, so that every edge of the tile
 *     was merged at once after the table's merges
 *  29 rounds of the output pass's chase loop, summed over waves and vertex
 *     groups (a wave's round issues the next step of all its lanes' chases;
 *     counter 15 over 256 times this is the share of chase slots in use)
 * Only a counting build writes them; after a timed build they read 0.
 */
int mt_set_counting(int on);
int mt_get_counting(void);
int mt_read_counters(const void *workspace, void *stream, uint64_t *counts, int n);

/*
 * mt_workspace_reset -- clear the status word and the counters at the head
 * of `workspace` (device, 256-byte aligned, ws_bytes long), asynchronously on
 * `stream`, with a kernel (no memset node, so it may be captured).  A workspace that did not
 * come out of a build holds arbitrary bytes, and mt_persistence_pairs keeps
 * the NaN and step-cap bits a build latched there so that it can report them;
 * call this once on such a workspace before mt_persistence_pairs.  The build
 * calls clear the head themselves.  Errors: MT_ERR_WORKSPACE (null,
 * misaligned, or shorter than the head, which every size returned by the
 * *_workspace_bytes calls exceeds), MT_ERR_HIP.
 */
int mt_workspace_reset(void *workspace, size_t ws_bytes, void *stream);

/* Free cached graph plans (device and host memory they hold).  Not safe to
 * call while another thread is inside the library. */
void mt_release_caches(void);

#ifdef __cplusplus
}
#endif

#endif /* MT_H */
