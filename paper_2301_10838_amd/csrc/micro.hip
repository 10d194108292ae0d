// micro.hip -- measurement kernels for the ceilings the merge-tree kernels are
// set against (libmt_micro.so, gfx950).  Nothing here is part of the merge
// tree path: these give the reference rates for the figures the benchmark
// reports beside it.
//
//   mtm_copy       streaming copy, 16-byte loads and stores (the HBM ceiling
//                  a sweep can reach)
//   mtm_cas        returning 64-bit compare-and-swap on global memory at
//                  hashed addresses over an array of n words: spread over a
//                  large array it is the uncontended rate, over a few words
//                  the contended one (the merge's swaps land between)
//   mtm_lds_cas    returning 64-bit compare-and-swap on LDS at hashed
//                  addresses of a 32 KiB table per workgroup (the tile pass)
//   mtm_chase      dependent loads along a random cycle (the chases of the
//                  repair and the merge): latency per step and loads per
//                  second at a given number of concurrent chains
//
// Every entry point checks its sizes on the host, launches, and times the
// launches with HIP events on `stream`; it synchronizes before returning the
// average milliseconds per launch.  The kernels' loops are bounded by their
// arguments; addresses are reduced modulo the array sizes the caller passes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace {

constexpr int kT = 256;

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    // splitmix64 finaliser: a counter-based hash, so no lane waits on another
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ __launch_bounds__(kT) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kT;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(kT) void k_cas(uint64_t *__restrict__ a, uint64_t n, int per_lane, uint64_t seed,
                                            uint64_t *__restrict__ sink)
{
    const uint64_t lane = (uint64_t)blockIdx.x * kT + threadIdx.x;
    uint64_t acc = 0;
    for (int i = 0; i < per_lane; ++i) {
        const uint64_t h = mix64(seed ^ (lane * 0x100000001B3ull + (uint64_t)i));
        uint64_t expect = h >> 20;
        __hip_atomic_compare_exchange_strong(a + (h % n), &expect, h, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        acc ^= expect;  // the returned word, so every swap is kept
    }
    if (acc == 0x5A5A5A5A5A5A5A5Aull) sink[0] = acc;  // practically never; keeps acc live
}

__global__ __launch_bounds__(kT) void k_lds_cas(int per_lane, uint64_t seed, uint64_t *__restrict__ sink)
{
    constexpr int W = 4096;  // 32 KiB of 64-bit words
    __shared__ uint64_t t[W];
    for (int i = threadIdx.x; i < W; i += kT) t[i] = 0;
    __syncthreads();
    const uint64_t lane = (uint64_t)blockIdx.x * kT + threadIdx.x;
    uint64_t acc = 0;
    for (int i = 0; i < per_lane; ++i) {
        const uint64_t h = mix64(seed ^ (lane * 0x100000001B3ull + (uint64_t)i));
        uint64_t expect = h >> 20;
        __hip_atomic_compare_exchange_strong(t + (h & (W - 1)), &expect, h, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP);
        acc ^= expect;
    }
    if (acc == 0x5A5A5A5A5A5A5A5Aull) sink[0] = acc;
}

__global__ __launch_bounds__(kT) void k_chase(const uint32_t *__restrict__ next, uint32_t n, int steps,
                                              int64_t chains, uint32_t *__restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (c >= chains) return;
    uint32_t x = (uint32_t)(((uint64_t)c * 2654435761u) % n);
    for (int i = 0; i < steps; ++i) x = next[x] < n ? next[x] : 0u;
    out[c] = x;
}

template <class L>
int timed(L &&launch, int reps, hipStream_t st, double *ms)
{
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -7;
    launch();  // warm-up
    int rc = 0;
    if (hipEventRecord(a, st) != hipSuccess) rc = -7;
    for (int r = 0; r < reps && rc == 0; ++r) launch();
    if (rc == 0 && hipGetLastError() != hipSuccess) rc = -7;
    if (rc == 0 && (hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess)) rc = -7;
    float t = 0.f;
    if (rc == 0 && hipEventElapsedTime(&t, a, b) != hipSuccess) rc = -7;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc == 0 && ms) *ms = (double)t / reps;
    return rc;
}

}  // namespace

extern "C" {

// Copy `bytes` (a multiple of 16, both pointers 16-byte aligned, device) from
// src to dst, `reps` times.  Returns 0, -1 on bad arguments, -7 on a HIP error.
int mtm_copy(const void *src, void *dst, int64_t bytes, int reps, void *stream, double *ms)
{
    if (!src || !dst || bytes <= 0 || (bytes & 15) || (((uintptr_t)src | (uintptr_t)dst) & 15) || reps < 1)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    const int64_t n = bytes / 16;
    const unsigned grid = (unsigned)std::min<int64_t>(8 * 256 * 8, (n + kT - 1) / kT);
    return timed([&] { hipLaunchKernelGGL(k_copy, dim3(grid), dim3(kT), 0, st, (const uint4 *)src, (uint4 *)dst, n); },
                 reps, st, ms);
}

// `lanes` lanes (a multiple of 256) each issue `per_lane` returning 64-bit
// compare-and-swaps at hashed word indices in [0, n_words) of `a` (device,
// 8-byte aligned, n_words >= 1 words); sink (device) is one spare word.
int mtm_cas(uint64_t *a, int64_t n_words, int64_t lanes, int per_lane, int reps, void *stream, uint64_t *sink,
            double *ms)
{
    if (!a || !sink || n_words < 1 || lanes < kT || (lanes % kT) || lanes > (1LL << 26) || per_lane < 1 ||
        reps < 1 || ((uintptr_t)a & 7))
        return -1;
    hipStream_t st = (hipStream_t)stream;
    uint64_t seed = 1;
    return timed([&] {
        hipLaunchKernelGGL(k_cas, dim3((unsigned)(lanes / kT)), dim3(kT), 0, st, a, (uint64_t)n_words, per_lane,
                           seed++, sink);
    }, reps, st, ms);
}

// `blocks` workgroups of 256 lanes, each lane `per_lane` LDS compare-and-swaps
// in a 32 KiB table of its workgroup.
int mtm_lds_cas(int64_t blocks, int per_lane, int reps, void *stream, uint64_t *sink, double *ms)
{
    if (!sink || blocks < 1 || blocks > (1 << 20) || per_lane < 1 || reps < 1) return -1;
    hipStream_t st = (hipStream_t)stream;
    uint64_t seed = 1;
    return timed([&] {
        hipLaunchKernelGGL(k_lds_cas, dim3((unsigned)blocks), dim3(kT), 0, st, per_lane, seed++, sink);
    }, reps, st, ms);
}

// `chains` independent chains, each `steps` dependent loads x = next[x] over
// next[0 .. n) (device uint32, a permutation; an entry >= n restarts at 0);
// out (device) receives each chain's last index (uint32[chains]).
int mtm_chase(const uint32_t *next, int64_t n, int steps, int64_t chains, int reps, void *stream, uint32_t *out,
              double *ms)
{
    if (!next || !out || n < 1 || n > 0xffffffffLL || steps < 1 || chains < 1 || chains > (1LL << 26) || reps < 1)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    const unsigned grid = (unsigned)((chains + kT - 1) / kT);
    return timed([&] {
        hipLaunchKernelGGL(k_chase, dim3(grid), dim3(kT), 0, st, next, (uint32_t)n, steps, chains, out);
    }, reps, st, ms);
}

}  // extern "C"
