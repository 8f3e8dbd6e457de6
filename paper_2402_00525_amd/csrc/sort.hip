// Stable LSD radix sort of (uint64 key, uint32 value) pairs with 8-bit digits.
// Sorting the (tile << 32 | depth bits) keys of the duplication stage gives
// every tile a depth-ordered list (Sec. 2.1); stability keeps equal keys in
// Gaussian order, which fixes one order for forward and backward (Sec. 3.5).
//
// Each pass: per-block digit histograms, an exclusive scan of the
// digit-major histogram table, and a scatter in which every block ranks its
// keys stably (rounds in index order, wavefronts in order, lanes in order).
// The number of keys is read on the device, so the sort can be enqueued
// without knowing it on the host.
#include "gsr_internal.h"

namespace gsr {

namespace {

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ n_ptr, int shift,
                                                             uint32_t* __restrict__ hist, uint32_t nblocks) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = *n_ptr;
    const size_t base = (size_t)blockIdx.x * kSortTile;
    if (base < n) {
#pragma unroll 4
        for (int r = 0; r < kSortRounds; ++r) {
            const size_t i = base + (size_t)r * kSortThreads + threadIdx.x;
            if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1u);
        }
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint64_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout,
                                                                const uint32_t* __restrict__ n_ptr, int shift,
                                                                const uint32_t* __restrict__ hist,
                                                                uint32_t nblocks) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kSortThreads / 64][256];
    const int tid = threadIdx.x, wave = tid >> 6;
    run[tid] = hist[(size_t)tid * nblocks + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const uint32_t n = *n_ptr;
    const size_t base = (size_t)blockIdx.x * kSortTile;
    if (base >= n) return;
    const uint64_t lt = lanemask_lt();
    for (int r = 0; r < kSortRounds; ++r) {
        const size_t i = base + (size_t)r * kSortThreads + tid;
        const bool valid = i < n;
        const uint64_t key = valid ? kin[i] : 0ull;
        const uint32_t val = valid ? vin[i] : 0u;
        const uint32_t d = (uint32_t)(key >> shift) & 255u;
        // Lanes of this wavefront holding the same digit.
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            if (pos < n) {
                kout[pos] = key;
                vout[pos] = val;
            }
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortThreads / 64; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        run[tid] += add;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_sort_pairs(uint64_t* const keys[2], uint32_t* const vals[2], const uint32_t* n_ptr, size_t cap,
                             uint32_t* hist, uint32_t* partial, int bits, int start, int* result_buf, hipStream_t s,
                             void* const* scatter_events) {
    const size_t nb = sort_blocks(cap);
    const int passes = (bits + 7) / 8;
    int cur = start;
    hipError_t e = hipSuccess;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, s, (const uint64_t*)keys[cur], n_ptr,
                           shift, hist, (uint32_t)nb);
        e = launch_scan(hist, hist, nb * 256, partial, nullptr, 0xffffffffu, nullptr, s);
        if (e != hipSuccess) return e;
        if (scatter_events && (e = hipEventRecord((hipEvent_t)scatter_events[2 * p], s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, s, (const uint64_t*)keys[cur],
                           (const uint32_t*)vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_ptr, shift, (const uint32_t*)hist,
                           (uint32_t)nb);
        if (scatter_events && (e = hipEventRecord((hipEvent_t)scatter_events[2 * p + 1], s)) != hipSuccess) return e;
        cur ^= 1;
    }
    *result_buf = cur;
    return hipGetLastError();
}

hipError_t launch_sort(const FrameBufs& b, int bits, int* result_buf, hipStream_t s, void* const* scatter_events) {
    // Duplication writes into buffer (passes & 1) so that the result lands in buffer 0.
    const int passes = (bits + 7) / 8;
    return launch_sort_pairs(b.keys, b.vals, b.counters, b.capacity, b.hist, b.scan_partial, bits, passes & 1,
                             result_buf, s, scatter_events);
}

namespace {
__global__ void k_tile_cost_keys(const uint32_t* __restrict__ ranges, uint32_t n_tiles, uint64_t* __restrict__ keys,
                                 uint32_t* __restrict__ vals) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint32_t len = ranges[2 * (size_t)t + 1] - ranges[2 * (size_t)t];
    keys[t] = (uint64_t)(~len);
    vals[t] = t;
}
}  // namespace

hipError_t launch_tile_cost_keys(const uint32_t* ranges, uint32_t n_tiles, uint64_t* keys, uint32_t* vals,
                                 hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tile_cost_keys, dim3((n_tiles + 255) / 256), dim3(256), 0, s, ranges, n_tiles, keys, vals);
    return hipGetLastError();
}

}  // namespace gsr
