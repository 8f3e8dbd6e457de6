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

hipError_t launch_sort(const FrameBufs& b, int bits, int* result_buf, hipStream_t s, void* const* scatter_events) {
    const size_t nb = sort_blocks(b.capacity);
    const int passes = (bits + 7) / 8;
    // Duplication writes into buffer (passes & 1) so that the result lands in buffer 0.
    int cur = passes & 1;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, s, (const uint64_t*)b.keys[cur],
                           (const uint32_t*)b.counters, shift, b.hist, (uint32_t)nb);
        hipError_t e = launch_scan(b.hist, b.hist, nb * 256, b.scan_partial, nullptr, 0xffffffffu, nullptr, s);
        if (e != hipSuccess) return e;
        if (scatter_events && (e = hipEventRecord((hipEvent_t)scatter_events[2 * p], s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, s, (const uint64_t*)b.keys[cur],
                           (const uint32_t*)b.vals[cur], b.keys[cur ^ 1], b.vals[cur ^ 1], (const uint32_t*)b.counters,
                           shift, (const uint32_t*)b.hist, (uint32_t)nb);
        if (scatter_events && (e = hipEventRecord((hipEvent_t)scatter_events[2 * p + 1], s)) != hipSuccess) return e;
        cur ^= 1;
    }
    *result_buf = cur;
    return hipGetLastError();
}

}  // namespace gsr
