// Stable LSD radix sort of (uint64 key, uint32 value) pairs with digits of up
// to 9 bits (45-bit frame keys take five passes).
// Sorting the (tile << 32 | depth bits) keys of the duplication stage gives
// every tile a depth-ordered list (Sec. 2.1); stability keeps equal keys in
// Gaussian order, which fixes one order for forward and backward (Sec. 3.5).
//
// Each pass: per-block digit histograms, an exclusive scan of the
// digit-major histogram table, and a scatter in which every block ranks its
// keys stably (rounds in index order, wavefronts in order, lanes in order).
// The number of keys is read on the device, so the sort can be enqueued
// without knowing it on the host.
#include <algorithm>

#include "gsr_internal.h"

namespace gsr {

namespace {

constexpr int kMaxDigitBits = 9;
constexpr int kMaxBins = 1 << kMaxDigitBits;
constexpr int kWaves = kSortThreads / 64;

// Digit histograms of one pass for kHistGroup consecutive sort tiles per
// workgroup (one wavefront per tile at a time), written digit-major as
// hist[digit * nblocks + tile]: each digit's counts of the group's tiles are
// one contiguous 64-byte run.
constexpr int kHistGroup = 16;

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ keys,
                                                             const uint32_t* __restrict__ n_ptr, int shift, int width,
                                                             uint32_t* __restrict__ hist, uint32_t nblocks) {
    __shared__ uint32_t h[kHistGroup][kMaxBins];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int bins = 1 << width;
    const uint32_t mask = (uint32_t)bins - 1u;
    for (int k = tid; k < kHistGroup * kMaxBins; k += kSortThreads) (&h[0][0])[k] = 0;
    __syncthreads();
    const uint32_t n = *n_ptr;
    const size_t tile0 = (size_t)blockIdx.x * kHistGroup;
    for (int j = wave; j < kHistGroup; j += kWaves) {
        const size_t base = (tile0 + j) * kSortTile;
        if (base >= n) break;
        for (int r = 0; r < kSortTile / 64; r += 8) {
            uint64_t k8[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const size_t i = base + (size_t)(r + u) * 64 + lane;
                k8[u] = i < n ? keys[i] : ~0ull;
            }
            // Keys with the digit of lane 0 are added as one count (runs of
            // equal digits would otherwise queue on one LDS address).
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool valid = k8[u] != ~0ull;
                const uint32_t d = (uint32_t)(k8[u] >> shift) & mask;
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
                const uint64_t same = __ballot(valid && d == d0);
                if (valid && d != d0) atomicAdd(&h[j][d], 1u);
                if (lane == 0 && same) atomicAdd(&h[j][d0], (uint32_t)__popcll(same));
            }
        }
    }
    __syncthreads();
    for (int v = tid; v < kHistGroup * bins; v += kSortThreads) {
        const int d = v / kHistGroup, j = v % kHistGroup;
        hist[(size_t)d * nblocks + tile0 + j] = h[j][d];
    }
}

template <int NW>
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* lw, uint32_t& total) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) lw[wave] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        const uint32_t sw = lw[w];
        if (w < wave) before += sw;
        tot += sw;
    }
    total = tot;
    return before + x - v;
}

// The scatter of a sort tile (8192 keys) runs 16 wavefronts of 8 rounds
// each, one workgroup per CU (132 KB of LDS): a digit's run in the output is
// twice as long as with 4096-key tiles, so fewer of the written lines are
// partial.
constexpr int kScatterWaves = 16;
constexpr int kScatterRounds = kSortTile / (64 * kScatterWaves);
constexpr int kScatterThreads = 64 * kScatterWaves;
static_assert(kScatterRounds * kScatterThreads == kSortTile, "scatter covers one sort tile");

// One stable counting pass over `width` key bits from `shift`.
//  1. Each wavefront ranks its 512 keys (8 rounds of 64, in index order):
//     lanes with equal digits are found by ballots over the digit bits, and
//     a per-wavefront running count per digit in LDS gives each key its rank
//     among equal digits -- no workgroup barrier inside the loop.
//  2. Per digit: offsets of the wavefronts, the block's local start
//     (exclusive scan over digits) and the distance to the global start.
//  3. Keys are placed in LDS in (digit, index) order, then written out so
//     that consecutive lanes write consecutive addresses of a digit's run.
__global__ __launch_bounds__(kScatterThreads) void k_radix_scatter(const uint64_t* __restrict__ kin,
                                                                const uint32_t* __restrict__ vin,
                                                                uint64_t* __restrict__ kout,
                                                                uint32_t* __restrict__ vout,
                                                                const uint32_t* __restrict__ n_ptr, int shift,
                                                                int width, const uint32_t* __restrict__ hist,
                                                                uint32_t nblocks) {
    __shared__ uint32_t cnt[kScatterWaves][kMaxBins];
    __shared__ uint32_t dstart[kMaxBins];
    __shared__ uint32_t gdelta[kMaxBins];
    __shared__ uint64_t sk[kSortTile];
    __shared__ uint32_t sv[kSortTile];
    __shared__ uint32_t lw[kScatterWaves];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int bins = 1 << width;
    const uint32_t mask = (uint32_t)bins - 1u;
    const uint32_t n = *n_ptr;
    const size_t base = (size_t)blockIdx.x * kSortTile;
    if (base >= n) return;
    for (int k = tid; k < kScatterWaves * kMaxBins; k += kScatterThreads) (&cnt[0][0])[k] = 0;
    __syncthreads();

    const uint64_t lt = lanemask_lt();
    uint64_t key[kScatterRounds];
    uint32_t val[kScatterRounds];
    uint32_t pos[kScatterRounds];
    // All loads first, so that they are in flight together.
#pragma unroll
    for (int r = 0; r < kScatterRounds; ++r) {
        const size_t i = base + (size_t)wave * (kScatterRounds * 64) + (size_t)r * 64 + lane;
        const bool valid = i < n;
        key[r] = valid ? kin[i] : 0ull;
        val[r] = valid ? vin[i] : 0u;
        pos[r] = valid ? 0u : 0xffffffffu;
    }
#pragma unroll
    for (int r = 0; r < kScatterRounds; ++r) {
        const bool valid = pos[r] == 0u;
        const uint32_t d = (uint32_t)(key[r] >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < width; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        const uint32_t c = valid ? cnt[wave][d] : 0u;
        pos[r] = valid ? c + rank : 0xffffffffu;
        wave_lds_sync();
        if (valid && rank == 0) cnt[wave][d] = c + (uint32_t)__popcll(peers);
        wave_lds_sync();
    }
    __syncthreads();
    // Wave offsets per digit (exclusive over wavefronts) and digit totals.
    uint32_t tot2[2] = {0u, 0u};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int d = 2 * tid + h;
        if (d < bins) {
            uint32_t acc = 0;
#pragma unroll
            for (int w = 0; w < kScatterWaves; ++w) {
                const uint32_t c = cnt[w][d];
                cnt[w][d] = acc;
                acc += c;
            }
            tot2[h] = acc;
        }
    }
    uint32_t total;
    const uint32_t ex = block_scan_excl<kScatterWaves>(tot2[0] + tot2[1], lw, total);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int d = 2 * tid + h;
        if (d < bins) {
            const uint32_t ls = ex + (h ? tot2[0] : 0u);
            dstart[d] = ls;
            gdelta[d] = hist[(size_t)d * nblocks + blockIdx.x] - ls;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kScatterRounds; ++r) {
        if (pos[r] != 0xffffffffu) {
            const uint32_t d = (uint32_t)(key[r] >> shift) & mask;
            const uint32_t lp = dstart[d] + cnt[wave][d] + pos[r];
            if (lp < (uint32_t)kSortTile) {
                sk[lp] = key[r];
                sv[lp] = val[r];
            }
        }
    }
    __syncthreads();
    const uint32_t cnt_tile = (n - base) < (size_t)kSortTile ? (uint32_t)(n - base) : (uint32_t)kSortTile;
#pragma unroll
    for (int r = 0; r < kScatterRounds; ++r) {
        const uint32_t idx = (uint32_t)r * kScatterThreads + tid;
        if (idx < cnt_tile) {
            const uint64_t k = sk[idx];
            const uint32_t d = (uint32_t)(k >> shift) & mask;
            const uint32_t g = gdelta[d] + idx;
            if (g < n) {
                kout[g] = k;
                vout[g] = sv[idx];
            }
        }
    }
}


}  // namespace

int sort_pass_count(int bits) { return (bits + kMaxDigitBits - 1) / kMaxDigitBits; }

hipError_t launch_sort_pairs(uint64_t* const keys[2], uint32_t* const vals[2], const uint32_t* n_ptr, size_t cap,
                             uint32_t* hist, uint32_t* partial, int bits, int start, int* result_buf, hipStream_t s,
                             void* const* scatter_events, int shift0) {
    const size_t nb = sort_blocks(cap);   // a multiple of kHistGroup
    const int passes = sort_pass_count(bits);
    const int width = (bits + passes - 1) / passes;
    int cur = start;
    hipError_t e = hipSuccess;
    for (int p = 0; p < passes; ++p) {
        const int shift = shift0 + width * p;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)(nb / kHistGroup)), dim3(kSortThreads), 0, s,
                           (const uint64_t*)keys[cur], n_ptr, shift, width, hist, (uint32_t)nb);
        e = launch_scan(hist, hist, nb * ((size_t)1 << width), partial, nullptr, 0xffffffffu, nullptr, s);
        if (e != hipSuccess) return e;
        if (scatter_events && (e = hipEventRecord((hipEvent_t)scatter_events[2 * p], s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nb), dim3(kScatterThreads), 0, s, (const uint64_t*)keys[cur],
                           (const uint32_t*)vals[cur], keys[cur ^ 1], vals[cur ^ 1], n_ptr, shift, width,
                           (const uint32_t*)hist, (uint32_t)nb);
        if (scatter_events && (e = hipEventRecord((hipEvent_t)scatter_events[2 * p + 1], s)) != hipSuccess) return e;
        cur ^= 1;
    }
    *result_buf = cur;
    return hipGetLastError();
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
