// Per-tile ordering of tile-grouped entries (Sec. 2.1 sort; Sec. 3.4 early
// termination).
//
// The renderer stops reading a tile's list once every pixel of the tile has
// terminated, so in dense scenes it reaches only the front of each list.  The
// entries are therefore grouped by tile only (a stable radix sort on the tile
// bits, which keeps Gaussian-id order inside a tile), and each tile's order
// by (depth bits, Gaussian id) -- the order a full sort of (tile, depth) keys
// with ties in id order gives -- is produced here in two steps:
//
//   k_tile_prefix        every tile: its range [start, end) in the grouped
//                        keys, and the first C <= M entries of that order,
//                        sorted in LDS;
//   k_tile_sort_flagged  tiles the renderer flagged because their pixels
//                        outlived the prefix: the whole list, sorted.
//
// Both write Gaussian ids to out[range start + j] and the length to len[tile].
#include <algorithm>

#include "gsr_internal.h"

namespace gsr {

namespace {

constexpr int kT = 256;              // threads per workgroup
constexpr int kTW = kT / 64;         // wavefronts per workgroup
constexpr int kPrefixBins = 4096;    // histogram bins of the prefix selection
constexpr int kBinsPerThread = kPrefixBins / kT;

// Fixed histogram bins over the order-preserving depth bits: bits 16..30 of
// (key - ord(2^-8)), i.e. 128 bins per octave of depth from 2^-8 to 2^24;
// nearer depths (and negative ones) fall into bin 0, farther ones into the
// last bin.  The map is monotone, so all entries of a bin follow all entries
// of earlier bins.
constexpr uint32_t kBinBase = 0xBB800000u;  // order-preserving bits of 2^-8
constexpr int kBinShift = 16;

__device__ __forceinline__ uint32_t depth_bin(uint32_t d) {
    if (d < kBinBase) return 0u;
    const uint32_t b = (d - kBinBase) >> kBinShift;
    return b < (uint32_t)(kPrefixBins - 1) ? b : (uint32_t)(kPrefixBins - 1);
}

__device__ __forceinline__ uint32_t depth_of(uint64_t key) { return (uint32_t)key; }

__device__ __forceinline__ uint32_t umin(uint32_t a, uint32_t b) { return a < b ? a : b; }
__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }

// Exclusive scan over the 256 threads of a workgroup.
__device__ __forceinline__ uint32_t wg_scan_excl(uint32_t v, uint32_t* lw, uint32_t& total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
    for (int w = 0; w < kTW; ++w) {
        const uint32_t s = lw[w];
        if (w < wave) before += s;
        tot += s;
    }
    total = tot;
    __syncthreads();  // lw may be reused right after
    return before + x - v;
}

// Minimum and maximum depth bits of keys[b, e), returned to every thread.
__device__ void depth_range(const uint64_t* __restrict__ keys, uint32_t b, uint32_t e, uint32_t* red, uint32_t& lo,
                            uint32_t& hi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t mn = 0xffffffffu, mx = 0u;
    uint32_t i = b + threadIdx.x;
    for (; i + 3 * kT < e; i += 4 * kT) {
        const uint32_t d0 = depth_of(keys[i]), d1 = depth_of(keys[i + kT]);
        const uint32_t d2 = depth_of(keys[i + 2 * kT]), d3 = depth_of(keys[i + 3 * kT]);
        mn = umin(mn, umin(umin(d0, d1), umin(d2, d3)));
        mx = umax(mx, umax(umax(d0, d1), umax(d2, d3)));
    }
    for (; i < e; i += kT) {
        const uint32_t d = depth_of(keys[i]);
        mn = umin(mn, d);
        mx = umax(mx, d);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = umin(mn, (uint32_t)__shfl_xor((int)mn, o));
        mx = umax(mx, (uint32_t)__shfl_xor((int)mx, o));
    }
    if (lane == 0) {
        red[wave] = mn;
        red[kTW + wave] = mx;
    }
    __syncthreads();
    lo = red[0];
    hi = red[kTW];
#pragma unroll
    for (int w = 1; w < kTW; ++w) {
        lo = umin(lo, red[w]);
        hi = umax(hi, red[kTW + w]);
    }
    __syncthreads();
}

// Ascending bitonic sort of sk[0, C) in LDS (padded with ~0 to a power of two
// that must fit the array).
__device__ void lds_bitonic(uint64_t* sk, uint32_t C) {
    uint32_t P = 1;
    while (P < C) P <<= 1;
    for (uint32_t j = C + threadIdx.x; j < P; j += kT) sk[j] = ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = threadIdx.x; t < P / 2; t += kT) {
                const uint32_t lo = 2 * t - (t & (stride - 1));
                const uint32_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = sk[lo], b = sk[hi];
                if ((a > b) == up) {
                    sk[lo] = b;
                    sk[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

// Wave-aggregated append: returns this lane's slot (valid lanes only).
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* counter) {
    const uint64_t m = __ballot(pred);
    const int lane = threadIdx.x & 63;
    const int leader = m ? __ffsll((long long)m) - 1 : 0;
    uint32_t base = 0;
    if (lane == leader && m) base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = (uint32_t)__shfl((int)base, leader);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    return base + (uint32_t)__popcll(m & lt);
}

// First positions in the tile-grouped keys[0, E) of tiles ta (threads
// 0..127) and tb (threads 128..255): each half narrows its interval 128-fold
// per round by probing 128 evenly spaced keys.  `cnt` holds 4 words.
__device__ void tile_starts(const uint64_t* __restrict__ keys, uint32_t E, uint32_t ta, uint32_t tb, uint32_t* cnt,
                            uint32_t& start_a, uint32_t& start_b) {
    const int tid = threadIdx.x, half = tid >> 7, k = tid & 127, wave = tid >> 6;
    const uint32_t target = half ? tb : ta;
    uint32_t lo = 0, hi = E;  // the answer lies in [lo, hi]; uniform over the half
    while (__syncthreads_or(hi > lo)) {
        const uint32_t span = hi - lo;
        const uint32_t step = span == 0u ? 0u : (span + 127u) / 128u;
        const uint64_t p = (uint64_t)lo + (uint64_t)k * step;
        const bool valid = span != 0u && p < hi;
        const bool below = valid && (uint32_t)(keys[p] >> 32) < target;
        const uint64_t m = __ballot(below);
        if ((tid & 63) == 0) cnt[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        const uint32_t c = cnt[2 * half] + cnt[2 * half + 1];
        __syncthreads();
        if (span != 0u) {
            const uint32_t nvalid = (span + step - 1u) / step;  // probes inside [lo, hi)
            const uint32_t nlo = c > 0u ? lo + (c - 1u) * step + 1u : lo;
            const uint32_t nhi = c < nvalid ? lo + c * step : hi;
            lo = nlo;
            hi = nhi;
        }
    }
    if (tid == 0) cnt[0] = lo;
    if (tid == 128) cnt[1] = lo;
    __syncthreads();
    start_a = cnt[0];
    start_b = cnt[1];
    __syncthreads();
}

// One workgroup per tile.  Finds the tile's range in the grouped keys (and
// writes it to ranges), then: a list of at most M entries is taken whole;
// a longer one gets a histogram of depth_bin over its entries, and C = the
// entries of the bins before the first bin at which the running count
// exceeds M (the C smallest keys).  The selected (depth << 32 | id) keys are
// sorted in LDS (dynamic, 8 * pow2ceil(M) bytes).
__global__ __launch_bounds__(kT) void k_tile_prefix(const uint64_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ vals,
                                                    const uint32_t* __restrict__ n_ptr, uint32_t n_tiles,
                                                    uint32_t* __restrict__ ranges, uint32_t* __restrict__ out,
                                                    uint32_t* __restrict__ len, uint32_t M) {
    extern __shared__ uint64_t sk[];
    __shared__ uint32_t hist[kPrefixBins];
    __shared__ uint32_t red[2 * kTW];
    __shared__ uint32_t s_fill, s_C, s_limit;
    const uint32_t tile = blockIdx.x;
    const int tid = threadIdx.x;
    if (tile >= n_tiles) return;
    uint32_t rb, re;
    tile_starts(keys, *n_ptr, tile, tile + 1u, red, rb, re);
    if (tid == 0) {  // an empty tile's range is written as [0, 0)
        ranges[2 * (size_t)tile] = re > rb ? rb : 0u;
        ranges[2 * (size_t)tile + 1] = re > rb ? re : 0u;
    }
    const uint32_t n = re - rb;
    if (n <= M) {
        for (uint32_t i = tid; i < n; i += kT) sk[i] = ((uint64_t)depth_of(keys[rb + i]) << 32) | vals[rb + i];
        __syncthreads();
        lds_bitonic(sk, n);
        for (uint32_t j = tid; j < n; j += kT) out[rb + j] = (uint32_t)sk[j];
        if (tid == 0) len[tile] = n;
        return;
    }
    for (int k = tid; k < kPrefixBins; k += kT) hist[k] = 0;
    if (tid == 0) s_fill = 0;
    __syncthreads();
    {
        uint32_t i = rb + tid;
        for (; i + 7 * kT < re; i += 8 * kT) {
            uint32_t d[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) d[u] = depth_of(keys[i + u * kT]);
#pragma unroll
            for (int u = 0; u < 8; ++u) atomicAdd(&hist[depth_bin(d[u])], 1u);
        }
        for (; i < re; i += kT) atomicAdd(&hist[depth_bin(depth_of(keys[i]))], 1u);
    }
    __syncthreads();
    // The first bin at which the running count exceeds M: each thread owns
    // kBinsPerThread consecutive bins; exactly one thread sees the crossing.
    {
        uint32_t h[kBinsPerThread], sum = 0;
#pragma unroll
        for (int k = 0; k < kBinsPerThread; ++k) {
            h[k] = hist[tid * kBinsPerThread + k];
            sum += h[k];
        }
        uint32_t total;
        uint32_t run = wg_scan_excl(sum, red, total);
#pragma unroll
        for (int k = 0; k < kBinsPerThread; ++k) {
            if (run <= M && run + h[k] > M) {
                s_C = run;
                s_limit = (uint32_t)(tid * kBinsPerThread + k);
            }
            run += h[k];
        }
    }
    __syncthreads();
    const uint32_t C = s_C, limit = s_limit;
    // Selection, eight keys per thread in flight (the order of appends does
    // not matter: the selected entries are sorted next).
    for (uint32_t i0 = rb; i0 < re; i0 += 8 * kT) {
        uint64_t k[8];
        uint32_t v[8];
        bool take[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = i0 + (uint32_t)u * kT + tid;
            k[u] = i < re ? keys[i] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = i0 + (uint32_t)u * kT + tid;
            take[u] = i < re && depth_bin(depth_of(k[u])) < limit;
            v[u] = take[u] ? vals[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t slot = wave_append(take[u], &s_fill);
            if (take[u]) sk[slot] = ((uint64_t)depth_of(k[u]) << 32) | v[u];
        }
    }
    __syncthreads();
    lds_bitonic(sk, C);
    for (uint32_t j = tid; j < C; j += kT) out[rb + j] = (uint32_t)sk[j];
    if (tid == 0) len[tile] = C;
}

// One stable LSD pass of a tile's list over 8 bits, from `shift`, of either
// (id - lo) (by_id) or (depth - lo): src/dst hold (depth << 32 | id) except in
// the first pass, which reads the grouped (tile << 32 | depth) keys and their
// ids.  Keys are taken in chunks of 256 in list order; inside a chunk a key's
// place among equal digits is its wavefront's ballot rank plus the counts of
// the wavefronts before it.
__device__ void tile_radix_pass(const uint64_t* __restrict__ src, const uint32_t* __restrict__ src_ids, bool first,
                                uint64_t* __restrict__ dst, uint32_t n, bool by_id, uint32_t lo, int shift,
                                uint32_t* hst, uint32_t* base, uint32_t (*wc)[256], uint32_t* lw) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    auto load = [&](uint32_t i) -> uint64_t {
        const uint64_t k = src[i];
        return first ? (((uint64_t)depth_of(k) << 32) | src_ids[i]) : k;
    };
    auto digit = [&](uint64_t x) -> uint32_t {
        const uint32_t v = by_id ? (uint32_t)x : (uint32_t)(x >> 32);
        return ((v - lo) >> shift) & 255u;
    };
    hst[tid] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kT) atomicAdd(&hst[digit(load(i))], 1u);
    __syncthreads();
    uint32_t total;
    base[tid] = wg_scan_excl(hst[tid], lw, total);
    __syncthreads();
    for (uint32_t c0 = 0; c0 < n; c0 += kT) {
        const uint32_t i = c0 + tid;
        const bool valid = i < n;
        const uint64_t x = valid ? load(i) : 0ull;
        const uint32_t dg = digit(x);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
#pragma unroll
        for (int w = 0; w < kTW; ++w) wc[w][tid] = 0;
        __syncthreads();
        if (valid && rank == 0) wc[wave][dg] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[dg] + rank;
            for (int w = 0; w < wave; ++w) pos += wc[w][dg];
            dst[pos] = x;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kTW; ++w) add += wc[w][tid];
        base[tid] += add;
        __syncthreads();
    }
}

// Minimum and maximum of the ids vals[b, e), returned to every thread.
__device__ void id_range(const uint32_t* __restrict__ vals, uint32_t b, uint32_t e, uint32_t* red, uint32_t& lo,
                         uint32_t& hi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t mn = 0xffffffffu, mx = 0u;
    for (uint32_t i = b + threadIdx.x; i < e; i += kT) {
        const uint32_t v = vals[i];
        mn = umin(mn, v);
        mx = umax(mx, v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = umin(mn, (uint32_t)__shfl_xor((int)mn, o));
        mx = umax(mx, (uint32_t)__shfl_xor((int)mx, o));
    }
    if (lane == 0) {
        red[wave] = mn;
        red[kTW + wave] = mx;
    }
    __syncthreads();
    lo = red[0];
    hi = red[kTW];
#pragma unroll
    for (int w = 1; w < kTW; ++w) {
        lo = umin(lo, red[w]);
        hi = umax(hi, red[kTW + w]);
    }
    __syncthreads();
}

__device__ __forceinline__ int bits_of(uint32_t span) {
    int b = 0;
    while (b < 32 && (span >> b) != 0u) ++b;
    return b;
}

// Grid-stride over tiles; a workgroup takes every tile flagged by the prefix
// render (flag = its entry count) and sorts its whole list by (depth, id): in
// LDS when it fits (lds_cap entries), else by stable 8-bit LSD passes over the
// bits that vary, ping-ponging between scratch (the tile's range of the other
// key buffer) and the grouped keys, which are no longer needed.  Counts flagged
// entries into counters[5] and tiles into counters[6]; appends flagged tiles
// to flist when given.
__global__ __launch_bounds__(kT) void k_tile_sort_flagged(uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                          uint64_t* __restrict__ scratch,
                                                          const uint32_t* __restrict__ ranges,
                                                          const uint32_t* __restrict__ flag, uint32_t n_tiles,
                                                          uint32_t* __restrict__ out, uint32_t* __restrict__ len,
                                                          uint32_t* __restrict__ counters, uint32_t* __restrict__ flist,
                                                          uint32_t lds_cap) {
    extern __shared__ uint64_t sk[];
    __shared__ uint32_t hst[256], base[256], wc[kTW][256], lw[kTW], red[2 * kTW];
    const int tid = threadIdx.x;
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const uint32_t n = flag[t];
        if (n == 0u) continue;
        if (tid == 0) {
            atomicAdd(counters + 5, n);
            const uint32_t slot = atomicAdd(counters + 6, 1u);
            if (flist) flist[slot] = t;
            len[t] = n;
        }
        const uint32_t rb = ranges[2 * (size_t)t];
        if (n <= lds_cap) {
            for (uint32_t i = tid; i < n; i += kT)
                sk[i] = ((uint64_t)depth_of(keys[rb + i]) << 32) | vals[rb + i];
            __syncthreads();
            lds_bitonic(sk, n);
            for (uint32_t j = tid; j < n; j += kT) out[rb + j] = (uint32_t)sk[j];
            __syncthreads();
            continue;
        }
        // Entries of a tile come in no particular order: sort by the whole
        // (depth, id) key, least significant part first.
        uint32_t dlo, dhi, ilo, ihi;
        depth_range(keys, rb, rb + n, red, dlo, dhi);
        id_range(vals, rb, rb + n, red, ilo, ihi);
        const int id_passes = (bits_of(ihi - ilo) + 7) / 8;
        const int passes = max(1, id_passes + (bits_of(dhi - dlo) + 7) / 8);  // at least one pass packs the ids
        uint64_t* a = keys + rb;
        uint64_t* b = scratch + rb;
        for (int p = 0; p < passes; ++p) {
            const bool by_id = p < id_passes;
            tile_radix_pass(a, vals + rb, p == 0, b, n, by_id, by_id ? ilo : dlo, 8 * (by_id ? p : p - id_passes), hst,
                            base, wc, lw);
            uint64_t* tmp = a;
            a = b;
            b = tmp;
        }
        for (uint32_t j = tid; j < n; j += kT) out[rb + j] = (uint32_t)a[j];
        __syncthreads();
    }
}

uint32_t pow2ceil(uint32_t x) {
    uint32_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

hipError_t launch_tile_prefix(const uint64_t* keys, const uint32_t* vals, const uint32_t* n_ptr, uint32_t n_tiles,
                              uint32_t* ranges, uint32_t* out, uint32_t* len, uint32_t M, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    const size_t shmem = 8 * (size_t)pow2ceil(std::max<uint32_t>(M, 1u));
    hipError_t e = hipFuncSetAttribute((const void*)k_tile_prefix, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(8 * kMaxPrefix));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_prefix, dim3(n_tiles), dim3(kT), shmem, s, keys, vals, n_ptr, n_tiles, ranges, out, len,
                       M);
    return hipGetLastError();
}

hipError_t launch_tile_sort_flagged(uint64_t* keys, const uint32_t* vals, uint64_t* scratch, const uint32_t* ranges,
                                    const uint32_t* flag, uint32_t n_tiles, uint32_t* out, uint32_t* len,
                                    uint32_t* counters, uint32_t* flist, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    const uint32_t lds_cap = kMaxPrefix;
    const unsigned grid = std::min<uint32_t>(n_tiles, 2048u);
    hipError_t e = hipFuncSetAttribute((const void*)k_tile_sort_flagged, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(8 * lds_cap));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_sort_flagged, dim3(grid), dim3(kT), 8 * (size_t)lds_cap, s, keys, vals, scratch, ranges,
                       flag, n_tiles, out, len, counters, flist, lds_cap);
    return hipGetLastError();
}

}  // namespace gsr
