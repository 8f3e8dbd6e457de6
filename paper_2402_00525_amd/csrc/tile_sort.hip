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
//                        sorted in LDS (or, M = 0, a flag for the whole-list
//                        sort on every non-empty tile);
//   k_flag_chunks,       tiles the renderer flagged because their pixels
//   k_sort_chunks        outlived the prefix: the whole list, cut into
//                        chunks of depth bins and sorted chunk by chunk.
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
constexpr int kStashRounds = 2;      // rounds of 8 depths per thread kept in registers
constexpr uint32_t kStash = kStashRounds * 8 * kT;  // entries whose depths are kept

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
// writes it to ranges), then (M = 0) flags a non-empty tile for the whole-list
// sort, or: a list of at most M entries is taken whole;
// a longer one gets a histogram of depth_bin over its entries, and C = the
// entries of the bins before the first bin at which the running count
// exceeds M (the C smallest keys).  The selected (depth << 32 | id) keys are
// sorted in LDS (dynamic, 8 * pow2ceil(M) bytes).
__global__ __launch_bounds__(kT) void k_tile_prefix(const uint64_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ vals,
                                                    const uint32_t* __restrict__ n_ptr, uint32_t n_tiles,
                                                    uint32_t* __restrict__ ranges, uint32_t* __restrict__ out,
                                                    uint32_t* __restrict__ len, uint32_t* __restrict__ flag,
                                                    uint32_t M) {
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
    if (M == 0u) {  // whole lists: every non-empty tile goes to the chunked sort
        if (tid == 0) {
            len[tile] = 0u;
            if (n > 0u) flag[tile] = n;
        }
        return;
    }
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
    // The depths of the first kStash entries stay in registers for the
    // selection; the rest of a longer list is read again there.
    uint32_t st[kStashRounds][8];
#pragma unroll
    for (int s = 0; s < kStashRounds; ++s) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = rb + (uint32_t)(s * 8 + u) * kT + tid;
            st[s][u] = i < re ? depth_of(keys[i]) : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = rb + (uint32_t)(s * 8 + u) * kT + tid;
            if (i < re) atomicAdd(&hist[depth_bin(st[s][u])], 1u);
        }
    }
    {
        uint32_t i = rb + kStash + tid;
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
#pragma unroll
    for (int s = 0; s < kStashRounds; ++s) {
        bool take[8];
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t i = rb + (uint32_t)(s * 8 + u) * kT + tid;
            take[u] = i < re && depth_bin(st[s][u]) < limit;
            v[u] = take[u] ? vals[i] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const uint32_t slot = wave_append(take[u], &s_fill);
            if (take[u]) sk[slot] = ((uint64_t)st[s][u] << 32) | v[u];
        }
    }
    for (uint32_t i0 = rb + kStash; i0 < re; i0 += 8 * kT) {
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

// Minimum and maximum of the high and of the low words of the (depth << 32 |
// id) keys a[0, n), returned to every thread.
__device__ void word_ranges(const uint64_t* __restrict__ a, uint32_t n, uint32_t* red, uint32_t& dlo, uint32_t& dhi,
                            uint32_t& ilo, uint32_t& ihi) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t mn[2] = {0xffffffffu, 0xffffffffu}, mx[2] = {0u, 0u};
    for (uint32_t i = threadIdx.x; i < n; i += kT) {
        const uint64_t k = a[i];
        const uint32_t w[2] = {(uint32_t)(k >> 32), (uint32_t)k};
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            mn[h] = umin(mn[h], w[h]);
            mx[h] = umax(mx[h], w[h]);
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn[h] = umin(mn[h], (uint32_t)__shfl_xor((int)mn[h], o));
            mx[h] = umax(mx[h], (uint32_t)__shfl_xor((int)mx[h], o));
        }
    }
    __syncthreads();
    if (lane == 0) {
        red[wave] = mn[0];
        red[kTW + wave] = mx[0];
        red[2 * kTW + wave] = mn[1];
        red[3 * kTW + wave] = mx[1];
    }
    __syncthreads();
    dlo = red[0];
    dhi = red[kTW];
    ilo = red[2 * kTW];
    ihi = red[3 * kTW];
#pragma unroll
    for (int w = 1; w < kTW; ++w) {
        dlo = umin(dlo, red[w]);
        dhi = umax(dhi, red[kTW + w]);
        ilo = umin(ilo, red[2 * kTW + w]);
        ihi = umax(ihi, red[3 * kTW + w]);
    }
    __syncthreads();
}

__device__ __forceinline__ int bits_of(uint32_t span) {
    int b = 0;
    while (b < 32 && (span >> b) != 0u) ++b;
    return b;
}

// Exclusive maximum over the 256 threads of a workgroup (-1 before thread 0).
__device__ __forceinline__ int wg_max_excl(int v, uint32_t* lw) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x = max(x, y);
    }
    if (lane == 63) lw[wave] = (uint32_t)x;
    __syncthreads();
    int before = -1;
#pragma unroll
    for (int w = 0; w < kTW; ++w)
        if (w < wave) before = max(before, (int)lw[w]);
    const int up = __shfl_up(x, 1);
    __syncthreads();
    return lane > 0 ? max(before, up) : before;
}

// The whole-list fallback runs in two launches so that the sorting is spread
// over many workgroups:
//
//   k_flag_chunks  one workgroup per flagged tile (flag = its entry count):
//                  splits the tile's list into chunks of consecutive depth
//                  bins and writes every entry, as a (depth << 32 | id) key,
//                  into its chunk's range of the scratch buffer, at the
//                  entry's place in the tile's range; appends each chunk
//                  (first position, size) to the chunk list;
//   k_sort_chunks  grid-stride over the chunk list: sorts each chunk by
//                  (depth, id) and writes its ids to out at the same places.
//
// Bins are monotone in depth, so the chunks in bin order, each sorted, are
// the tile's list sorted.  A chunk gathers the bins whose first entry lies
// in the same block of kChunkHalf positions of the tile's bin order, so it
// holds fewer than kChunkHalf entries plus its last bin; one beyond
// kChunkEntries (a bin that large) is sorted by radix passes instead of in
// LDS.  A tile has at most n / kChunkHalf + 1 chunks.
constexpr uint32_t kChunkEntries = 4096;
constexpr uint32_t kChunkHalf = kChunkEntries / 2;

__global__ __launch_bounds__(kT) void k_flag_chunks(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals,
                                                    uint64_t* __restrict__ scratch, const uint32_t* __restrict__ ranges,
                                                    const uint32_t* __restrict__ flag, uint32_t n_tiles,
                                                    uint32_t* __restrict__ len, uint32_t* __restrict__ counters,
                                                    uint32_t* __restrict__ flist, uint2* __restrict__ chunks) {
    __shared__ uint32_t hist[kPrefixBins];   // bin counts, then chunk fill counts
    __shared__ uint32_t cstart[kPrefixBins];  // first position of each chunk in the tile
    __shared__ uint16_t cmap[kPrefixBins];    // chunk of each bin
    __shared__ uint32_t lw[kTW], s_base, s_nc;
    const int tid = threadIdx.x;
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const uint32_t n = flag[t];
        if (n == 0u) continue;
        const uint32_t rb = ranges[2 * (size_t)t];
        if (tid == 0) {
            atomicAdd(counters + 5, n);
            const uint32_t slot = atomicAdd(counters + 6, 1u);
            if (flist) flist[slot] = t;
            len[t] = n;
        }
        if (n <= kChunkEntries) {
#pragma unroll 4
            for (uint32_t i = tid; i < n; i += kT)
                scratch[rb + i] = ((uint64_t)depth_of(keys[rb + i]) << 32) | vals[rb + i];
            if (tid == 0) chunks[atomicAdd(counters + 7, 1u)] = make_uint2(rb, n);
            continue;
        }
        for (int k = tid; k < kPrefixBins; k += kT) hist[k] = 0;
        __syncthreads();
        {   // eight keys per thread in flight
            uint32_t i = rb + tid;
            for (; i + 7 * kT < rb + n; i += 8 * kT) {
                uint32_t d[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) d[u] = depth_of(keys[i + u * kT]);
#pragma unroll
                for (int u = 0; u < 8; ++u) atomicAdd(&hist[depth_bin(d[u])], 1u);
            }
            for (; i < rb + n; i += kT) atomicAdd(&hist[depth_bin(depth_of(keys[i]))], 1u);
        }
        __syncthreads();
        // Thread tid owns bins [16 tid, 16 tid + 16).  A non-empty bin b
        // belongs to block pre(b) / kChunkHalf (pre = entries of earlier
        // bins) and starts a chunk when the last non-empty bin before it
        // belongs to another block.
        uint32_t h[kBinsPerThread], sum = 0;
#pragma unroll
        for (int k = 0; k < kBinsPerThread; ++k) {
            h[k] = hist[tid * kBinsPerThread + k];
            sum += h[k];
        }
        uint32_t total;
        const uint32_t pre0 = wg_scan_excl(sum, lw, total);
        int last_block = -1;
        {
            uint32_t pre = pre0;
#pragma unroll
            for (int k = 0; k < kBinsPerThread; ++k) {
                if (h[k]) last_block = (int)(pre / kChunkHalf);
                pre += h[k];
            }
        }
        const int prev0 = wg_max_excl(last_block, lw);
        int prev = prev0;
        uint32_t starts = 0;
        {
            uint32_t pre = pre0;
#pragma unroll
            for (int k = 0; k < kBinsPerThread; ++k) {
                const int blk = (int)(pre / kChunkHalf);
                if (h[k] && blk != prev) ++starts;
                if (h[k]) prev = blk;
                pre += h[k];
            }
        }
        uint32_t nc;
        const uint32_t c0 = wg_scan_excl(starts, lw, nc);
        {
            // chunk of each bin, and each chunk's first position
            prev = prev0;
            uint32_t pre = pre0, c = c0;
#pragma unroll
            for (int k = 0; k < kBinsPerThread; ++k) {
                const int blk = (int)(pre / kChunkHalf);
                if (h[k] && blk != prev) {
                    cstart[c] = pre;
                    ++c;
                }
                if (h[k]) prev = blk;
                cmap[tid * kBinsPerThread + k] = (uint16_t)(c > 0u ? c - 1u : 0u);
                pre += h[k];
            }
        }
        if (tid == 0) {
            s_base = atomicAdd(counters + 7, nc);
            s_nc = nc;
        }
        __syncthreads();
        for (uint32_t c = tid; c < s_nc; c += kT) {
            const uint32_t e = c + 1u < s_nc ? cstart[c + 1] : n;
            chunks[s_base + c] = make_uint2(rb + cstart[c], e - cstart[c]);
            hist[c] = 0;  // fill counts
        }
        __syncthreads();
        {   // eight entries per thread in flight
            uint32_t i = rb + tid;
            for (; i + 7 * kT < rb + n; i += 8 * kT) {
                uint32_t d[8], v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    d[u] = depth_of(keys[i + u * kT]);
                    v[u] = vals[i + u * kT];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const uint32_t c = cmap[depth_bin(d[u])];
                    const uint32_t slot = atomicAdd(&hist[c], 1u);
                    scratch[rb + cstart[c] + slot] = ((uint64_t)d[u] << 32) | v[u];
                }
            }
            for (; i < rb + n; i += kT) {
                const uint32_t d = depth_of(keys[i]);
                const uint32_t c = cmap[depth_bin(d)];
                const uint32_t slot = atomicAdd(&hist[c], 1u);
                scratch[rb + cstart[c] + slot] = ((uint64_t)d << 32) | vals[i];
            }
        }
        __syncthreads();
    }
}

// One stable LSD pass over 8 bits, from `shift`, of (id - lo) (by_id) or
// (depth - lo) of the (depth << 32 | id) keys src[0, n) into dst.  Keys are
// taken in chunks of 256 in order; inside a chunk a key's place among equal
// digits is its wavefront's ballot rank plus the counts of the wavefronts
// before it.
__device__ void chunk_radix_pass(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst, uint32_t n, bool by_id,
                                 uint32_t lo, int shift, uint32_t* hst, uint32_t* base, uint32_t (*wc)[256],
                                 uint32_t* lw) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    auto digit = [&](uint64_t x) -> uint32_t {
        const uint32_t v = by_id ? (uint32_t)x : (uint32_t)(x >> 32);
        return ((v - lo) >> shift) & 255u;
    };
    hst[tid] = 0;
    __syncthreads();
    for (uint32_t i = tid; i < n; i += kT) atomicAdd(&hst[digit(src[i])], 1u);
    __syncthreads();
    uint32_t total;
    base[tid] = wg_scan_excl(hst[tid], lw, total);
    __syncthreads();
    for (uint32_t c0 = 0; c0 < n; c0 += kT) {
        const uint32_t i = c0 + tid;
        const bool valid = i < n;
        const uint64_t x = valid ? src[i] : 0ull;
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

// Grid-stride over the chunk list (counters[7] chunks): a chunk of at most
// kChunkEntries keys is sorted in LDS, a larger one by stable 8-bit LSD
// passes over the bits that vary (id bits first), ping-ponging between the
// scratch keys and the grouped keys at the same places (no longer needed).
__global__ __launch_bounds__(kT) void k_sort_chunks(uint64_t* __restrict__ keys, uint64_t* __restrict__ scratch,
                                                    const uint2* __restrict__ chunks,
                                                    const uint32_t* __restrict__ counters, uint32_t* __restrict__ out) {
    extern __shared__ uint64_t sk[];
    __shared__ uint32_t hst[256], base[256], wc[kTW][256], lw[4 * kTW];
    const int tid = threadIdx.x;
    const uint32_t nc = counters[7];
    for (uint32_t c = blockIdx.x; c < nc; c += gridDim.x) {
        const uint2 ch = chunks[c];
        const uint32_t pos = ch.x, n = ch.y;
        if (n <= kChunkEntries) {
#pragma unroll 4
            for (uint32_t i = tid; i < n; i += kT) sk[i] = scratch[pos + i];
            __syncthreads();
            lds_bitonic(sk, n);
            for (uint32_t j = tid; j < n; j += kT) out[pos + j] = (uint32_t)sk[j];
            __syncthreads();
            continue;
        }
        uint32_t dlo, dhi, ilo, ihi;
        word_ranges(scratch + pos, n, lw, dlo, dhi, ilo, ihi);
        const int id_passes = (bits_of(ihi - ilo) + 7) / 8;
        const int passes = id_passes + (bits_of(dhi - dlo) + 7) / 8;
        uint64_t* a = scratch + pos;
        uint64_t* b = keys + pos;
        for (int p = 0; p < passes; ++p) {
            const bool by_id = p < id_passes;
            chunk_radix_pass(a, b, n, by_id, by_id ? ilo : dlo, 8 * (by_id ? p : p - id_passes), hst, base, wc, lw);
            uint64_t* tmp = a;
            a = b;
            b = tmp;
        }
        for (uint32_t j = tid; j < n; j += kT) out[pos + j] = (uint32_t)a[j];
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
                              uint32_t* ranges, uint32_t* out, uint32_t* len, uint32_t* flag, uint32_t M,
                              hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    const size_t shmem = 8 * (size_t)pow2ceil(std::max<uint32_t>(M, 1u));
    hipError_t e = hipFuncSetAttribute((const void*)k_tile_prefix, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(8 * kMaxPrefix));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_prefix, dim3(n_tiles), dim3(kT), shmem, s, keys, vals, n_ptr, n_tiles, ranges, out, len,
                       flag, M);
    return hipGetLastError();
}

hipError_t launch_tile_sort_flagged(uint64_t* keys, const uint32_t* vals, uint64_t* scratch, const uint32_t* ranges,
                                    const uint32_t* flag, uint32_t n_tiles, uint32_t* out, uint32_t* len,
                                    uint32_t* counters, uint32_t* flist, uint2* chunks, hipStream_t s) {
    if (n_tiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_flag_chunks, dim3(std::min<uint32_t>(n_tiles, 2048u)), dim3(kT), 0, s, keys, vals, scratch,
                       ranges, flag, n_tiles, len, counters, flist, chunks);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int lds = 8 * (int)kChunkEntries;
    e = hipFuncSetAttribute((const void*)k_sort_chunks, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_chunks, dim3(1024), dim3(kT), (size_t)lds, s, keys, scratch, (const uint2*)chunks,
                       (const uint32_t*)counters, out);
    return hipGetLastError();
}

size_t flagged_chunk_capacity(size_t entries, size_t tiles) { return entries / kChunkHalf + tiles + 1; }

}  // namespace gsr
