// Internal launch interface shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gsr_device.h"

namespace gsr {

enum { kModeGlobal = 0, kModeHier = 1 };
// Ablations of the hierarchical mode (bits of gsr_config.flags).
enum { kAblateTileDepth = 1, kAblateTileCull = 2, kAblateHierCull = 4, kTileCentreDepth = 8 };
// lb_threshold at or above this: no load balancing (every lane walks its own
// Gaussian's rectangle).
constexpr int kNoLoadBalance = 1 << 30;

// Device regions of one frame inside the caller's workspace.
struct FrameBufs {
    float4* pk;       // 4 float4 per Gaussian: the splat as the renderer reads it
    float4* col;      // colour (r, g, b) and |mu - o|
    float2* zd;       // view depth, |mu - o|
    int4* rect;       // tile rectangle, inclusive
    uint32_t* touched;
    uint64_t* kmask;          // kept-tile bit mask of lane-handled Gaussians
    uint32_t* offsets;
    uint32_t* dhist;          // grouped duplication counts, kDupBins x workgroups
    uint32_t* scan_partial;   // scan scratch, >= scan_partial_len(max(n, hist)) + 2
    uint64_t* keys[2];
    uint32_t* vals[2];
    uint32_t* hist;           // radix histograms, kSortMaxBins x sort blocks
    uint32_t* ranges;         // [tiles][2]
    uint32_t* counters;       // [0] entries, [1] consumed, [3] entries needed, [5] / [6] fallback entries /
                              // tiles, [7] fallback chunks, [8..11] the frame's fingerprint (checked by
                              // the backward)
    uint32_t capacity;
    uint32_t* pre_vals;       // [capacity] sorted prefix ids at each tile's range begin
    uint32_t* pre_len;        // [tiles]
    uint32_t* tile_flag;      // [tiles] entry count of a tile rendered from the fallback, else 0
    uint32_t* flist;          // [tiles] flagged tiles (batch)
    uint2* chunks;            // chunk list of the fallback sort
};

struct SceneArgs {
    int n, deg;
    const float* means;
    const float* scales;
    const float* rots;
    const float* opac;
    const float* sh;
};

// Scan tiles
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Radix sort tiles
constexpr int kSortThreads = 256;
constexpr int kSortRounds = 32;
constexpr int kSortTile = kSortThreads * kSortRounds;

inline size_t div_up(size_t a, size_t b) { return (a + b - 1) / b; }
inline size_t scan_partial_len(size_t n) { return div_up(n, kScanTile); }
// Sort tiles for `cap` keys, rounded up to whole histogram groups of 16.
inline size_t sort_blocks(size_t cap) { return div_up(div_up(cap, kSortTile), 16) * 16; }
// Radix passes for `bits` key bits (digits of at most 9 bits, equal widths).
int sort_pass_count(int bits);
constexpr int kSortMaxBins = 512;

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s);
// Grouped duplication (hierarchical lists): entries are written straight
// into buckets of the low kDupDigitBits bits of their tile id.  Preprocessing
// counts each workgroup's kept tiles per bucket into hist[d * stride + wg_base
// + workgroup]; after an exclusive scan of hist (digit-major, so buckets are in
// digit order), duplication places every entry at its bucket's next slot.
// Inside a bucket the order is unspecified; only the tile grouping is used.
constexpr int kDupDigitBits = 5;
constexpr int kDupBins = 1 << kDupDigitBits;
struct DupGroups {
    uint32_t* hist;
    uint32_t stride;     // workgroups of the whole batch
    uint32_t wg_base;    // first workgroup of this launch
    uint32_t tile_base;  // first tile of this view
};
hipError_t launch_preprocess(const SceneArgs& sc, const DevCam& cam, int mode, int lb, int flags, const FrameBufs& b,
                             hipStream_t s, const DupGroups* groups = nullptr);
// Exclusive scan of n uint32 values; the total (clamped to `clamp`) goes to
// *total, and `status` gets the overflow bit if the total exceeds `clamp`;
// raw_total (optional) receives the unclamped total, saturated at 2^32 - 1.
hipError_t launch_scan(const uint32_t* in, uint32_t* out, size_t n, uint32_t* partial, uint32_t* total,
                       uint32_t clamp, int32_t* status, hipStream_t s, uint32_t* raw_total = nullptr);
// Writes the unsorted entries into key/value buffer `buf`; tile ids are
// offset by tile_base and Gaussian ids by id_base (zero for one view).
hipError_t launch_duplicate(int n, const DevCam& cam, int mode, int lb, int flags, const FrameBufs& b, int buf,
                            int32_t* status, hipStream_t s, uint32_t tile_base = 0, uint32_t id_base = 0,
                            const DupGroups* groups = nullptr);
// Stable LSD sort of the first *n_ptr pairs of (keys[start], vals[start]) on
// the low `bits` key bits, for at most `cap` pairs; the result lands in
// buffer start ^ (passes & 1), returned in *result_buf.  hist holds
// kSortMaxBins * sort_blocks(cap) words, partial
// scan_partial_len(kSortMaxBins * sort_blocks(cap)) + 2.
hipError_t launch_sort_pairs(uint64_t* const keys[2], uint32_t* const vals[2], const uint32_t* n_ptr, size_t cap,
                             uint32_t* hist, uint32_t* partial, int bits, int start, int* result_buf, hipStream_t s,
                             void* const* scatter_events = nullptr, int shift0 = 0);
// Largest supported sorted prefix per tile (LDS of k_tile_prefix).
constexpr int kMaxPrefix = 16384;  // entries a workgroup sorts in LDS (128 KiB of keys)
// Per tile of the tile-grouped keys[0, *n_ptr): its range [start, end) into
// ranges, and its sorted prefix -- the C <= M entries of smallest (depth, id)
// -- as ids at out[start + j], len[tile] = C (C = all entries when the tile
// has at most M).  M <= kMaxPrefix.  M = 0 sorts nothing here: every
// non-empty tile gets flag[tile] = its entry count, for the whole-list sort.
hipError_t launch_tile_prefix(const uint64_t* keys, const uint32_t* vals, const uint32_t* n_ptr, uint32_t n_tiles,
                              uint32_t* ranges, uint32_t* out, uint32_t* len, uint32_t* flag, uint32_t M,
                              hipStream_t s);
// Whole sorted list of every flagged tile (flag[t] = its entry count) at
// out[range begin ..], len[t] = count; `scratch` is a second key buffer of the
// same capacity and the grouped keys are overwritten.  The lists are split
// into chunks of consecutive depth bins, listed in `chunks` (room for
// flagged_chunk_capacity(capacity, n_tiles) entries, counted in counters[7],
// which must be 0 on entry) and sorted by many workgroups.  counters[5] +=
// flagged entries, counters[6] += flagged tiles; flagged tiles appended to
// flist if given.
hipError_t launch_tile_sort_flagged(uint64_t* keys, const uint32_t* vals, uint64_t* scratch, const uint32_t* ranges,
                                    const uint32_t* flag, uint32_t n_tiles, uint32_t* out, uint32_t* len,
                                    uint32_t* counters, uint32_t* flist, uint2* chunks, hipStream_t s);
size_t flagged_chunk_capacity(size_t entries, size_t tiles);
// Cost keys for ordering tiles: key[t] = ~(list length of tile t), val[t] = t.
hipError_t launch_tile_cost_keys(const uint32_t* ranges, uint32_t n_tiles, uint64_t* keys, uint32_t* vals,
                                 hipStream_t s);

struct RenderArgs {
    DevCam cam;
    uint32_t n;   // number of Gaussians (ids are checked against it)
    const float4* pk;
    const float4* col;
    const float2* zd;
    const uint32_t* vals;
    const uint32_t* ranges;
    uint32_t* counters;
    float* rgb;
    float* depth;
    int32_t* count;
    float* T;
    int32_t* blend_ids;
    int max_k;
    float* delta;  // debug renders: each pixel's sort error (Sec. 3.3) [H,W], or null
    float bg0, bg1, bg2;
    // backward only (grad2d != nullptr): dL/d rgb [3,H,W], the forward image and
    // transmittance, and the per-Gaussian 2D gradients [N][9] =
    // (mean x, mean y, conic a, b, c, opacity, r, g, b) accumulated atomically.
    const float* dL;
    const float* rgb_in;
    const float* T_in;
    float* grad2d;
    // Which list a tile is rendered from (list_mode):
    //   kListFull     vals + ranges (fully sorted entries)
    //   kListPrefix   the tile's sorted prefix pre_vals[range begin ..], pre_len[tile];
    //                 a tile whose pixels outlive a truncated prefix gets
    //                 tile_flag[tile] = its entry count
    //   kListFlagged  only flagged tiles, from pre_vals (now their whole list)
    //   kListSorted   every tile from pre_vals / pre_len (after the fallback)
    int list_mode;
    const uint32_t* pre_vals;
    const uint32_t* pre_len;
    uint32_t* tile_flag;
    int flags;  // kAblateHierCull: no culling at the 4x4 and 2x2 levels
    // The hierarchical forward loads every splat a level reads ahead (for
    // views of few, deep tiles, where nothing else hides a wavefront's
    // memory latency; more registers per lane).
    bool deep;
    unsigned long long* work;  // if set: the hierarchical render counts its evaluations (head 4 only)
    // backward only: the fingerprint the forward left in the workspace (fp,
    // kFingerprintWords words) and the one this call expects; on a mismatch
    // the backward render adds nothing and sets kStatusMismatch in *status
    const uint32_t* fp;
    uint32_t fp_expect[4];
    int32_t* status;
};
constexpr int kFingerprintWords = 4;
constexpr int kFingerprintOffset = 8;   // counters[8..11] of a frame's workspace
constexpr int32_t kStatusMismatch = 2;
enum { kListFull = 0, kListPrefix = 1, kListFlagged = 2, kListSorted = 3 };

// Per-view descriptor of a batch, in device memory.
struct ViewDev {
    DevCam cam;
    float* rgb;
    float* depth;
    int32_t* count;
    float* T;
    uint32_t tile_base;  // first global tile id of this view
    uint32_t rec_base;   // first record of this view
};

// Work queues of the batched render: tile slot s of the work order goes to
// queue s % kBatchQueues, the queue of the XCD that runs workgroups b with
// b % kBatchQueues == s % kBatchQueues.
constexpr int kBatchQueues = 8;

struct BatchArgs {
    const ViewDev* views;
    int n_views;
    uint32_t n_records;
    const float4* pk;
    const float4* col;
    const float2* zd;
    const uint32_t* vals;
    const uint32_t* ranges;   // per global tile
    const uint32_t* order;    // global tiles in work order (nullptr: natural order)
    int list_mode;            // as RenderArgs::list_mode
    const uint32_t* pre_vals;
    const uint32_t* pre_len;
    uint32_t* tile_flag;
    int flags;                // as RenderArgs::flags
    uint32_t* queue;          // kBatchQueues work-queue heads (one per XCD), zero before the launch
    uint32_t n_tiles;         // tiles listed in `order` (4 strips each)
    const uint32_t* n_tiles_dev;  // if set, the number of tiles is read here instead
    float bg0, bg1, bg2;
};

hipError_t launch_render_global(const RenderArgs& a, hipStream_t s);
// Full per-pixel sort over the tile-grouped (exactly culled) lists.
hipError_t launch_render_full(const RenderArgs& a, hipStream_t s);
// Per-ray resorting window of `head` samples over the global order's lists.
hipError_t launch_render_window(const RenderArgs& a, int head, hipStream_t s);
hipError_t launch_render_hier_batch(const BatchArgs& b, int head, unsigned grid, hipStream_t s);
bool hier_head_supported(int head);
// Hierarchical render with head capacity `head` (1..24).
hipError_t launch_render_hier(const RenderArgs& a, int head, hipStream_t s);

// Per-Gaussian chain from the 2D gradients to the parameters.
hipError_t launch_preprocess_backward(const SceneArgs& sc, const DevCam& cam, const float4* pk, const float* grad2d,
                                      float* dmeans, float* dscales, float* drots, float* dopac, float* dsh,
                                      hipStream_t s);

hipError_t launch_probe_math(const float* a, const float* b, int n, float* out, hipStream_t s);

}  // namespace gsr
