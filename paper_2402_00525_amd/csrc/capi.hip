// Host side of the C ABI: argument validation, workspace layout and the
// stream-ordered launch sequence of a frame.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/gsr.h"
#include "gsr_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* msg) {
    g_last_error = msg;
    return code;
}

int fail_hip(hipError_t e, const char* where) {
    g_last_error = std::string(where) + ": " + hipGetErrorString(e);
    return GSR_EDEVICE;
}

inline int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

int bits_for_tiles(int tiles) {
    int b = 0;
    while ((1 << b) < tiles) ++b;
    return b;
}

// Radix passes of the sort stage and the buffer duplication writes into.
// HIER: duplication already places entries in buckets of the low
// kDupDigitBits tile bits (grouped duplication); stable radix passes over the
// remaining tile bits finish the grouping by tile, which lands in buffer 0;
// buffer 1 is then free scratch for the per-tile fallback sort.  GLOBAL: the
// full (tile, depth) sort, result in buffer 0.
struct SortPlan {
    int tile_bits, key_bits, group_bits, group_shift, tile_passes, full_passes, dup_buf;
};

SortPlan sort_plan(int tiles, int mode) {
    SortPlan p;
    p.tile_bits = bits_for_tiles(tiles);
    p.key_bits = 32 + p.tile_bits;
    p.full_passes = gsr::sort_pass_count(p.key_bits);
    // The hierarchical order's duplication already buckets entries by the low
    // tile bits; the global order's writes them at per-Gaussian offsets, so
    // its grouping passes cover every tile bit.
    const int done_bits = mode == GSR_MODE_HIER ? gsr::kDupDigitBits : 0;
    p.group_shift = 32 + done_bits;
    p.group_bits = p.tile_bits > done_bits ? p.tile_bits - done_bits : 0;
    p.tile_passes = p.group_bits > 0 ? gsr::sort_pass_count(p.group_bits) : 0;
    p.dup_buf = p.tile_passes & 1;
    return p;
}

int64_t dup_workgroups(int64_t n) { return (n + 255) / 256; }

// Records of a batch view start at a multiple of 256 (one preprocessing
// workgroup), so that workgroups are numbered across the batch.
int64_t align_records(int64_t n) { return (n + 255) & ~(int64_t)255; }

// Workspace regions not published in gsr_layout.
struct InnerLayout {
    int64_t scan_partial, hist, keys1, vals1, chunks;
};

// Layout for a given entry capacity.
void layout_for(int64_t n, int tiles, int64_t cap, gsr_layout* L, InnerLayout* in) {
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L->splat = take(64 * n);
    L->colour = take(16 * n);
    L->zd = take(8 * n);
    L->rect = take(16 * n);
    L->touched = take(4 * n);
    L->kmask = take(8 * n);
    L->offsets = take(4 * n);
    L->dup_hist = take(4 * gsr::kDupBins * dup_workgroups(n));
    L->grad2d = take(36 * n);
    L->ranges = take(8 * (int64_t)tiles);
    L->counters = take(64);
    L->pre_len = take(4 * (int64_t)tiles);
    L->tile_flag = take(4 * 3 * (int64_t)tiles);  // flags, then the render's per-tile scratch
    const int64_t nb = (int64_t)gsr::sort_blocks((size_t)cap);
    const int64_t sp = (int64_t)std::max({gsr::scan_partial_len((size_t)n), gsr::scan_partial_len((size_t)tiles),
                                          gsr::scan_partial_len((size_t)(gsr::kDupBins * dup_workgroups(n))),
                                          gsr::scan_partial_len((size_t)nb * gsr::kSortMaxBins)}) +
                       2;
    in->scan_partial = take(4 * sp);
    in->hist = take(4 * gsr::kSortMaxBins * nb);
    in->chunks = take(8 * (int64_t)gsr::flagged_chunk_capacity((size_t)cap, (size_t)tiles));
    L->keys = take(8 * cap);
    in->keys1 = take(8 * cap);
    L->values = take(4 * cap);
    in->vals1 = take(4 * cap);
    L->pre_vals = take(4 * cap);
    L->entry_capacity = cap;
    L->total_bytes = off;
}

int tiles_of(int W, int H) { return ((W + 15) / 16) * ((H + 15) / 16); }

int compute_layout(int64_t n, int32_t W, int32_t H, size_t ws_bytes, gsr_layout* L, InnerLayout* in) {
    if (n < 0 || W <= 0 || H <= 0 || W > 32768 || H > 32768) return GSR_EINVAL;
    const int tiles = tiles_of(W, H);
    // Largest capacity whose layout fits (the layout size grows with it).
    int64_t lo = 0, hi = ((int64_t)1 << 31) - 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        layout_for(n, tiles, mid, L, in);
        if (L->total_bytes <= (int64_t)ws_bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    if (lo <= 0) return GSR_ECAPACITY;
    layout_for(n, tiles, lo, L, in);
    return GSR_OK;
}

gsr::DevCam make_cam(const gsr_camera* c) {
    gsr::DevCam d;
    for (int i = 0; i < 9; ++i) d.R[i] = c->R[i];
    for (int i = 0; i < 3; ++i) {
        d.t[i] = c->t[i];
        d.o[i] = c->center[i];
    }
    d.fx = c->fx;
    d.fy = c->fy;
    d.rfx = 1.0f / c->fx;
    d.rfy = 1.0f / c->fy;
    d.cx = c->cx;
    d.cy = c->cy;
    d.znear = c->znear;
    d.W = c->W;
    d.H = c->H;
    d.tiles_x = (c->W + 15) / 16;
    d.tiles_y = (c->H + 15) / 16;
    // Frustum clamp of the EWA Jacobian: 1.3 x tan(half field of view).
    d.limx = 1.3f * ((float)c->W / (2.0f * c->fx));
    d.limy = 1.3f * ((float)c->H / (2.0f * c->fy));
    return d;
}

int check_scene(const gsr_scene* s) {
    if (!s) return fail(GSR_EINVAL, "scene is NULL");
    if (s->n < 0) return fail(GSR_EINVAL, "scene n < 0");
    if (s->sh_degree < 0 || s->sh_degree > 3) return fail(GSR_EINVAL, "sh_degree must be 0..3");
    if (s->n > 0 && (!s->means || !s->scales || !s->rots || !s->opacities || !s->sh))
        return fail(GSR_EINVAL, "scene array is NULL");
    return GSR_OK;
}

int check_camera(const gsr_camera* c) {
    if (!c) return fail(GSR_EINVAL, "camera is NULL");
    if (c->W <= 0 || c->H <= 0 || c->W > 32768 || c->H > 32768) return fail(GSR_EINVAL, "bad image size");
    if (!(c->fx > 0.0f) || !(c->fy > 0.0f)) return fail(GSR_EINVAL, "focal lengths must be > 0");
    return GSR_OK;
}

gsr::FrameBufs frame_bufs(char* base, const gsr_layout& L, const InnerLayout& in) {
    gsr::FrameBufs b;
    b.pk = (float4*)(base + L.splat);
    b.col = (float4*)(base + L.colour);
    b.zd = (float2*)(base + L.zd);
    b.rect = (int4*)(base + L.rect);
    b.touched = (uint32_t*)(base + L.touched);
    b.kmask = (uint64_t*)(base + L.kmask);
    b.offsets = (uint32_t*)(base + L.offsets);
    b.dhist = (uint32_t*)(base + L.dup_hist);
    b.scan_partial = (uint32_t*)(base + in.scan_partial);
    b.hist = (uint32_t*)(base + in.hist);
    b.keys[0] = (uint64_t*)(base + L.keys);
    b.keys[1] = (uint64_t*)(base + in.keys1);
    b.vals[0] = (uint32_t*)(base + L.values);
    b.vals[1] = (uint32_t*)(base + in.vals1);
    b.ranges = (uint32_t*)(base + L.ranges);
    b.counters = (uint32_t*)(base + L.counters);
    b.capacity = (uint32_t)L.entry_capacity;
    b.pre_vals = (uint32_t*)(base + L.pre_vals);
    b.pre_len = (uint32_t*)(base + L.pre_len);
    b.tile_flag = (uint32_t*)(base + L.tile_flag);
    b.flist = nullptr;
    b.chunks = (uint2*)(base + in.chunks);
    return b;
}

// Fingerprint of a frame: what the workspace's lists and records depend on
// (scene arrays and sizes, camera, blend order and queue configuration).  The
// forward writes it to counters[8..11]; the backward compares it with its own
// arguments on the device (no host synchronisation).
void frame_fingerprint(const gsr_scene* sc, const gsr_camera* c, const gsr_config* cfg, uint32_t out[4]) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xffu;
            h *= 1099511628211ull;
        }
    };
    auto mixf = [&](float f) {
        uint32_t u;
        std::memcpy(&u, &f, 4);
        mix(u);
    };
    mix((uint64_t)(uint32_t)sc->sh_degree);
    mix((uint64_t)(uintptr_t)sc->means);
    mix((uint64_t)(uintptr_t)sc->scales);
    mix((uint64_t)(uintptr_t)sc->rots);
    mix((uint64_t)(uintptr_t)sc->opacities);
    mix((uint64_t)(uintptr_t)sc->sh);
    for (int k = 0; k < 9; ++k) mixf(c->R[k]);
    for (int k = 0; k < 3; ++k) {
        mixf(c->t[k]);
        mixf(c->center[k]);
    }
    mixf(c->fx);
    mixf(c->fy);
    mixf(c->cx);
    mixf(c->cy);
    mixf(c->znear);
    mix((uint64_t)(uint32_t)cfg->mode);
    mix((uint64_t)(uint32_t)cfg->head);
    mix((uint64_t)cfg->flags);
    mix((uint64_t)(uint32_t)cfg->sort_prefix);
    out[0] = (uint32_t)sc->n;
    out[1] = ((uint32_t)c->W & 0xffffu) | ((uint32_t)c->H << 16);
    out[2] = (uint32_t)h;
    out[3] = (uint32_t)(h >> 32);
}

__global__ void k_write_words(uint32_t* dst, uint4 v) {
    if (threadIdx.x == 0) {
        dst[0] = v.x;
        dst[1] = v.y;
        dst[2] = v.z;
        dst[3] = v.w;
    }
}

// Default entries per tile sorted up front for an image of `tiles` tiles:
// about 2^23 entries over the frame (2^25 for the 3DGS lists of the global
// order and the resort window, which keep every rectangle tile and reach
// deeper before their pixels finish), a power of two from 1024 (4096) up to
// 8192.  Views with fewer tiles have longer lists whose pixels reach deeper,
// and a longer prefix spares their tiles the whole-list fallback and the
// second render (1M-Gaussian scene, ms per frame at M = 1024 / 2048 / 8192:
// 1280x720 2.51 / 1.70 / -, 512x512 - / 3.73 / 2.40).  Below 512 tiles a
// dense scene's pixels reach deeper than any prefix sorted in LDS and most
// deep tiles would be rendered twice, so 0 is returned: every tile's whole
// list is sorted up front (by the chunked fallback sort) and rendered once.
int default_prefix(int tiles, int mode) {
    const bool global = mode == GSR_MODE_GLOBAL || mode == GSR_MODE_WINDOW;
    int m = global ? 4096 : 1024;
    if (tiles < 512) return 0;
    const int64_t budget = global ? ((int64_t)1 << 25) : ((int64_t)1 << 23);
    while (2 * m <= 8192 && (int64_t)(2 * m) * tiles <= budget) m *= 2;
    return m;
}

int prefix_len(const gsr_config* cfg, int tiles) {
    if (cfg->sort_prefix != 0) return cfg->sort_prefix;
    return default_prefix(tiles, cfg->mode);
}

// Sort stage of a frame (or a batch): group by tile, tile ranges and each
// tile's sorted prefix.
hipError_t sort_stage(const gsr::FrameBufs& b, int tiles, int mode, uint32_t M, hipStream_t s,
                      void* const* scatter_events, void* const* order_events = nullptr) {
    const SortPlan sp = sort_plan(tiles, mode);
    hipError_t e;
    int res = 0;
    auto mark = [&](int k) -> hipError_t {
        return order_events ? hipEventRecord((hipEvent_t)order_events[k], s) : hipSuccess;
    };
    // Both orders: group by tile (stable radix passes over the tile bits not
    // yet grouped), then order each tile's first M entries by (depth, id).
    if ((e = gsr::launch_fill_u32(b.tile_flag, 3 * (size_t)tiles, 0u, s)) != hipSuccess) return e;
    if (sp.tile_passes > 0) {
        if ((e = gsr::launch_sort_pairs(b.keys, b.vals, b.counters, b.capacity, b.hist, b.scan_partial, sp.group_bits,
                                        sp.dup_buf, &res, s, scatter_events, sp.group_shift)) != hipSuccess)
            return e;
    }
    if ((e = mark(0)) != hipSuccess) return e;
    if ((e = gsr::launch_tile_prefix(b.keys[0], b.vals[0], b.counters, (uint32_t)tiles, b.ranges, b.pre_vals,
                                     b.pre_len, b.tile_flag, M, s)) != hipSuccess)
        return e;
    (void)mode;
    return mark(1);
}

// Fallback of the HIER sort: the whole sorted list of every tile the prefix
// render flagged (counters[5] = their entries, counters[6] = their number).
hipError_t fallback_sort(const gsr::FrameBufs& b, int tiles, hipStream_t s) {
    return gsr::launch_tile_sort_flagged(b.keys[0], b.vals[0], b.keys[1], b.ranges, b.tile_flag, (uint32_t)tiles,
                                         b.pre_vals, b.pre_len, b.counters, b.flist, b.chunks, s);
}

void set_prefix_lists(gsr::RenderArgs& ra, const gsr::FrameBufs& b, int list_mode) {
    ra.list_mode = list_mode;
    ra.vals = b.vals[0];
    ra.pre_vals = b.pre_vals;
    ra.pre_len = b.pre_len;
    ra.tile_flag = b.tile_flag;
}

int render_impl(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws, size_t ws_bytes,
                float* rgb, float* depth, int32_t* count, float* T_final, int32_t* blend_ids, int32_t max_k,
                int32_t* status_dev, gsr_stream_t stream, void* const* events, int32_t n_events,
                uint64_t* work = nullptr, float* delta = nullptr) {
    int rc = check_scene(scene);
    if (rc) return rc;
    if ((rc = check_camera(cam))) return rc;
    if (!cfg) return fail(GSR_EINVAL, "config is NULL");
    if ((rc = gsr_check_config(cfg))) return rc;
    if (!ws || !rgb || !depth || !count || !T_final || !status_dev) return fail(GSR_EINVAL, "output or workspace is NULL");
    if (blend_ids && max_k <= 0) return fail(GSR_EINVAL, "max_k must be > 0");
    if ((cfg->mode == GSR_MODE_HIER || cfg->mode == GSR_MODE_WINDOW) && !gsr::hier_head_supported(cfg->head))
        return fail(GSR_EUNSUPPORTED, "head size not built (1,2,3,4,6,8,12,16,20,24)");
    gsr_layout L;
    InnerLayout in;
    rc = compute_layout(scene->n, cam->W, cam->H, ws_bytes, &L, &in);
    if (rc) return fail(rc, "workspace too small");
    char* base = (char*)ws;
    if (((uintptr_t)base & 255) != 0) return fail(GSR_EINVAL, "workspace must be 256-byte aligned");
    const gsr::FrameBufs b = frame_bufs(base, L, in);

    hipStream_t s = (hipStream_t)stream;
    const gsr::DevCam dc = make_cam(cam);
    const int tiles = dc.tiles_x * dc.tiles_y;
    // GSR_MODE_WINDOW walks the lists of the global order, GSR_MODE_FULL the
    // exactly culled lists of the hierarchical one.
    const int mode = cfg->mode == GSR_MODE_WINDOW ? GSR_MODE_GLOBAL
                     : cfg->mode == GSR_MODE_FULL ? GSR_MODE_HIER
                                                  : cfg->mode;
    const SortPlan sp = sort_plan(tiles, mode);
    const uint32_t M = (uint32_t)prefix_len(cfg, tiles);
    gsr::SceneArgs sc{scene->n, scene->sh_degree, scene->means, scene->scales, scene->rots, scene->opacities, scene->sh};

    hipError_t e;
    auto mark = [&](int k) -> hipError_t {
        return events ? hipEventRecord((hipEvent_t)events[k], s) : hipSuccess;
    };
    if ((e = mark(0)) != hipSuccess) return fail_hip(e, "event");
    if ((e = gsr::launch_fill_u32(b.counters, 16, 0u, s)) != hipSuccess) return fail_hip(e, "clear");
    {
        uint32_t fp[gsr::kFingerprintWords];
        frame_fingerprint(scene, cam, cfg, fp);
        hipLaunchKernelGGL(k_write_words, dim3(1), dim3(64), 0, s, b.counters + gsr::kFingerprintOffset,
                           make_uint4(fp[0], fp[1], fp[2], fp[3]));
        if ((e = hipGetLastError()) != hipSuccess) return fail_hip(e, "fingerprint");
    }
    // Hierarchical lists use grouped duplication (entries bucketed by their
    // low tile bits), the global order duplication at per-Gaussian offsets.
    const gsr::DupGroups grp{b.dhist, (uint32_t)dup_workgroups(scene->n), 0u, 0u};
    const gsr::DupGroups* groups = mode == GSR_MODE_HIER ? &grp : nullptr;
    if ((e = gsr::launch_preprocess(sc, dc, mode, cfg->lb_threshold, cfg->flags, b, s, groups)) != hipSuccess)
        return fail_hip(e, "preprocess");
    if ((e = mark(1)) != hipSuccess) return fail_hip(e, "event");
    if (groups)
        e = gsr::launch_scan(b.dhist, b.dhist, (size_t)gsr::kDupBins * grp.stride, b.scan_partial, b.counters,
                             b.capacity, status_dev, s, b.counters + 3);
    else
        e = gsr::launch_scan(b.touched, b.offsets, (size_t)scene->n, b.scan_partial, b.counters, b.capacity, status_dev,
                             s, b.counters + 3);
    if (e != hipSuccess) return fail_hip(e, "scan");
    if ((e = gsr::launch_duplicate(scene->n, dc, mode, cfg->lb_threshold, cfg->flags, b, sp.dup_buf, status_dev, s, 0u,
                                   0u, groups)) != hipSuccess)
        return fail_hip(e, "duplicate");
    if ((e = mark(2)) != hipSuccess) return fail_hip(e, "event");
    const int n_sort_ev = sp.tile_passes;
    void* const* scatter_ev = (events && n_events >= 5 + 2 * n_sort_ev) ? events + 5 : nullptr;
    // Optional brackets of single launches: the per-tile ordering and the
    // first render pass.
    void* const* kernel_ev = (events && n_events >= 9 + 2 * n_sort_ev) ? events + 5 + 2 * n_sort_ev : nullptr;
    auto kmark = [&](int k) -> hipError_t {
        return kernel_ev ? hipEventRecord((hipEvent_t)kernel_ev[k], s) : hipSuccess;
    };
    if ((e = sort_stage(b, tiles, mode, M, s, scatter_ev, kernel_ev)) != hipSuccess) return fail_hip(e, "sort");
    if ((e = mark(3)) != hipSuccess) return fail_hip(e, "event");
    gsr::RenderArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.cam = dc;
    ra.n = (uint32_t)scene->n;
    ra.pk = b.pk;
    ra.col = b.col;
    ra.zd = b.zd;
    ra.vals = b.vals[0];
    ra.ranges = b.ranges;
    ra.counters = b.counters;
    ra.rgb = rgb;
    ra.depth = depth;
    ra.count = count;
    ra.T = T_final;
    ra.blend_ids = blend_ids;
    ra.max_k = blend_ids ? max_k : 0;
    ra.delta = delta;
    ra.bg0 = cfg->bg[0];
    ra.bg1 = cfg->bg[1];
    ra.bg2 = cfg->bg[2];
    ra.flags = (int)cfg->flags;
    if (work) {
        if ((e = gsr::launch_fill_u32((uint32_t*)work, 2 * GSR_WORK_COUNTS, 0u, s)) != hipSuccess)
            return fail_hip(e, "clear");
        ra.work = (unsigned long long*)work;
    }
    if (cfg->mode == GSR_MODE_FULL) {
        ra.list_mode = gsr::kListFull;  // the grouped lists, in any order
        if ((e = kmark(2)) != hipSuccess) return fail_hip(e, "event");
        if ((e = gsr::launch_render_full(ra, s)) != hipSuccess) return fail_hip(e, "render");
        if ((e = kmark(3)) != hipSuccess) return fail_hip(e, "event");
    } else {
        // Prefix pass, then the fallback: the flagged tiles' whole lists are
        // sorted and those tiles rendered again.  With M = 0 every tile's
        // whole list is sorted first and one pass renders them.
        const bool window = cfg->mode == GSR_MODE_WINDOW;
        auto render = [&]() -> hipError_t {
            if (mode == GSR_MODE_HIER) return gsr::launch_render_hier(ra, cfg->head, s);
            return window ? gsr::launch_render_window(ra, cfg->head, s) : gsr::launch_render_global(ra, s);
        };
        if (M == 0 && (e = fallback_sort(b, tiles, s)) != hipSuccess) return fail_hip(e, "whole-list sort");
        ra.deep = M == 0;  // few tiles with whole lists: one wavefront per SIMD or fewer
        set_prefix_lists(ra, b, gsr::kListPrefix);
        if ((e = kmark(2)) != hipSuccess) return fail_hip(e, "event");
        if ((e = render()) != hipSuccess) return fail_hip(e, "render");
        if ((e = kmark(3)) != hipSuccess) return fail_hip(e, "event");
        if (M != 0) {
            if ((e = fallback_sort(b, tiles, s)) != hipSuccess) return fail_hip(e, "fallback sort");
            ra.work = nullptr;  // the work of the prefix pass is counted
            ra.list_mode = gsr::kListFlagged;
            if ((e = render()) != hipSuccess) return fail_hip(e, "render fallback");
        }
    }
    if ((e = mark(4)) != hipSuccess) return fail_hip(e, "event");
    return GSR_OK;
}


int backward_impl(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws, size_t ws_bytes,
                  const float* dL, const float* rgb, const float* T_final, float* dmeans, float* dscales, float* drots,
                  float* dopac, float* dsh, int32_t* status_dev, gsr_stream_t stream) {
    int rc = check_scene(scene);
    if (rc) return rc;
    if ((rc = check_camera(cam))) return rc;
    if (!cfg) return fail(GSR_EINVAL, "config is NULL");
    if ((rc = gsr_check_config(cfg))) return rc;
    if (cfg->mode != GSR_MODE_HIER) return fail(GSR_EUNSUPPORTED, "backward is built for the hierarchical order");
    if (!gsr::hier_head_supported(cfg->head)) return fail(GSR_EUNSUPPORTED, "head size not built");
    if (!ws || !dL || !rgb || !T_final) return fail(GSR_EINVAL, "input is NULL");
    if (scene->n > 0 && (!dmeans || !dscales || !drots || !dopac || !dsh)) return fail(GSR_EINVAL, "gradient is NULL");
    gsr_layout L;
    InnerLayout in;
    rc = compute_layout(scene->n, cam->W, cam->H, ws_bytes, &L, &in);
    if (rc) return fail(rc, "workspace too small");
    char* base = (char*)ws;
    if (((uintptr_t)base & 255) != 0) return fail(GSR_EINVAL, "workspace must be 256-byte aligned");
    const gsr::FrameBufs b = frame_bufs(base, L, in);
    float* g2 = (float*)(base + L.grad2d);
    hipStream_t s = (hipStream_t)stream;
    const gsr::DevCam dc = make_cam(cam);
    gsr::SceneArgs sc{scene->n, scene->sh_degree, scene->means, scene->scales, scene->rots, scene->opacities, scene->sh};
    hipError_t e;
    if ((e = gsr::launch_fill_u32((uint32_t*)g2, (size_t)9 * scene->n, 0u, s)) != hipSuccess) return fail_hip(e, "clear");
    gsr::RenderArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.cam = dc;
    ra.n = (uint32_t)scene->n;
    ra.pk = b.pk;
    ra.col = b.col;
    ra.zd = b.zd;
    ra.vals = b.vals[0];
    ra.ranges = b.ranges;
    ra.counters = b.counters;
    ra.bg0 = cfg->bg[0];
    ra.bg1 = cfg->bg[1];
    ra.bg2 = cfg->bg[2];
    ra.dL = dL;
    ra.rgb_in = rgb;
    ra.T_in = T_final;
    ra.grad2d = g2;
    ra.flags = (int)cfg->flags;
    ra.fp = b.counters + gsr::kFingerprintOffset;
    frame_fingerprint(scene, cam, cfg, ra.fp_expect);
    ra.status = status_dev;
    set_prefix_lists(ra, b, gsr::kListSorted);
    if ((e = gsr::launch_render_hier(ra, cfg->head, s)) != hipSuccess) return fail_hip(e, "render backward");
    if ((e = gsr::launch_preprocess_backward(sc, dc, b.pk, g2, dmeans, dscales, drots, dopac, dsh, s)) != hipSuccess)
        return fail_hip(e, "preprocess backward");
    return GSR_OK;
}

// ---------------------------------------------------------------------------
// Batched rendering: many views of several scenes in one launch sequence.
// ---------------------------------------------------------------------------
// Batch counters (uint32 words): [0] entries, [2] tiles, [3] entries needed,
// [5], [6] flagged entries and tiles, from kBatchQueue0 the work-queue heads
// of the prefix pass, then those of the flagged pass.
constexpr int kBatchQueue0 = 16;
constexpr int kBatchCounters = kBatchQueue0 + 2 * gsr::kBatchQueues;

struct BatchLayout {
    int64_t views, pk, col, zd, rect, touched, kmask, offsets, dhist, ranges, counters;
    int64_t pre_vals, pre_len, tile_flag, flist, chunks;
    int64_t keys[2], vals[2], hist, partial;
    int64_t tkeys[2], tvals[2], thist, tpartial;
    int64_t cap, total;
};

void batch_layout_for(int64_t R, int64_t tiles, int64_t n_views, int64_t cap, BatchLayout* L) {
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        const int64_t o = off;
        off = align256(off + bytes);
        return o;
    };
    L->views = take((int64_t)sizeof(gsr::ViewDev) * n_views);
    L->pk = take(64 * R);
    L->col = take(16 * R);
    L->zd = take(8 * R);
    L->rect = take(16 * R);
    L->touched = take(4 * R);
    L->kmask = take(8 * R);
    L->offsets = take(4 * R);
    L->dhist = take(4 * gsr::kDupBins * dup_workgroups(R));
    L->ranges = take(8 * tiles);
    L->counters = take(4 * kBatchCounters);
    L->pre_len = take(4 * tiles);
    L->tile_flag = take(4 * 3 * tiles);
    L->flist = take(4 * tiles);
    const int64_t nbt = (int64_t)gsr::sort_blocks((size_t)tiles);
    L->tkeys[0] = take(8 * tiles);
    L->tkeys[1] = take(8 * tiles);
    L->tvals[0] = take(4 * tiles);
    L->tvals[1] = take(4 * tiles);
    L->thist = take(4 * gsr::kSortMaxBins * nbt);
    L->tpartial = take(4 * ((int64_t)gsr::scan_partial_len((size_t)nbt * gsr::kSortMaxBins) + 2));
    const int64_t nb = (int64_t)gsr::sort_blocks((size_t)cap);
    L->partial = take(4 * ((int64_t)std::max({gsr::scan_partial_len((size_t)R), gsr::scan_partial_len((size_t)tiles),
                                              gsr::scan_partial_len((size_t)(gsr::kDupBins * dup_workgroups(R))),
                                              gsr::scan_partial_len((size_t)nb * gsr::kSortMaxBins)}) +
                           2));
    L->hist = take(4 * gsr::kSortMaxBins * nb);
    L->chunks = take(8 * (int64_t)gsr::flagged_chunk_capacity((size_t)cap, (size_t)tiles));
    L->keys[0] = take(8 * cap);
    L->keys[1] = take(8 * cap);
    L->vals[0] = take(4 * cap);
    L->vals[1] = take(4 * cap);
    L->pre_vals = take(4 * cap);
    L->cap = cap;
    L->total = off;
}

}  // namespace

struct gsr_batch {
    std::vector<gsr_scene> scenes;
    std::vector<gsr_view> views;
    gsr_config cfg;
    gsr_schedule sched;
    char* ws;
    size_t ws_bytes;
    BatchLayout L;
    int64_t R, tiles;
    std::vector<int64_t> rec_base, tile_base;
    int cu_count;
};

namespace {

int validate_batch(const gsr_scene* scenes, int32_t n_scenes, const gsr_view* views, int32_t n_views,
                   int64_t* R, int64_t* tiles) {
    if (!scenes || n_scenes <= 0 || !views || n_views <= 0) return fail(GSR_EINVAL, "empty batch");
    for (int i = 0; i < n_scenes; ++i)
        if (int rc = check_scene(&scenes[i])) return rc;
    *R = 0;
    *tiles = 0;
    for (int v = 0; v < n_views; ++v) {
        if (views[v].scene < 0 || views[v].scene >= n_scenes) return fail(GSR_EINVAL, "view scene index out of range");
        if (int rc = check_camera(&views[v].cam)) return rc;
        if (!views[v].rgb || !views[v].depth || !views[v].count || !views[v].T)
            return fail(GSR_EINVAL, "view output is NULL");
        *R += align_records(scenes[views[v].scene].n);
        *tiles += tiles_of(views[v].cam.W, views[v].cam.H);
    }
    if (*R >= ((int64_t)1 << 32) - 1 || *tiles >= ((int64_t)1 << 31)) return fail(GSR_EINVAL, "batch too large");
    return GSR_OK;
}

int batch_capacity(int64_t R, int64_t tiles, int64_t n_views, size_t ws_bytes, BatchLayout* L) {
    int64_t lo = 0, hi = ((int64_t)1 << 31) - 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        batch_layout_for(R, tiles, n_views, mid, L);
        if (L->total <= (int64_t)ws_bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    if (lo <= 0) return GSR_ECAPACITY;
    batch_layout_for(R, tiles, n_views, lo, L);
    return GSR_OK;
}

int batch_render_impl(gsr_batch* b, int32_t* status_dev, hipStream_t s) {
    char* base = b->ws;
    const BatchLayout& L = b->L;
    gsr::FrameBufs fb;
    fb.pk = (float4*)(base + L.pk);
    fb.col = (float4*)(base + L.col);
    fb.zd = (float2*)(base + L.zd);
    fb.rect = (int4*)(base + L.rect);
    fb.touched = (uint32_t*)(base + L.touched);
    fb.kmask = (uint64_t*)(base + L.kmask);
    fb.offsets = (uint32_t*)(base + L.offsets);
    fb.dhist = (uint32_t*)(base + L.dhist);
    fb.scan_partial = (uint32_t*)(base + L.partial);
    fb.hist = (uint32_t*)(base + L.hist);
    fb.keys[0] = (uint64_t*)(base + L.keys[0]);
    fb.keys[1] = (uint64_t*)(base + L.keys[1]);
    fb.vals[0] = (uint32_t*)(base + L.vals[0]);
    fb.vals[1] = (uint32_t*)(base + L.vals[1]);
    fb.ranges = (uint32_t*)(base + L.ranges);
    fb.counters = (uint32_t*)(base + L.counters);
    fb.capacity = (uint32_t)L.cap;
    fb.pre_vals = (uint32_t*)(base + L.pre_vals);
    fb.pre_len = (uint32_t*)(base + L.pre_len);
    fb.tile_flag = (uint32_t*)(base + L.tile_flag);
    fb.flist = (uint32_t*)(base + L.flist);
    fb.chunks = (uint2*)(base + L.chunks);
    const int tiles = (int)b->tiles;
    const SortPlan sp = sort_plan(tiles, GSR_MODE_HIER);
    const int lb = b->sched.lb_threshold;
    hipError_t e;
    if ((e = gsr::launch_fill_u32(fb.counters, kBatchCounters, 0u, s)) != hipSuccess) return fail_hip(e, "clear");
    if ((e = gsr::launch_fill_u32(fb.counters + 2, 1, (uint32_t)b->tiles, s)) != hipSuccess) return fail_hip(e, "clear");
    auto shifted = [&](int64_t r0) {
        gsr::FrameBufs v = fb;
        v.pk += 4 * r0;
        v.col += r0;
        v.zd += r0;
        v.rect += r0;
        v.touched += r0;
        v.kmask += r0;
        v.offsets += r0;
        return v;
    };
    // Grouped duplication over the whole batch: workgroup w of view v is
    // number rec_base[v] / 256 + w of the batch (every view's records start
    // at a multiple of 256, so each column of the counts has one writer).
    const uint32_t nwg = (uint32_t)dup_workgroups(b->R);
    auto groups_of = [&](size_t v) {
        return gsr::DupGroups{fb.dhist, nwg, (uint32_t)(b->rec_base[v] / 256), (uint32_t)b->tile_base[v]};
    };
    for (size_t v = 0; v < b->views.size(); ++v) {
        const gsr_scene& sc = b->scenes[b->views[v].scene];
        const gsr::SceneArgs sa{sc.n, sc.sh_degree, sc.means, sc.scales, sc.rots, sc.opacities, sc.sh};
        const gsr::DupGroups g = groups_of(v);
        if ((e = gsr::launch_preprocess(sa, make_cam(&b->views[v].cam), GSR_MODE_HIER, lb, b->cfg.flags,
                                        shifted(b->rec_base[v]), s, &g)) != hipSuccess)
            return fail_hip(e, "preprocess");
    }
    if ((e = gsr::launch_scan(fb.dhist, fb.dhist, (size_t)gsr::kDupBins * nwg, fb.scan_partial, fb.counters,
                              fb.capacity, status_dev, s, fb.counters + 3)) != hipSuccess)
        return fail_hip(e, "scan");
    for (size_t v = 0; v < b->views.size(); ++v) {
        const gsr_scene& sc = b->scenes[b->views[v].scene];
        const gsr::DupGroups g = groups_of(v);
        if ((e = gsr::launch_duplicate(sc.n, make_cam(&b->views[v].cam), GSR_MODE_HIER, lb, b->cfg.flags,
                                       shifted(b->rec_base[v]), sp.dup_buf, status_dev, s, (uint32_t)b->tile_base[v],
                                       (uint32_t)b->rec_base[v], &g)) != hipSuccess)
            return fail_hip(e, "duplicate");
    }
    // a batch holds many views: its default prefix is that of a large frame
    if ((e = sort_stage(fb, tiles, GSR_MODE_HIER, (uint32_t)prefix_len(&b->cfg, 1 << 30), s, nullptr)) != hipSuccess)
        return fail_hip(e, "sort");
    const uint32_t* order = nullptr;
    if (b->sched.cost_order) {
        uint64_t* tk[2] = {(uint64_t*)(base + L.tkeys[0]), (uint64_t*)(base + L.tkeys[1])};
        uint32_t* tv[2] = {(uint32_t*)(base + L.tvals[0]), (uint32_t*)(base + L.tvals[1])};
        if ((e = gsr::launch_tile_cost_keys(fb.ranges, (uint32_t)b->tiles, tk[0], tv[0], s)) != hipSuccess)
            return fail_hip(e, "tile costs");
        int tres = 0;
        if ((e = gsr::launch_sort_pairs(tk, tv, fb.counters + 2, (size_t)b->tiles, (uint32_t*)(base + L.thist),
                                        (uint32_t*)(base + L.tpartial), 32, 0, &tres, s)) != hipSuccess)
            return fail_hip(e, "tile order");
        order = tv[tres];
    }
    gsr::BatchArgs ba;
    std::memset(&ba, 0, sizeof(ba));
    ba.views = (const gsr::ViewDev*)(base + L.views);
    ba.n_views = (int)b->views.size();
    ba.n_records = (uint32_t)b->R;
    ba.pk = fb.pk;
    ba.col = fb.col;
    ba.zd = fb.zd;
    ba.vals = fb.vals[0];
    ba.ranges = fb.ranges;
    ba.order = order;
    ba.list_mode = gsr::kListPrefix;
    ba.pre_vals = fb.pre_vals;
    ba.pre_len = fb.pre_len;
    ba.tile_flag = fb.tile_flag;
    ba.flags = (int)b->cfg.flags;
    ba.queue = fb.counters + kBatchQueue0;
    ba.n_tiles = (uint32_t)b->tiles;
    ba.n_tiles_dev = nullptr;
    ba.bg0 = b->cfg.bg[0];
    ba.bg1 = b->cfg.bg[1];
    ba.bg2 = b->cfg.bg[2];
    const unsigned grid = (unsigned)(b->cu_count * std::max(1, b->sched.wgs_per_cu));
    if ((e = gsr::launch_render_hier_batch(ba, b->cfg.head, grid, s)) != hipSuccess) return fail_hip(e, "render");
    // Tiles whose prefix ran out: compacted, fully sorted and rendered again.
    if ((e = fallback_sort(fb, tiles, s)) != hipSuccess) return fail_hip(e, "fallback sort");
    ba.list_mode = gsr::kListFlagged;
    ba.order = fb.flist;
    ba.n_tiles_dev = fb.counters + 6;
    ba.queue = fb.counters + kBatchQueue0 + gsr::kBatchQueues;
    if ((e = gsr::launch_render_hier_batch(ba, b->cfg.head, grid, s)) != hipSuccess)
        return fail_hip(e, "render fallback");
    return GSR_OK;
}

std::string batch_key(const gsr_batch* b) {
    std::ostringstream k;
    k << "gfx950-" << b->cu_count << "cu-views" << b->views.size() << "-records" << b->R << "-tiles" << b->tiles
      << "-head" << b->cfg.head << "-prefix" << prefix_len(&b->cfg, 1 << 30);
    return k.str();
}

}  // namespace

namespace {
// The schedules gsr_batch_set_schedule accepts (and the autotuner may reuse).
bool schedule_valid(const gsr_schedule& c) {
    return c.wgs_per_cu >= 1 && c.wgs_per_cu <= 8 && (c.cost_order == 0 || c.cost_order == 1) && c.lb_threshold >= 0;
}
}  // namespace

// The workspace of gsr_render_noalloc: a static device array, one copy per
// GPU at its own address.  In host code `scratch` names a host-side stand-in,
// not device memory, so kernels get the address hipGetSymbolAddress returns
// for the current device, looked up once per device and kept.
constexpr size_t kNoAllocBytes = GSR_NOALLOC_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_workspace(void** out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(GSR_EUNSUPPORTED, "device index beyond the static workspace table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p & 255) != 0) return fail(GSR_EDEVICE, "static workspace is not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GSR_OK;
}
}  // namespace

extern "C" {

size_t gsr_batch_workspace_bytes(const gsr_scene* scenes, int32_t n_scenes, const gsr_view* views, int32_t n_views,
                                 int64_t entries_max) {
    int64_t R, tiles;
    if (validate_batch(scenes, n_scenes, views, n_views, &R, &tiles) || entries_max < 1 ||
        entries_max > ((int64_t)1 << 31) - 1)
        return 0;
    BatchLayout L;
    batch_layout_for(R, tiles, n_views, entries_max, &L);
    return (size_t)L.total;
}

void gsr_default_schedule(gsr_schedule* s) {
    if (!s) return;
    s->wgs_per_cu = 2;
    s->cost_order = 1;
    s->lb_threshold = 64;
}

int gsr_batch_create(const gsr_scene* scenes, int32_t n_scenes, const gsr_view* views, int32_t n_views,
                     const gsr_config* cfg, const gsr_schedule* sched, void* ws, size_t ws_bytes, gsr_batch** out) {
    if (!out) return fail(GSR_EINVAL, "out is NULL");
    *out = nullptr;
    int64_t R, tiles;
    if (int rc = validate_batch(scenes, n_scenes, views, n_views, &R, &tiles)) return rc;
    if (!cfg) return fail(GSR_EINVAL, "config is NULL");
    if (int rc = gsr_check_config(cfg)) return rc;
    if (cfg->mode != GSR_MODE_HIER) return fail(GSR_EUNSUPPORTED, "batches render the hierarchical order");
    if (!gsr::hier_head_supported(cfg->head)) return fail(GSR_EUNSUPPORTED, "head size not built");
    if (!ws || ((uintptr_t)ws & 255) != 0) return fail(GSR_EINVAL, "workspace NULL or not 256-byte aligned");
    gsr_batch* b = new gsr_batch();
    b->scenes.assign(scenes, scenes + n_scenes);
    b->views.assign(views, views + n_views);
    b->cfg = *cfg;
    if (sched)
        b->sched = *sched;
    else
        gsr_default_schedule(&b->sched);
    if (b->sched.wgs_per_cu < 1 || b->sched.wgs_per_cu > 8 || b->sched.lb_threshold < 0) {
        delete b;
        return fail(GSR_EINVAL, "bad schedule");
    }
    b->ws = (char*)ws;
    b->ws_bytes = ws_bytes;
    b->R = R;
    b->tiles = tiles;
    if (batch_capacity(R, tiles, n_views, ws_bytes, &b->L)) {
        delete b;
        return fail(GSR_ECAPACITY, "workspace too small for the batch");
    }
    std::vector<gsr::ViewDev> vd(n_views);
    int64_t r = 0, t = 0;
    for (int v = 0; v < n_views; ++v) {
        b->rec_base.push_back(r);
        b->tile_base.push_back(t);
        vd[v].cam = make_cam(&views[v].cam);
        vd[v].rgb = views[v].rgb;
        vd[v].depth = views[v].depth;
        vd[v].count = views[v].count;
        vd[v].T = views[v].T;
        vd[v].tile_base = (uint32_t)t;
        vd[v].rec_base = (uint32_t)r;
        r += align_records(scenes[views[v].scene].n);
        t += tiles_of(views[v].cam.W, views[v].cam.H);
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipMemcpy(b->ws + b->L.views, vd.data(), sizeof(gsr::ViewDev) * n_views, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        delete b;
        return fail_hip(e, "batch create");
    }
    *out = b;
    return GSR_OK;
}

int gsr_batch_render(gsr_batch* b, int32_t* status_dev, gsr_stream_t stream) {
    if (!b || !status_dev) return fail(GSR_EINVAL, "batch or status is NULL");
    return batch_render_impl(b, status_dev, (hipStream_t)stream);
}

int gsr_batch_set_schedule(gsr_batch* b, const gsr_schedule* sched) {
    if (!b || !sched || !schedule_valid(*sched)) return fail(GSR_EINVAL, "bad schedule");
    b->sched = *sched;
    return GSR_OK;
}

int gsr_batch_get_schedule(const gsr_batch* b, gsr_schedule* sched) {
    if (!b || !sched) return fail(GSR_EINVAL, "NULL argument");
    *sched = b->sched;
    return GSR_OK;
}

int64_t gsr_batch_records(const gsr_batch* b) { return b ? b->R : -1; }
int64_t gsr_batch_tiles(const gsr_batch* b) { return b ? b->tiles : -1; }
int64_t gsr_batch_entry_capacity(const gsr_batch* b) { return b ? b->L.cap : -1; }
int64_t gsr_batch_counters_offset(const gsr_batch* b) { return b ? b->L.counters : -1; }

int gsr_batch_tune(gsr_batch* b, int32_t* status_dev, gsr_stream_t stream, const char* cache_path, int32_t repeats,
                   gsr_schedule* best_out, float* best_ms) {
    if (!b || !status_dev) return fail(GSR_EINVAL, "batch or status is NULL");
    hipStream_t s = (hipStream_t)stream;
    const std::string key = batch_key(b);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string k;
        gsr_schedule c;
        float ms;
        // A line that does not hold a valid schedule (a stale or damaged
        // cache) is ignored, and the batch is tuned again.
        while (in >> k >> c.wgs_per_cu >> c.cost_order >> c.lb_threshold >> ms) {
            if (k == key && schedule_valid(c) && ms > 0.0f) {
                b->sched = c;
                if (best_out) *best_out = c;
                if (best_ms) *best_ms = ms;
                return GSR_OK;
            }
        }
    }
    // Every candidate renders the same pixels: only speed differs.
    std::vector<gsr_schedule> cands;
    for (int w : {1, 2, 3})
        for (int c : {0, 1})
            for (int lb : {32, 64, 128}) cands.push_back(gsr_schedule{w, c, lb});
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return fail(GSR_EDEVICE, "event");
    float best = 1e30f;
    gsr_schedule bs = b->sched;
    const int reps = repeats > 0 ? repeats : 3;
    int rc = GSR_OK;
    for (const gsr_schedule& c : cands) {
        b->sched = c;
        if ((rc = batch_render_impl(b, status_dev, s))) break;
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && !rc; ++r) rc = batch_render_impl(b, status_dev, s);
        (void)hipEventRecord(e1, s);
        if (rc) break;
        if (hipEventSynchronize(e1) != hipSuccess) {
            rc = fail(GSR_EDEVICE, "tune sync");
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms /= (float)reps;
        if (ms < best) {
            best = ms;
            bs = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->sched = bs;
    if (rc) return rc;
    if (best_out) *best_out = bs;
    if (best_ms) *best_ms = best;
    if (cache_path) {
        std::ofstream o(cache_path, std::ios::app);
        o << key << " " << bs.wgs_per_cu << " " << bs.cost_order << " " << bs.lb_threshold << " " << best << "\n";
    }
    return GSR_OK;
}

void gsr_batch_destroy(gsr_batch* b) { delete b; }


size_t gsr_workspace_bytes(int64_t n, int32_t W, int32_t H, int64_t entries_max) {
    if (n < 0 || W <= 0 || H <= 0 || entries_max < 1 || entries_max > ((int64_t)1 << 31) - 1) return 0;
    gsr_layout L;
    InnerLayout in;
    layout_for(n, tiles_of(W, H), entries_max, &L, &in);
    return (size_t)L.total_bytes;
}

int gsr_workspace_layout(int64_t n, int32_t W, int32_t H, size_t ws_bytes, gsr_layout* out) {
    if (!out) return fail(GSR_EINVAL, "layout is NULL");
    InnerLayout in;
    const int rc = compute_layout(n, W, H, ws_bytes, out, &in);
    if (rc) return fail(rc, "workspace too small or bad size");
    return GSR_OK;
}

void gsr_default_config(gsr_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->mode = GSR_MODE_HIER;
    c->batch = 32;
    c->tail = 64;
    c->pop = 16;
    c->mid = 8;
    c->mid_batch = 4;
    c->head = 4;
    c->lb_threshold = 64;
    c->sort_prefix = 0;
}

int gsr_check_config(const gsr_config* c) {
    if (!c) return fail(GSR_EINVAL, "config is NULL");
    if (c->mode != GSR_MODE_GLOBAL && c->mode != GSR_MODE_HIER && c->mode != GSR_MODE_FULL &&
        c->mode != GSR_MODE_WINDOW)
        return fail(GSR_EINVAL, "unknown mode");
    const uint32_t ablate = GSR_ABLATE_TILE_DEPTH | GSR_ABLATE_TILE_CULL | GSR_ABLATE_HIER_CULL;
    if ((c->flags & ~(ablate | (uint32_t)GSR_TILE_CENTRE_DEPTH)) != 0) return fail(GSR_EINVAL, "unknown flag");
    if ((c->flags & ablate) != 0 && c->mode != GSR_MODE_HIER)
        return fail(GSR_EINVAL, "ablation flags apply to GSR_MODE_HIER");
    if ((c->flags & GSR_TILE_CENTRE_DEPTH) != 0 && c->mode != GSR_MODE_GLOBAL)
        return fail(GSR_EINVAL, "GSR_TILE_CENTRE_DEPTH applies to GSR_MODE_GLOBAL");
    if (c->lb_threshold < 0) return fail(GSR_EINVAL, "lb_threshold must be >= 0");
    if (c->sort_prefix < 0 || c->sort_prefix > gsr::kMaxPrefix) return fail(GSR_EINVAL, "sort_prefix must be 0..16384");
    if (c->mode == GSR_MODE_HIER) {
        if (c->tail < 64 || (c->tail - 32) % 32 != 0) return fail(GSR_EINVAL, "tail must be 32n+32, n>=1");
        if (c->mid < 8 || (c->mid - 4) % 4 != 0) return fail(GSR_EINVAL, "mid must be 4m+4, m>=1");
        if (c->head < 1) return fail(GSR_EINVAL, "head must be >= 1");
        if (c->batch != 32 || c->tail != 64 || c->pop != 16 || c->mid != 8 || c->mid_batch != 4 || c->head > 24)
            return fail(GSR_EUNSUPPORTED, "only batch/tail/pop/mid/mid_batch = 32/64/16/8/4 and head <= 24 are built");
    }
    if (c->mode == GSR_MODE_WINDOW) {
        if (c->head < 1) return fail(GSR_EINVAL, "window must be >= 1");
        if (c->head > 24) return fail(GSR_EUNSUPPORTED, "windows up to 24 are built");
    }
    return GSR_OK;
}

int gsr_render(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws, size_t ws_bytes,
               float* rgb, float* depth, int32_t* count, float* T_final, int32_t* status_dev, gsr_stream_t stream) {
    return render_impl(scene, cam, cfg, ws, ws_bytes, rgb, depth, count, T_final, nullptr, 0, status_dev, stream,
                       nullptr, 0);
}

int gsr_render_staged(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws, size_t ws_bytes,
                      float* rgb, float* depth, int32_t* count, float* T_final, int32_t* status_dev,
                      gsr_stream_t stream, void* const* events, int32_t n_events) {
    if (!events || n_events < 5) return fail(GSR_EINVAL, "need at least 5 events");
    for (int k = 0; k < n_events; ++k)
        if (!events[k]) return fail(GSR_EINVAL, "event is NULL");
    return render_impl(scene, cam, cfg, ws, ws_bytes, rgb, depth, count, T_final, nullptr, 0, status_dev, stream,
                       events, n_events);
}

int gsr_render_work(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws, size_t ws_bytes,
                    float* rgb, float* depth, int32_t* count, float* T_final, int32_t* status_dev, uint64_t* work_dev,
                    gsr_stream_t stream) {
    if (!cfg || !work_dev) return fail(GSR_EINVAL, "config or work is NULL");
    if (cfg->mode != GSR_MODE_HIER || cfg->head != 4)
        return fail(GSR_EUNSUPPORTED, "work counts are built for the hierarchical render with head 4");
    return render_impl(scene, cam, cfg, ws, ws_bytes, rgb, depth, count, T_final, nullptr, 0, status_dev, stream,
                       nullptr, 0, work_dev);
}

int gsr_render_backward(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws,
                        size_t ws_bytes, const float* dL_drgb, const float* rgb, const float* T_final, float* dmeans,
                        float* dscales, float* drots, float* dopacities, float* dsh, int32_t* status_dev,
                        gsr_stream_t stream) {
    return backward_impl(scene, cam, cfg, ws, ws_bytes, dL_drgb, rgb, T_final, dmeans, dscales, drots, dopacities, dsh,
                         status_dev, stream);
}

int gsr_sort_passes(int32_t W, int32_t H) {
    if (W <= 0 || H <= 0) return fail(GSR_EINVAL, "bad image size");
    return sort_plan(tiles_of(W, H), GSR_MODE_GLOBAL).tile_passes;
}

int gsr_default_prefix(int32_t W, int32_t H, int32_t mode) {
    if (W <= 0 || H <= 0) return fail(GSR_EINVAL, "bad image size");
    if (mode != GSR_MODE_GLOBAL && mode != GSR_MODE_HIER && mode != GSR_MODE_FULL && mode != GSR_MODE_WINDOW)
        return fail(GSR_EINVAL, "unknown mode");
    return default_prefix(tiles_of(W, H), mode);
}

int gsr_group_passes(int32_t W, int32_t H) {
    if (W <= 0 || H <= 0) return fail(GSR_EINVAL, "bad image size");
    return sort_plan(tiles_of(W, H), GSR_MODE_HIER).tile_passes;
}

int gsr_render_sort_error(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws,
                          size_t ws_bytes, float* rgb, float* depth, int32_t* count, float* T_final, float* sort_error,
                          int32_t* status_dev, gsr_stream_t stream) {
    if (!sort_error) return fail(GSR_EINVAL, "sort_error is NULL");
    return render_impl(scene, cam, cfg, ws, ws_bytes, rgb, depth, count, T_final, nullptr, 0, status_dev, stream,
                       nullptr, 0, nullptr, sort_error);
}

int gsr_render_debug(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws, size_t ws_bytes,
                     float* rgb, float* depth, int32_t* count, float* T_final, int32_t* blend_ids, int32_t max_k,
                     int32_t* status_dev, gsr_stream_t stream) {
    if (!blend_ids) return fail(GSR_EINVAL, "blend_ids is NULL");
    return render_impl(scene, cam, cfg, ws, ws_bytes, rgb, depth, count, T_final, blend_ids, max_k, status_dev, stream,
                       nullptr, 0);
}

int gsr_render_noalloc(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, float* rgb,
                       float* depth, int32_t* count, float* T_final, int32_t* status_dev, gsr_stream_t stream) {
    if (!scene || !cam) return fail(GSR_EINVAL, "scene or camera is NULL");
    {
        gsr_layout L;
        InnerLayout in;
        if (compute_layout(scene->n, cam->W, cam->H, kNoAllocBytes, &L, &in) != GSR_OK)
            return fail(GSR_ECAPACITY, "scene and image do not fit the fixed workspace of GSR_NOALLOC_BYTES");
    }
    void* ws = nullptr;
    const int rc = noalloc_workspace(&ws);
    if (rc) return rc;
    return render_impl(scene, cam, cfg, ws, kNoAllocBytes, rgb, depth, count, T_final, nullptr, 0, status_dev, stream,
                       nullptr, 0);
}

int gsr_probe_math(const float* a, const float* b, int32_t n, float* out, gsr_stream_t stream) {
    if (n < 0 || (n > 0 && (!a || !b || !out))) return fail(GSR_EINVAL, "bad probe arguments");
    const hipError_t e = gsr::launch_probe_math(a, b, n, out, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "probe");
    return GSR_OK;
}

const char* gsr_last_error(void) { return g_last_error.c_str(); }

const char* gsr_version(void) { return "gsr 0.1 (gfx950)"; }

}  // extern "C"
