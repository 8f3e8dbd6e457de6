/*
 * gsr.h -- C ABI of the MI355X (gfx950) sorted Gaussian-splatting rasterizer.
 *
 * The library renders 3D Gaussians for a pinhole camera with the hierarchical
 * per-pixel resorting of "StopThePop: Sorted Gaussian Splatting for
 * View-Consistent Real-time Rendering" (Sec. 3.4), or with the global depth
 * order of 3D Gaussian Splatting (Sec. 2.1) for comparison.
 *
 * Conventions for every entry point:
 *  - Array pointers are DEVICE pointers (hipMalloc'd or torch CUDA tensors),
 *    except where a comment says host.  The caller allocates and owns every
 *    input, output and workspace buffer; the library keeps no device memory
 *    between calls.
 *  - All work is enqueued on the caller's stream and the call returns at once;
 *    there is no hidden host synchronisation.  Results are ready when the
 *    stream reaches that point.
 *  - Return value: GSR_OK (0) or a negative GSR_E* code; a message for the
 *    last error of the calling thread is available from gsr_last_error().
 *  - Data-dependent overflow (more tile entries than the workspace holds) is
 *    reported on the device, in bit 0 of *status_dev, which the library only
 *    ever ORs into; the caller clears it.  Outputs of such a call are
 *    undefined; size the workspace up and call again.
 *  - A Gaussian with a non-finite parameter, a non-positive scale or an
 *    opacity below 1/255 is culled; it is not an error.
 *  - Floating point is IEEE binary32 throughout: correctly rounded division
 *    and square root, fused multiply-adds only where written out (t_opt's dot
 *    products, the compositing sums, exp), and one project-written exp
 *    (Cody-Waite reduction + degree-7 polynomial).
 */
#ifndef GSR_H
#define GSR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* gsr_stream_t; /* a hipStream_t; NULL is the null stream */

enum {
    GSR_OK = 0,
    GSR_EINVAL = -1,       /* null pointer, bad size or invalid configuration */
    GSR_ECAPACITY = -2,    /* workspace smaller than gsr_workspace_bytes() requires */
    GSR_EDEVICE = -3,      /* a HIP call failed; see gsr_last_error() */
    GSR_EUNSUPPORTED = -4  /* device is not gfx950 */
};

/* Blend orders:
 *   GSR_MODE_GLOBAL  3DGS: 3-sigma rectangles, view-space depth keys, each
 *                    pixel blends its tile's list in key order (Sec. 2.1);
 *   GSR_MODE_HIER    the hierarchical resorting of Sec. 3.4 (opacity-aware
 *                    bounds, exact tile culling, tile-depth keys, tail / mid /
 *                    head queues on per-level t_opt);
 *   GSR_MODE_FULL    the full per-pixel sort (Sec. 3.2), a quality
 *                    reference: every contributor of a pixel (from the
 *                    exactly culled tile lists of GSR_MODE_HIER) blended in
 *                    (t_opt along the pixel ray, Gaussian id) order; many
 *                    times slower than the other modes;
 *   GSR_MODE_WINDOW  per-ray resorting (Sec. 3.3): the 3DGS lists of
 *                    GSR_MODE_GLOBAL, each pixel keeping a window of `head`
 *                    samples ordered by t_opt along its ray and blending the
 *                    front whenever the window overflows. */
enum { GSR_MODE_GLOBAL = 0, GSR_MODE_HIER = 1, GSR_MODE_FULL = 2, GSR_MODE_WINDOW = 3 };

/* Bits of *status_dev: GSR_STATUS_OVERFLOW, more tile entries than the
 * workspace holds (outputs undefined); GSR_STATUS_MISMATCH, a backward call
 * whose workspace does not hold the forward of the same scene, camera and
 * configuration (its gradients are then zero). */
enum { GSR_STATUS_OVERFLOW = 1, GSR_STATUS_MISMATCH = 2 };

/* Ablations of GSR_MODE_HIER (Sec. 4.3, Table performance_ablation), bits of
 * gsr_config.flags:
 *   GSR_ABLATE_TILE_DEPTH  (B) no tile-depth adjustment: every key of a
 *                          Gaussian uses its distance |mu - o| (t_opt along
 *                          the ray through its own mean);
 *   GSR_ABLATE_TILE_CULL   (D) no tile-based culling: every tile of the
 *                          opacity-aware rectangle gets an entry;
 *   GSR_ABLATE_HIER_CULL   (E) no culling at the 4x4 and 2x2 levels of the
 *                          render (the per-pixel alpha test remains).
 * (C), no load balancing, is lb_threshold >= GSR_NO_LOAD_BALANCE. */
enum { GSR_ABLATE_TILE_DEPTH = 1, GSR_ABLATE_TILE_CULL = 2, GSR_ABLATE_HIER_CULL = 4 };
#define GSR_NO_LOAD_BALANCE (1 << 30)

/* Variant of GSR_MODE_GLOBAL (Sec. 3.3, Fig. pertiledepth), a bit of
 * gsr_config.flags: GSR_TILE_CENTRE_DEPTH keys every tile entry with t_opt
 * along the ray through the tile's centre (the centre of its pixel-centre
 * hull) instead of the view-space depth; the 3DGS rectangle and the blend in
 * list order are unchanged (the naive per-tile depth, without per-pixel
 * resorting). */
enum { GSR_TILE_CENTRE_DEPTH = 8 };

/* Gaussians of one scene (Sec. 2.1): N rows per array, row-major, float32.
 *   means     [N,3]  centre mu
 *   scales    [N,3]  activated scales s (> 0)
 *   rots      [N,4]  quaternion (w, x, y, z), normalised inside; zero -> identity
 *   opacities [N]    activated opacity in [0, 1]
 *   sh        [N,(d+1)^2,3] real SH coefficients of degree d in 0..3 */
typedef struct gsr_scene {
    int32_t n;
    int32_t sh_degree;
    const float* means;
    const float* scales;
    const float* rots;
    const float* opacities;
    const float* sh;
} gsr_scene;

/* Pinhole camera.  p_cam = R p + t with R world->camera (row-major), camera
 * looking along +z, x right, y down; `center` is the camera centre -R^T t.
 * Pixel (i, j) has its centre at image coordinates (i, j). */
typedef struct gsr_camera {
    float R[9];
    float t[3];
    float center[3];
    float fx, fy, cx, cy;
    float znear;
    int32_t W, H;
} gsr_camera;

/* Render configuration (Sec. 3.4).  Queue sizes change results:
 *   batch     tail batch B (32; the kernel is built for 32)
 *   tail      tail capacity, 32 n + 32 with n >= 1 (64)
 *   pop       tail -> mid chunk (16)
 *   mid       mid capacity, 4 m + 4 with m >= 1 (8)
 *   mid_batch mid sub-batch (4)
 *   head      per-pixel head capacity K (HIER) or window size (WINDOW),
 *             one of 1, 2, 3, 4, 6, 8, 12, 16, 20, 24 (4); from 12 on, a
 *             tile's list is walked up to its first 2^27 entries
 * lb_threshold only changes speed (tiles above which preprocessing and
 * duplication share a Gaussian across the wavefront; 64; Gaussians of at most
 * min(lb_threshold, 64) tiles share their tiles with the other lanes, those
 * between 64 and lb_threshold are walked by their own lane, and at
 * GSR_NO_LOAD_BALANCE or above every Gaussian is walked by its own lane).
 * bg is the background colour. */
typedef struct gsr_config {
    int32_t mode;
    int32_t batch, tail, pop, mid, mid_batch, head;
    int32_t lb_threshold;
    float bg[3];
    uint32_t flags;      /* GSR_ABLATE_* bits (GSR_MODE_HIER only), GSR_TILE_CENTRE_DEPTH
                            (GSR_MODE_GLOBAL only), else 0 */
    int32_t sort_prefix; /* speed only: entries per tile sorted up front (1..16384;
                            0 = gsr_default_prefix for the image); see gsr_render */
} gsr_config;

/* Byte offsets of the regions of a workspace, for inspection and debugging.
 * Records (App. B.4), one row per Gaussian, zero when culled:
 *   splat    float[16]: 2D mean x y, conic a b | conic c, opacity, Sigma^-1 s00 s01 |
 *            s02 s11 s12 s22 | w = Sigma^-1 (mu - o) w0 w1 w2, ln(eps_O / opacity)
 *            (one 64-byte line per Gaussian, the record every render level reads)
 *   colour   float4 (r, g, b, |mu - o|)
 *   zd       float2 (view depth, |mu - o|)
 *   rect     int32[4] tile rectangle (x0, y0, x1, y1), inclusive
 *   touched  uint32 kept tiles          offsets uint32 exclusive prefix sum of touched
 *            (GSR_MODE_GLOBAL / GSR_MODE_WINDOW)
 *   dup_hist uint32 [32][ceil(N / 256)]: GSR_MODE_HIER / GSR_MODE_FULL count the
 *            kept tiles of each block of 256 Gaussians by the low 5 bits of the
 *            tile id, then hold their exclusive prefix sum (digit-major): the
 *            start of each block's bucket in the entries
 *   kmask    uint64 kept-tile bit mask (row-major over rect) of Gaussians whose
 *            rectangle holds at most min(lb_threshold, 64) tiles, else 0
 * Sort: keys uint64 (tile << 32 | order-preserving depth bits), values uint32
 * (Gaussian id), ranges uint32[tiles][2] = [start, end) per tile; counters
 * uint32[8] = (entries, entries consumed by the renderer, unused, entries needed before
 * clamping to the capacity (saturated at 2^32 - 1), unused, entries of the tiles that took
 * the fallback, number of such tiles, unused);
 * grad2d float[N][9] = backward scratch (d mean_2, d conic, d opacity, d rgb).
 * Every mode (GSR_MODE_GLOBAL and GSR_MODE_WINDOW with view-depth keys):
 * keys/values hold the entries grouped by tile (in no
 * particular order inside a tile; the keys of tiles that took the fallback
 * are overwritten), pre_vals uint32[capacity] each tile's sorted ids from its
 * range start (a prefix, or the whole list for a tile that took the
 * fallback), pre_len uint32[tiles] their number, tile_flag uint32[3][tiles]:
 * the entry count of a tile that took the fallback (else 0), then two rows
 * of per-tile scratch of the render. */
typedef struct gsr_layout {
    int64_t splat, colour, zd, rect, touched, kmask, offsets, dup_hist, grad2d;
    int64_t keys, values, ranges, counters;
    int64_t pre_vals, pre_len, tile_flag;
    int64_t entry_capacity;
    int64_t total_bytes;
} gsr_layout;

/* Workspace needed to render n Gaussians at W x H with room for
 * entries_max (tile, Gaussian) entries.  Returns 0 for invalid sizes. */
size_t gsr_workspace_bytes(int64_t n, int32_t W, int32_t H, int64_t entries_max);

/* Layout of a workspace of ws_bytes for n Gaussians at W x H.  The entry
 * capacity is whatever the workspace holds beyond the per-Gaussian and
 * per-tile regions.  Returns GSR_ECAPACITY if not even one entry fits. */
int gsr_workspace_layout(int64_t n, int32_t W, int32_t H, size_t ws_bytes, gsr_layout* out /* host */);

/* Default configuration (hierarchical, 32/64/16/8/4/4, black background). */
void gsr_default_config(gsr_config* cfg /* host */);

/* Validate a configuration (Sec. 3.4: tail = 32 n + 32, mid = 4 m + 4).
 * Returns GSR_OK or GSR_EINVAL. */
int gsr_check_config(const gsr_config* cfg /* host */);

/* Render one frame: preprocess, count and duplicate (tile, depth) entries,
 * sort them, find tile ranges, and blend every pixel front to back with
 * early termination (Eq. volume_desc).  In every mode the entries are
 * grouped by tile, each tile's first (at most sort_prefix) entries in (depth,
 * Gaussian id) order are selected and sorted, and a tile whose pixels are
 * still unfinished when its prefix runs out has its whole list sorted and is
 * rendered again (enqueued always; tiles that need nothing exit at once): the
 * order is that of a full sort by (tile, depth, id) in every case.  When the
 * default prefix is 0 (small images) every tile's whole list is sorted first
 * and rendered once.  The
 * blend order is that of the mode (see GSR_MODE_*).
 *   rgb     [3,H,W] float32 out   colour + T_final * bg
 *   depth   [H,W]   float32 out   sum of t_opt alpha T (t_opt along the pixel ray in FULL and
 *                                 WINDOW; GLOBAL: |mu - o|)
 *   count   [H,W]   int32   out   number of Gaussians blended
 *   T_final [H,W]   float32 out   final transmittance
 *   status_dev      int32   in/out, see above
 * ws must stay unmodified between a forward call and its backward. */
int gsr_render(const gsr_scene* scene /* host struct, device arrays */, const gsr_camera* cam /* host */,
               const gsr_config* cfg /* host */, void* ws, size_t ws_bytes, float* rgb, float* depth,
               int32_t* count, float* T_final, int32_t* status_dev, gsr_stream_t stream);

/* As gsr_render, and also writes the first max_k blended Gaussian ids of
 * every pixel, in blend order, to blend_ids [H,W,max_k] (int32, -1 padded). */
int gsr_render_debug(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws,
                     size_t ws_bytes, float* rgb, float* depth, int32_t* count, float* T_final,
                     int32_t* blend_ids, int32_t max_k, int32_t* status_dev, gsr_stream_t stream);

/* As gsr_render, and also writes each pixel's sort error (Sec. 3.3; the
 * measure of Table sortcost) to sort_error [H,W] (float32, device): over the
 * Gaussians the pixel blended, in blend order, the sum of t_k - t_{k+1} over
 * consecutive pairs with t_k > t_{k+1}, where t is t_opt along the pixel's
 * ray (Eq. dopt), in every mode (0 for an exact order).  Errors as gsr_render;
 * GSR_EINVAL when sort_error is NULL. */
int gsr_render_sort_error(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws,
                          size_t ws_bytes, float* rgb, float* depth, int32_t* count, float* T_final,
                          float* sort_error, int32_t* status_dev, gsr_stream_t stream);

/* Backward of gsr_render (Sec. 3.5), for the hierarchical order.  Given
 * dL_drgb [3,H,W] and the forward call's rgb and T_final, re-runs the same
 * per-pixel resorting front to back (nothing per pixel is stored by the
 * forward pass) and writes the gradients of L with respect to
 *   dmeans [N,3], dscales [N,3], drots [N,4] (unnormalised quaternion),
 *   dopacities [N], dsh [N,(d+1)^2,3]   (device, float32, overwritten).
 * scene, cam, cfg and ws must be exactly those of the forward call, and ws
 * unmodified since: the forward leaves a fingerprint of its scene arrays,
 * sizes, camera and configuration in ws, and a backward whose arguments do
 * not match it adds nothing (zero gradients) and sets GSR_STATUS_MISMATCH in
 * *status_dev (checked on the device; status_dev may be NULL).  The order of
 * floating-point atomic additions makes the gradients reproducible only to
 * rounding.  No gradient flows through the blend order, culling or early
 * termination (they are piecewise constant), nor through the depth output.
 * Returns GSR_EUNSUPPORTED for the global order. */
int gsr_render_backward(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws,
                        size_t ws_bytes, const float* dL_drgb, const float* rgb, const float* T_final,
                        float* dmeans, float* dscales, float* drots, float* dopacities, float* dsh,
                        int32_t* status_dev, gsr_stream_t stream);

/* As gsr_render, and records caller-created HIP events (hipEvent_t, passed
 * as void*) on the stream at the stage boundaries of the paper's per-stage
 * timing (Sec. 4.3): events[0] before Preprocess, [1] after Preprocess, [2]
 * after Duplicate (prefix sum + key emission), [3] after Sort (grouping by
 * tile, tile ranges and the per-tile sorted prefixes), [4] after Render
 * (including the fallback sort of flagged tiles and their second render).
 * With n_events >= 5 + 2 * passes (passes = gsr_group_passes(W, H) in
 * GSR_MODE_HIER and GSR_MODE_FULL, gsr_sort_passes(W, H) in GSR_MODE_GLOBAL
 * and GSR_MODE_WINDOW), events[5 + 2p] and [6 + 2p] also bracket the scatter
 * launch of radix pass p; with n_events >= 9 + 2 * passes, events[5 + 2 passes]
 * and [6 + 2 passes] bracket the per-tile ordering launch (the tile prefixes)
 * and [7 + 2 passes] and [8 + 2 passes] the first render launch.  The caller
 * owns the events. */
int gsr_render_staged(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws,
                      size_t ws_bytes, float* rgb, float* depth, int32_t* count, float* T_final,
                      int32_t* status_dev, gsr_stream_t stream, void* const* events, int32_t n_events);

/* As gsr_render, with the render counting the work of its levels (a model of
 * its arithmetic, for roofline accounting; the result images are the same):
 * work_dev uint64[GSR_WORK_COUNTS] (device, overwritten) =
 *   (cull tests at the 4x4 level, entries keyed there by t_opt,
 *    cull tests at the 2x2 level, entries keyed there,
 *    alpha tests at the pixels, entries keyed there, blends)
 * for the pass over the tiles' sorted prefixes.  GSR_MODE_HIER with head 4
 * only (else GSR_EUNSUPPORTED). */
#define GSR_WORK_COUNTS 7
int gsr_render_work(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, void* ws,
                    size_t ws_bytes, float* rgb, float* depth, int32_t* count, float* T_final,
                    int32_t* status_dev, uint64_t* work_dev, gsr_stream_t stream);

/* Number of radix passes that group a W x H frame's entries by tile in
 * GSR_MODE_GLOBAL and GSR_MODE_WINDOW: every tile bit (their duplication
 * writes entries at per-Gaussian offsets), digits of at most 9 bits. */
int gsr_sort_passes(int32_t W, int32_t H);

/* Number of radix passes that group a W x H frame's entries by tile: over the
 * tile bits above the low 5, which duplication already buckets by (0 for at
 * most 32 tiles). */
int gsr_group_passes(int32_t W, int32_t H);

/* The entries per tile that gsr_render sorts up front when
 * gsr_config.sort_prefix is 0, for a W x H image in `mode` (speed only; the
 * blend order never depends on it): a power of two near 2^23 / tiles (2^25 /
 * tiles for GSR_MODE_GLOBAL and GSR_MODE_WINDOW), at least 1024 (4096) and at
 * most 8192 -- 1024 at 1920x1080, 2048 at 1280x720, 8192 at 512x512; below
 * 512 tiles 0: no prefix, every tile's whole list sorted before one render
 * pass (256x256).  The batch API's default is the large-frame one (1024;
 * 4096).  GSR_EINVAL for bad arguments. */
int gsr_default_prefix(int32_t W, int32_t H, int32_t mode);

/* ---------------------------------------------------------------------------
 * Batched rendering: many views (cameras of any resolution) of several scenes
 * rendered by one launch sequence.  All views' Gaussians are preprocessed into
 * one record array, all (view, tile, depth) keys are sorted once, and one
 * persistent render kernel pulls (tile, 16x4 strip) work items of all views
 * from eight atomic queues, one per XCD (tile slot s of the work order, which
 * is largest tile lists first when cost-ordered, in queue s mod 8; a
 * wavefront drains its own XCD's queue, then the others).  Each view's pixels
 * equal those of gsr_render for that view (hierarchical order).
 * ------------------------------------------------------------------------- */
typedef struct gsr_view {
    int32_t scene;        /* index into the scenes array */
    gsr_camera cam;
    float* rgb;           /* [3,H,W] device outputs of this view */
    float* depth;         /* [H,W] */
    int32_t* count;       /* [H,W] */
    float* T;             /* [H,W] */
} gsr_view;

/* Launch parameters that change speed only, never results. */
typedef struct gsr_schedule {
    int32_t wgs_per_cu;   /* persistent render grid = compute units x this (1..8) */
    int32_t cost_order;   /* 1: tiles with the longest lists first; 0: view order */
    int32_t lb_threshold; /* see gsr_config */
} gsr_schedule;

typedef struct gsr_batch gsr_batch; /* opaque host-side plan */

/* Workspace for a batch with room for entries_max (view, tile, Gaussian)
 * entries in total; 0 for an invalid batch. */
size_t gsr_batch_workspace_bytes(const gsr_scene* scenes, int32_t n_scenes, const gsr_view* views, int32_t n_views,
                                 int64_t entries_max);

void gsr_default_schedule(gsr_schedule* sched /* host */);

/* Plan a batch (host arrays; the scenes' device arrays and the views' outputs
 * must stay valid while the plan is used).  Copies a per-view table into ws
 * with a blocking copy, so call it outside stream capture.  sched may be NULL
 * (default).  Only the hierarchical order is supported. */
int gsr_batch_create(const gsr_scene* scenes, int32_t n_scenes, const gsr_view* views, int32_t n_views,
                     const gsr_config* cfg, const gsr_schedule* sched, void* ws, size_t ws_bytes, gsr_batch** out);

/* Enqueue the whole batch on `stream`: kernel launches only (no allocation,
 * no host synchronisation, no memset nodes), so the call can be captured
 * into a HIP graph and replayed.  Overflow sets bit 0 of *status_dev. */
int gsr_batch_render(gsr_batch* batch, int32_t* status_dev, gsr_stream_t stream);

int gsr_batch_set_schedule(gsr_batch* batch, const gsr_schedule* sched);
int gsr_batch_get_schedule(const gsr_batch* batch, gsr_schedule* sched);

/* Autotuner: times every candidate schedule (persistent grid 1-3 workgroups
 * per compute unit, cost order on/off, load-balancing threshold 16/32/64) with
 * `repeats` renders each, keeps the fastest in the plan and returns it.  With
 * cache_path, a schedule stored for the same device and batch shape is reused
 * without timing, and a new result is appended.  Synchronises the stream. */
int gsr_batch_tune(gsr_batch* batch, int32_t* status_dev, gsr_stream_t stream, const char* cache_path,
                   int32_t repeats, gsr_schedule* best, float* best_ms);

int64_t gsr_batch_records(const gsr_batch* batch);        /* total Gaussian records */
int64_t gsr_batch_tiles(const gsr_batch* batch);          /* total 16x16 tiles */
int64_t gsr_batch_entry_capacity(const gsr_batch* batch); /* entries the workspace holds */
int64_t gsr_batch_counters_offset(const gsr_batch* batch);/* byte offset of uint32 counters[32] in ws:
                                                             [0] entries, [2] tiles, [3] entries needed,
                                                             [5] / [6] entries / tiles of the fallback,
                                                             [16..31] work-queue heads */
void gsr_batch_destroy(gsr_batch* batch);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): gsr_render
 * with a fixed workspace of GSR_NOALLOC_BYTES that the library holds in a
 * static device array, one per GPU, from the first call on that GPU until the
 * process ends.  The call allocates nothing (no hipMalloc, no allocating
 * library routine); the caller still owns scene, outputs and status_dev, as
 * for gsr_render.  The device current on the calling thread must be the
 * stream's device.
 *   - Sizes: the per-Gaussian and per-tile regions (about 157 B per Gaussian
 *     and 32 B per 16x16 tile) plus 28 B per tile entry must fit in
 *     GSR_NOALLOC_BYTES; a scene and image too large for even one entry is
 *     refused with GSR_ECAPACITY before anything is enqueued.  More entries
 *     than the rest holds is the data-dependent overflow of gsr_render
 *     (GSR_STATUS_OVERFLOW in *status_dev, outputs undefined); it cannot be
 *     cured by a larger workspace here, only by the workspace entry points.
 *   - The array keeps the last call's contents; every call clears what it
 *     needs.  Calls that overlap on one GPU (other streams, other threads)
 *     share that GPU's array and race: serialise them.
 *   - Results equal gsr_render's with the same scene, camera and
 *     configuration (the same kernels run).  A backward is not offered: the
 *     next call overwrites the forward's workspace. */
#define GSR_NOALLOC_BYTES ((size_t)64 << 20)
int gsr_render_noalloc(const gsr_scene* scene, const gsr_camera* cam, const gsr_config* cfg, float* rgb,
                       float* depth, int32_t* count, float* T_final, int32_t* status_dev, gsr_stream_t stream);

/* Element-wise arithmetic probe of the device (diagnostic): for n inputs
 * a[i], b[i] writes out[k*n + i] for k = 0..5:
 *   a/b, sqrt(a), project exp(a), project ln(a) (a >= 1), rint(a), a*b+a. */
int gsr_probe_math(const float* a, const float* b, int32_t n, float* out, gsr_stream_t stream);

const char* gsr_last_error(void);
const char* gsr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
