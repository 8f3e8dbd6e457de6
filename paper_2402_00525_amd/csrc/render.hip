// Render kernels.
//
// k_render_hier: the hierarchical per-pixel resorting of Sec. 3.4 on wave64.
// One workgroup of 256 lanes renders one 16x16 tile; every wavefront owns a
// 16x4 strip of four 4x4 sub-tiles and never synchronises with the other
// wavefronts.  Inside a wavefront:
//   * a 16-lane row owns one 4x4 sub-tile and its tail queue (LDS, 64
//     entries); every batch of 32 list entries is culled against the
//     sub-tile (Algorithm 1), keyed by t_opt along the sub-tile's centre ray,
//     ranked, and merged into the tail; while the tail holds more than 32,
//     its front 16 go to the mid level;
//   * a 4-lane quad owns one 2x2 block and its mid queue (LDS, 8 entries);
//     sub-batches of 4 are culled against the block, keyed along the block's
//     centre ray, ranked with quad shuffles and merged; while the mid queue
//     holds more than 4, its front 4 go to the heads;
//   * every lane owns one pixel and its head queue (registers, K entries);
//     an entry is inserted by (t_opt along the pixel ray, list rank) and the
//     front is blended front to back whenever the head holds more than K.
// Queue keys are (depth bits << 32 | rank in the tile list), a total order,
// so every sort and merge has one result.
//
// k_render_global: the 3DGS order -- each pixel blends its tile's list in
// key order.
//
// k_render_full: the full per-pixel sort (Sec. 3.2) as a reference -- each
// pixel blends every contributor in (t_opt along its ray, id) order.
//
// k_render_window: per-ray resorting (Sec. 3.3) -- each pixel walks its
// tile's 3DGS list and keeps a window of K samples in registers, ordered by
// (t_opt along the pixel ray, list rank); the front is blended whenever the
// window overflows, the rest at the end of the list.
#include "gsr_internal.h"

namespace gsr {

namespace {

// Kernel modes: forward, forward writing blend-id lists, backward, and
// forward counting the evaluations of every level (a work model for the
// render's arithmetic roofline; the counts do not depend on timing).
enum { kFwd = 0, kFwdDebug = 1, kBwd = 2, kFwdCount = 3, kFwdPlain = 4 };

// Whether a blend's colour terms are added at the next blend, so that the
// colour load overlaps the work in between (forward heads of up to 4; the
// extra registers would cost occupancy elsewhere, and kFwdPlain is the
// forward without it).
constexpr bool defer_colour(int K, int MODE) { return MODE != kBwd && MODE != kFwdPlain && K <= 4; }
// Work counters (RenderArgs::work): cull tests and keyed (t_opt) entries at
// the 4x4 and 2x2 levels, alpha tests and keyed entries at the pixels, blends.
enum { kWorkTailTest = 0, kWorkTailKey, kWorkMidTest, kWorkMidKey, kWorkHeadTest, kWorkHeadKey, kWorkBlend, kWorkN };

constexpr int kBatch = 32;
// Backward: per-tile LDS accumulators for the first kAccSlots list entries.
constexpr int kAccSlots = 512;
constexpr int kTailCap = 64;
constexpr int kPop = 16;
constexpr int kMidCap = 8;
constexpr int kMidBatch = 4;

// Value of lane M of this lane's quad (all four lanes active), by a DPP
// quad permutation: a VALU move, no LDS round trip.
template <int M>
__device__ __forceinline__ uint64_t quad_bcast(uint64_t v) {
    constexpr int ctrl = M | (M << 2) | (M << 4) | (M << 6);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, ctrl, 0xf, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), ctrl, 0xf, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ void quad_all(uint64_t v, uint64_t (&out)[4]) {
    out[0] = quad_bcast<0>(v);
    out[1] = quad_bcast<1>(v);
    out[2] = quad_bcast<2>(v);
    out[3] = quad_bcast<3>(v);
}

// Number of entries of sorted arr[0..n) below key.
__device__ __forceinline__ int count_below(const uint64_t* arr, int n, uint64_t key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (arr[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Queues of one wavefront.  Merges are done in place: every lane reads the
// entries it moves into registers, the wavefront synchronises, then writes.
struct WaveQueues {
    uint64_t tkey[4][kTailCap];
    uint32_t tid[4][kTailCap];
    uint64_t nkey[4][kBatch];
    uint32_t nid[4][kBatch];
    uint64_t skey[4][kBatch];
    uint32_t sid[4][kBatch];
    uint64_t mkey[16][kMidCap];
    uint32_t mid[16][kMidCap];
};

// Heads up to 8 keep each slot's Gaussian (forward and backward alike: the
// backward's blend then issues its splat and colour loads without first
// reading the tile list).
constexpr bool head_keeps_ids(int K, int MODE) { return K <= 8; }
// Large forward heads keep their alphas in LDS (one word per lane and slot),
// not in registers: with the keys alone the K = 16 head fits three
// wavefronts per SIMD.  Their keys' low word is then rank << 5 | slot, where
// slot is the LDS word of the entry's alpha, so list ranks must stay below
// kMaxPayloadRank.
constexpr bool head_alpha_in_lds(int K, int MODE) { return K >= 12 && MODE != kBwd; }
constexpr uint32_t kMaxPayloadRank = 1u << 27;

template <int K, int MODE>
struct PixelState {
    float T, C0, C1, C2, D;
    int n;
    bool done;
    // head: keys (t_opt bits << 32 | low word) and alphas, sorted; empty
    // slots hold kInvalidKey, above every real key.  The low word of a key is
    // the entry's rank in the tile list `ids` (its Gaussian is ids[rank]), or
    // the Gaussian id itself when `ids` is null.  Small heads also keep each
    // slot's Gaussian, so that a blend needs no dependent load before its
    // colour load; large heads save those registers and read ids[rank].
    uint64_t hk[K];
    float ha[head_alpha_in_lds(K, MODE) ? 1 : K];   // alphas in registers (else in pay)
    uint32_t hid[head_keeps_ids(K, MODE) ? K : 1];  // the slots' Gaussians (small heads only)
    int hn;
    float* pay;  // large heads: this lane's alpha of LDS slot j at pay[64 j]
    const uint32_t* ids;
    uint32_t n_ids;  // Gaussians: ids at or above are read as 0
    // backward only: dL/dC and the forward's final colour (background included)
    float g0, g1, g2, R0, R1, R2;
    float px, py;
    // forward: the last blend's colour terms, added at the next blend (or
    // at the end) so that its colour load is in flight meanwhile
    float4 pe;
    float pa, pT;
    // backward: the last blend's gradient terms, added when the pixel's quad
    // next meets (quad_flush), so that equal ranks of a quad add once
    float gv[9];
    uint32_t grank, gid;
    bool gpend;
    // debug: sort error so far and the last blended depth
    float dl, tl;
};

// Adds the pending blend's colour: C += (c alpha) T, exactly as if done at
// its blend (the sums stay in blend order).  Zero terms while none is pending.
template <int K, int MODE>
__device__ __forceinline__ void flush_colour(PixelState<K, MODE>& s) {
    if (!defer_colour(K, MODE)) return;
    s.C0 = fmaf(s.pe.x * s.pa, s.pT, s.C0);
    s.C1 = fmaf(s.pe.y * s.pa, s.pT, s.C1);
    s.C2 = fmaf(s.pe.z * s.pa, s.pT, s.C2);
}

template <int K, int MODE>
__device__ __forceinline__ void init_colour(PixelState<K, MODE>& s) {
    s.C0 = s.C1 = s.C2 = 0.0f;
    s.pe = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    s.pa = 0.0f;
    s.pT = 0.0f;
}

template <int M>
__device__ __forceinline__ float quad_bcast_f(float v) {
    constexpr int ctrl = M | (M << 2) | (M << 4) | (M << 6);
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xf, 0xf, false));
}
template <int M>
__device__ __forceinline__ uint32_t quad_bcast_u(uint32_t v) {
    constexpr int ctrl = M | (M << 2) | (M << 4) | (M << 6);
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xf, 0xf, false);
}

// Adds the 9 gradient terms of one blend: into the tile's LDS accumulators
// (slot = rank in the tile list; the backward always has them) when the rank
// has a slot, else to global memory.
__device__ __forceinline__ void add_grad(const RenderArgs& a, float* acc, uint32_t rank, uint32_t id, int c, float v) {
    if (rank < (uint32_t)kAccSlots)
        atomicAdd(acc + c * kAccSlots + rank, v);
    else
        atomicAdd(a.grad2d + 9 * (size_t)id + c, v);
}

// Adds the pending gradient terms of the four lanes of this quad (all four
// must be active): lanes with the same list rank are summed by DPP and added
// once by the lowest of them, so a quad blending one Gaussian costs one set
// of atomics instead of four.
template <int K, int MODE>
__device__ __forceinline__ void quad_flush(const RenderArgs& a, PixelState<K, MODE>& s, float* acc) {
    if (MODE != kBwd) return;
    if (__ballot(s.gpend) == 0ull) return;
    const uint32_t r = s.gpend ? s.grank : 0xffffffffu;
    const uint32_t rq[4] = {quad_bcast_u<0>(r), quad_bcast_u<1>(r), quad_bcast_u<2>(r), quad_bcast_u<3>(r)};
    const int pl = (int)(threadIdx.x & 3u);
    bool leader = s.gpend;
#pragma unroll
    for (int m = 0; m < 4; ++m) leader = leader && !(m < pl && rq[m] == r);
    float sum[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) {
        const float v0 = quad_bcast_f<0>(s.gv[c]), v1 = quad_bcast_f<1>(s.gv[c]);
        const float v2 = quad_bcast_f<2>(s.gv[c]), v3 = quad_bcast_f<3>(s.gv[c]);
        float t = rq[0] == r ? v0 : 0.0f;
        t = t + (rq[1] == r ? v1 : 0.0f);
        t = t + (rq[2] == r ? v2 : 0.0f);
        t = t + (rq[3] == r ? v3 : 0.0f);
        sum[c] = t;
    }
    // Every component is added, zero or not: a branch per component cost
    // more than the zero adds.
    if (leader && r < (uint32_t)kAccSlots) {
#pragma unroll
        for (int c = 0; c < 9; ++c) atomicAdd(acc + c * kAccSlots + r, sum[c]);
    } else if (leader) {
#pragma unroll
        for (int c = 0; c < 9; ++c) atomicAdd(a.grad2d + 9 * (size_t)s.gid + c, sum[c]);
    }
    s.gpend = false;
}

template <int K, int MODE>
__device__ __forceinline__ void blend_one(const RenderArgs& a, PixelState<K, MODE>& s, int pix, uint32_t id,
                                          float alpha, float t, uint32_t rank, float* acc) {
    if (s.done) return;
    const float Tn = s.T * (1.0f - alpha);
    if (Tn < kTMin) {
        s.done = true;
        return;
    }
    const float4 e = a.col[id];
    if (!defer_colour(K, MODE)) {
        s.C0 = fmaf(e.x * alpha, s.T, s.C0);
        s.C1 = fmaf(e.y * alpha, s.T, s.C1);
        s.C2 = fmaf(e.z * alpha, s.T, s.C2);
    } else {
        flush_colour(s);
        s.pe = e;
        s.pa = alpha;
        s.pT = s.T;
    }
    s.D = fmaf(t * alpha, s.T, s.D);
    if (MODE == kFwdDebug) {
        if (s.n < a.max_k) a.blend_ids[(size_t)pix * a.max_k + s.n] = (int32_t)id;
        // sort error (Sec. 3.3): consecutive blends out of order add their
        // difference in t_opt
        if (s.n > 0 && s.tl > t) s.dl = s.dl + (s.tl - t);
        s.tl = t;
    }
    if (MODE == kBwd) {
        // Sec. 3.5, front to back: everything behind this Gaussian contributes
        // C - C_i (C_i includes it), and dC/dalpha = c T - (C - C_i + T_N bg) / (1 - alpha),
        // where C + T_N bg is the forward's output R.
        const float w = alpha * s.T;
        const float inv = 1.0f / (1.0f - alpha);
        const float ga = s.g0 * (e.x * s.T - (s.R0 - s.C0) * inv) + s.g1 * (e.y * s.T - (s.R1 - s.C1) * inv) +
                         s.g2 * (e.z * s.T - (s.R2 - s.C2) * inv);
        if (s.gpend)  // not flushed since the last blend: add those terms directly
            for (int c = 0; c < 9; ++c) add_grad(a, acc, s.grank, s.gid, c, s.gv[c]);
        s.gpend = true;
        s.grank = rank;
        s.gid = id;
        s.gv[6] = s.g0 * w;
        s.gv[7] = s.g1 * w;
        s.gv[8] = s.g2 * w;
        // 2D mean, conic and opacity from the packed splat (one cache line)
        const float4 p0 = a.pk[4 * (size_t)id], p1 = a.pk[4 * (size_t)id + 1];
        const float2 m = make_float2(p0.x, p0.y);
        const float4 c = make_float4(p0.z, p0.w, p1.x, p1.y);
        const float dx = m.x - s.px, dy = m.y - s.py;
        const float pw = power_at_offset(c.x, c.y, c.z, dx, dy);
        const float G = exp_cw(pw);
        const bool live = c.w * G < kAlphaMax;  // alpha not clamped: it depends on the Gaussian
        const float gp = ga * alpha;            // d alpha / d power = o G
        s.gv[0] = live ? gp * (-c.x * dx - c.y * dy) : 0.0f;
        s.gv[1] = live ? gp * (-c.z * dy - c.y * dx) : 0.0f;
        s.gv[2] = live ? gp * (-0.5f * dx * dx) : 0.0f;
        s.gv[3] = live ? gp * (-dx * dy) : 0.0f;
        s.gv[4] = live ? gp * (-0.5f * dy * dy) : 0.0f;
        s.gv[5] = live ? ga * G : 0.0f;
    }
    s.n += 1;
    s.T = Tn;
}

// List rank of a head key (see PixelState::hk).
template <int K, int MODE>
__device__ __forceinline__ uint32_t key_rank(uint64_t key) {
    return head_alpha_in_lds(K, MODE) ? (uint32_t)key >> 5 : (uint32_t)key;
}

// Gaussian of a head key.
template <int K, int MODE>
__device__ __forceinline__ uint32_t head_id(const PixelState<K, MODE>& s, uint64_t key) {
    const uint32_t lo = key_rank<K, MODE>(key);
    const uint32_t id = s.ids ? s.ids[lo] : lo;
    return id < s.n_ids ? id : 0u;
}

// Gaussian and alpha of the front slot.
template <int K, int MODE>
__device__ __forceinline__ uint32_t front_id(const PixelState<K, MODE>& s) {
    if (head_keeps_ids(K, MODE)) return s.hid[0];
    return head_id(s, s.hk[0]);
}
template <int K, int MODE>
__device__ __forceinline__ float front_alpha(const PixelState<K, MODE>& s) {
    if (head_alpha_in_lds(K, MODE)) return s.pay[64 * ((uint32_t)s.hk[0] & 31u)];
    return s.ha[0];
}

// Remove the front of the head and blend it.
template <int K, int MODE>
__device__ __forceinline__ void head_pop_blend(const RenderArgs& a, PixelState<K, MODE>& s, int pix, float* acc) {
    const uint64_t k0 = s.hk[0];
    const float a0 = front_alpha(s);
    const uint32_t i0 = front_id(s);
#pragma unroll
    for (int i = 0; i + 1 < K; ++i) {
        s.hk[i] = s.hk[i + 1];
        if (!head_alpha_in_lds(K, MODE)) s.ha[i] = s.ha[i + 1];
        if (head_keeps_ids(K, MODE)) s.hid[i] = s.hid[i + 1];
    }
    s.hk[K - 1] = kInvalidKey;
    if (!head_alpha_in_lds(K, MODE)) s.ha[K - 1] = 0.0f;
    s.hn -= 1;
    blend_one<K, MODE>(a, s, pix, i0, a0, depth_from_bits((uint32_t)(k0 >> 32)), key_rank<K, MODE>(k0), acc);
}

// Insertion into the sorted head (s.hn < K on entry, so the last slot is
// empty).  With c_i = (slot i holds a key below the entry), true exactly for
// the slots before the entry's place, slot i keeps its key if c_i, takes the
// entry if c_(i-1) (or i = 0) and not c_i, and else its predecessor's.  Every
// slot takes its new value by selects, never by a store at a computed slot,
// so the head stays in registers at every K.  `key` is in head form (see
// head_push); a large head puts the alpha into LDS word s.hn, the first free
// one (entries leave only in the drain, after the last insertion).
template <int K, int MODE>
__device__ __forceinline__ void head_insert(PixelState<K, MODE>& s, uint64_t key, uint32_t id, float alpha) {
    if (head_alpha_in_lds(K, MODE)) {
        s.pay[64 * s.hn] = alpha;
        key |= (uint64_t)(uint32_t)s.hn;
    }
    bool c[K];
#pragma unroll
    for (int i = 0; i < K; ++i) c[i] = s.hk[i] < key;
    // from the back, so that slot i - 1 still holds its old entry
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        const bool take = i == 0 || c[i - 1];
        const uint64_t pk = i > 0 ? s.hk[i - 1] : 0ull;
        s.hk[i] = c[i] ? s.hk[i] : (take ? key : pk);
        if (!head_alpha_in_lds(K, MODE)) {
            const float pa = i > 0 ? s.ha[i - 1] : 0.0f;
            s.ha[i] = c[i] ? s.ha[i] : (take ? alpha : pa);
        }
        if (head_keeps_ids(K, MODE)) {
            const uint32_t pi = i > 0 ? s.hid[i - 1] : 0u;
            s.hid[i] = c[i] ? s.hid[i] : (take ? id : pi);
        }
    }
    s.hn += 1;
}

// Push into a head of capacity K, blending the front whenever it would hold
// more than K (the k-buffer rule of Sec. 3.3): while it is not full the entry
// is inserted; when it is full the smallest of the K + 1 (the entry or the
// front) is blended and the other K stay sorted, in one pass of selects:
// with c_i = (slot i + 1 holds a key below the entry) and c_(-1) = (the front
// is below the entry), slot i takes slot i + 1's key if c_i, the entry if
// c_(i-1) and not c_i, and else keeps its own.  `key` = t_opt bits << 32 |
// list rank; a large head stores rank << 5 | (its alpha's LDS word), the
// word the blended front frees.
template <int K, int MODE>
__device__ __forceinline__ void head_push(const RenderArgs& a, PixelState<K, MODE>& s, int pix, uint64_t key,
                                          uint32_t id, float alpha, float* acc) {
    if (head_alpha_in_lds(K, MODE)) key = (key & 0xffffffff00000000ull) | ((key & 0xffffffffull) << 5);
    if (s.hn < K) {
        head_insert<K, MODE>(s, key, id, alpha);
        return;
    }
    const uint64_t k0 = s.hk[0];
    const bool front_goes = k0 < key;
    float a0;
    if (head_alpha_in_lds(K, MODE)) {
        const uint32_t w = (uint32_t)k0 & 31u;
        a0 = s.pay[64 * w];
        if (front_goes) {
            s.pay[64 * w] = alpha;
            key |= (uint64_t)w;
        }
    } else {
        a0 = s.ha[0];
    }
    const uint32_t bid = front_goes ? front_id(s) : id;
    bool c[K];
#pragma unroll
    for (int i = 0; i + 1 < K; ++i) c[i] = s.hk[i + 1] < key;
    c[K - 1] = false;
    // from the front, so that slot i + 1 still holds its old entry
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const bool take = i == 0 ? front_goes : c[i - 1];
        const uint64_t nk = i + 1 < K ? s.hk[i + 1] : 0ull;
        s.hk[i] = c[i] ? nk : (take ? key : s.hk[i]);
        if (!head_alpha_in_lds(K, MODE)) {
            const float na = i + 1 < K ? s.ha[i + 1] : 0.0f;
            s.ha[i] = c[i] ? na : (take ? alpha : s.ha[i]);
        }
        if (head_keeps_ids(K, MODE)) {
            const uint32_t ni = i + 1 < K ? s.hid[i + 1] : 0u;
            s.hid[i] = c[i] ? ni : (take ? id : s.hid[i]);
        }
    }
    const uint64_t bk = front_goes ? k0 : key;
    blend_one<K, MODE>(a, s, pix, bid, front_goes ? a0 : alpha, depth_from_bits((uint32_t)(bk >> 32)),
                       key_rank<K, MODE>(bk), acc);
}

// DEEP: the variant for views of few, deep tiles (one wavefront per SIMD or
// fewer, so nothing else hides a wavefront's memory latency): every splat a
// level will read is loaded ahead -- the next tail batch's while the current
// one is merged, all of a tail pop's mid sub-batches and all of a mid pop's
// head entries at once -- in registers that the default variant cannot spare
// without losing occupancy.  The arithmetic and the order are the same.
template <int K, int MODE, bool DEEP = false>
struct HierCtx {
    const RenderArgs& a;
    WaveQueues& q;
    int row, j, quad, pl, gq, lane;
    int px, py, pix;
    bool quad_ok, pix_ok;
    float Q0, Q1, Q2, Q3;
    float3 dQ, dP;
    // mid queue state (uniform over the quad)
    int ms, mn;
    PixelState<K, MODE> st;
    float* acc;  // backward: the tile's LDS gradient accumulators
    uint32_t work[kWorkN];  // kFwdCount only

    __device__ HierCtx(const RenderArgs& a_, WaveQueues& q_) : a(a_), q(q_) {}

    // Head level: the c entries of this quad's mid buffer from position ms0.
    __device__ void push_head(int c, int ms0) {
        // The backward keeps the whole quad in the loop: its gradient terms
        // are combined across the quad after every entry.
        if (MODE != kBwd && (st.done || !pix_ok)) return;
        if (DEEP) {
            push_head_all(c, ms0);
            return;
        }
        uint32_t idn = q.mid[gq][ms0];
        idn = idn < a.n ? idn : 0u;
        Splat gn = load_packed(a.pk, idn);  // the next entry's splat, loaded one entry ahead
        for (int e = 0; e < c; ++e) {
            const uint64_t mk = q.mkey[gq][ms0 + e];
            const uint32_t id = idn;
            const Splat g = gn;
            if (e + 1 < c) {
                idn = q.mid[gq][ms0 + e + 1];
                idn = idn < a.n ? idn : 0u;
                gn = load_packed(a.pk, idn);
            }
            if (!st.done && pix_ok) {
                float alpha;
                if (MODE == kFwdCount) ++work[kWorkHeadTest];
                if (pixel_alpha(g, (float)px, (float)py, alpha)) {
                    if (MODE == kFwdCount) ++work[kWorkHeadKey];
                    const float t = t_opt(g, dP);
                    head_push<K, MODE>(a, st, pix, ((uint64_t)depth_bits(t) << 32) | (mk & 0xffffffffull), id, alpha,
                                       acc);
                }
            }
            quad_flush(a, st, acc);
        }
    }

    // push_head with every entry's splat loaded up front (DEEP; forward).
    __device__ void push_head_all(int c, int ms0) {
        uint32_t ids[kMidBatch];
        Splat gs[kMidBatch];
#pragma unroll
        for (int e = 0; e < kMidBatch; ++e) {
            if (e < c) {
                uint32_t id = q.mid[gq][ms0 + e];
                ids[e] = id < a.n ? id : 0u;
                gs[e] = load_packed(a.pk, ids[e]);
            }
        }
#pragma unroll
        for (int e = 0; e < kMidBatch; ++e) {
            if (e < c && !st.done) {
                const uint64_t mk = q.mkey[gq][ms0 + e];
                float alpha;
                if (MODE == kFwdCount) ++work[kWorkHeadTest];
                if (pixel_alpha(gs[e], (float)px, (float)py, alpha)) {
                    if (MODE == kFwdCount) ++work[kWorkHeadKey];
                    const float t = t_opt(gs[e], dP);
                    head_push<K, MODE>(a, st, pix, ((uint64_t)depth_bits(t) << 32) | (mk & 0xffffffffull), ids[e],
                                       alpha, acc);
                }
            }
        }
    }

    // Mid level: a chunk of cl <= kPop tail entries of row `row`, from
    // position cs, in sub-batches of kMidBatch (one entry per lane of a quad).
    __device__ void push_mid(int cs, int cl) {
        if (!quad_ok) return;
        if (DEEP) {
            // every sub-batch's tail entry and splat loaded up front (the
            // tail queue does not change during a pop)
            uint64_t dtk[kPop / kMidBatch];
            uint32_t did[kPop / kMidBatch];
            Splat dg[kPop / kMidBatch];
#pragma unroll
            for (int sb = 0; sb < kPop / kMidBatch; ++sb) {
                const int idx = sb * kMidBatch + pl;
                dtk[sb] = kInvalidKey;
                did[sb] = 0u;
                if (idx < cl) {
                    dtk[sb] = q.tkey[row][cs + idx];
                    const uint32_t id = q.tid[row][cs + idx];
                    did[sb] = id < a.n ? id : 0u;
                    dg[sb] = load_packed(a.pk, did[sb]);
                }
            }
#pragma unroll
            for (int sb = 0; sb < kPop / kMidBatch; ++sb) {
                if (sb * kMidBatch >= cl) break;
                mid_sub_batch(cl, sb * kMidBatch, dtk[sb], did[sb], dg[sb]);
            }
            return;
        }
        for (int r0 = 0; r0 < cl; r0 += kMidBatch) {
            const int idx = r0 + pl;
            uint64_t tk = kInvalidKey;
            uint32_t id = 0;
            Splat g;
            if (idx < cl) {
                tk = q.tkey[row][cs + idx];
                id = q.tid[row][cs + idx];
                id = id < a.n ? id : 0u;
                g = load_packed(a.pk, id);
            }
            mid_sub_batch(cl, r0, tk, id, g);
        }
    }

    // One sub-batch: lane pl's tail entry r0 + pl (tail key tk, Gaussian id,
    // splat g; none when r0 + pl >= cl) is culled against the quad and keyed
    // along its ray, merged into the quad's mid queue, and the queue pops
    // into the heads when it holds more than kMidCap - kMidBatch.
    __device__ __forceinline__ void mid_sub_batch(int cl, int r0, uint64_t tk, uint32_t id, const Splat& g) {
        const int idx = r0 + pl;
        uint64_t key = kInvalidKey;
        if (idx < cl) {
            if (MODE == kFwdCount) ++work[kWorkMidTest];
            if ((a.flags & kAblateHierCull) || block_clears(g, Q0, Q1, Q2, Q3)) {
                if (MODE == kFwdCount) ++work[kWorkMidKey];
                key = ((uint64_t)depth_bits(t_opt(g, dQ)) << 32) | (tk & 0xffffffffull);
            }
        }
        uint64_t qk[4];
        quad_all(key, qk);
        int rnk = 0, nnew = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            rnk += qk[m] < key ? 1 : 0;
            nnew += qk[m] != kInvalidKey ? 1 : 0;
        }
        // The queue holds mn <= 4 entries from ms: one per lane of the quad.
        uint64_t ek = kInvalidKey;
        uint32_t eid = 0;
        if (pl < mn) {
            ek = q.mkey[gq][ms + pl];
            eid = q.mid[gq][ms + pl];
        }
        uint64_t qe[4];
        quad_all(ek, qe);
        wave_lds_sync();
        if (pl < mn) {
            int c = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) c += qk[m] < ek ? 1 : 0;
            q.mkey[gq][pl + c] = ek;
            q.mid[gq][pl + c] = eid;
        }
        if (key != kInvalidKey) {
            int c = 0;
#pragma unroll
            for (int m = 0; m < 4; ++m) c += (m < mn && qe[m] < key) ? 1 : 0;
            q.mkey[gq][rnk + c] = key;
            q.mid[gq][rnk + c] = id;
        }
        wave_lds_sync();
        ms = 0;
        mn += nnew;
        // at most one pop: the queue held at most kMidBatch before this
        // sub-batch of at most kMidBatch (kMidCap = 2 kMidBatch)
        if (mn > kMidCap - kMidBatch) {
            push_head(kMidBatch, ms);
            ms += kMidBatch;
            mn -= kMidBatch;
        }
    }
};

// One wavefront renders one 16x4 strip (`strip` = 0..3) of four 4x4 sub-tiles
// of tile `tile` (image tile index); its list is ranges[range_tile].  Returns
// the number of list entries the wavefront read before its pixels finished.
// The entry list a tile is rendered from (ranks are positions in it).
struct TileList {
    const uint32_t* ids;
    uint32_t len;    // entries in ids
    uint32_t n_all;  // entries of the tile
    bool truncated;  // ids is a prefix of the tile's order
    bool skip;       // nothing to do for this tile in this pass
};

__device__ __forceinline__ TileList tile_list(const RenderArgs& a, int t) {
    const uint32_t rb = a.ranges[2 * t], re = a.ranges[2 * t + 1];
    TileList L{a.vals + rb, re - rb, re - rb, false, false};
    if (a.list_mode == kListFull) return L;
    if (a.list_mode == kListFlagged && a.tile_flag[t] == 0u) {
        L.skip = true;
        return L;
    }
    L.ids = a.pre_vals + rb;
    L.len = a.pre_len[t];
    L.truncated = a.list_mode == kListPrefix && L.len < L.n_all;
    return L;
}

template <int K, int MODE, bool DEEP = false>
__device__ __forceinline__ uint32_t render_strip(const RenderArgs& a, int tile, int range_tile, int strip,
                                                 WaveQueues& q, float* acc, float* pay) {
    const int lane = threadIdx.x & 63, wave = strip;
    const DevCam& cam = a.cam;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    HierCtx<K, MODE, DEEP> h(a, q);
    h.acc = acc;
    if (MODE == kFwdCount)
        for (int w = 0; w < kWorkN; ++w) h.work[w] = 0u;
    h.lane = lane;
    h.row = lane >> 4;
    h.j = lane & 15;
    h.quad = h.j >> 2;
    h.pl = h.j & 3;
    h.gq = h.row * 4 + h.quad;
    const int sx0 = tx * 16 + h.row * 4, sy0 = ty * 16 + wave * 4;
    const int qx0 = sx0 + 2 * (h.quad & 1), qy0 = sy0 + 2 * (h.quad >> 1);
    h.px = qx0 + (h.pl & 1);
    h.py = qy0 + (h.pl >> 1);
    const bool sub_ok = sx0 < cam.W && sy0 < cam.H;
    h.quad_ok = qx0 < cam.W && qy0 < cam.H;
    h.pix_ok = h.px < cam.W && h.py < cam.H;
    h.pix = h.py * cam.W + h.px;
    const float S0 = (float)sx0, S1 = (float)min(sx0 + 3, cam.W - 1);
    const float S2 = (float)sy0, S3 = (float)min(sy0 + 3, cam.H - 1);
    h.Q0 = (float)qx0;
    h.Q1 = (float)min(qx0 + 1, cam.W - 1);
    h.Q2 = (float)qy0;
    h.Q3 = (float)min(qy0 + 1, cam.H - 1);
    const float3 dS = cam_ray(cam, 0.5f * (S0 + S1), 0.5f * (S2 + S3));
    h.dQ = cam_ray(cam, 0.5f * (h.Q0 + h.Q1), 0.5f * (h.Q2 + h.Q3));
    h.dP = cam_ray(cam, (float)h.px, (float)h.py);
    h.st.T = 1.0f;
    init_colour(h.st);
    h.st.D = 0.0f;
    h.st.gpend = false;
    h.st.dl = h.st.tl = 0.0f;
    h.st.n = 0;
    h.st.done = !h.pix_ok;
    h.st.hn = 0;
    h.st.px = (float)h.px;
    h.st.py = (float)h.py;
    if (MODE == kBwd && h.pix_ok) {
        const size_t P = (size_t)cam.W * cam.H, p = (size_t)h.pix;
        h.st.g0 = a.dL[p];
        h.st.g1 = a.dL[P + p];
        h.st.g2 = a.dL[2 * P + p];
        h.st.R0 = a.rgb_in[p];
        h.st.R1 = a.rgb_in[P + p];
        h.st.R2 = a.rgb_in[2 * P + p];
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        h.st.hk[i] = kInvalidKey;
        if (!head_alpha_in_lds(K, MODE)) h.st.ha[i] = 0.0f;
        if (head_keeps_ids(K, MODE)) h.st.hid[i] = 0u;
    }
    h.ms = 0;
    h.mn = 0;
    int ts = 0, tn = 0;  // tail state, uniform over the row
    const int row = h.row, j = h.j;

    // The tile's list: entries list[0 .. end), rank = position in the list.
    const TileList tl = tile_list(a, range_tile);
    if (tl.skip) return 0u;
    const uint32_t* list = tl.ids;
    h.st.ids = list;
    h.st.n_ids = a.n;
    h.st.pay = pay + lane;
    // A truncated prefix is walked in whole batches only: the last, partial
    // batch of a prefix is not the batch the whole list has at that place,
    // and the pops that follow it could differ.  The strip is then flagged
    // unless its pixels finished within the whole batches.
    uint32_t end = tl.truncated ? (tl.len & ~(uint32_t)(kBatch - 1)) : tl.len;
    if (head_alpha_in_lds(K, MODE) && end > kMaxPayloadRank) end = kMaxPayloadRank;  // ranks fit 27 bits
    const bool truncated = tl.truncated;
    const uint32_t begin = 0;
    uint32_t b0 = begin;
    // ids of the next batch, loaded one batch ahead (DEEP: ids two batches
    // ahead, splats of the next batch one batch ahead)
    uint32_t nx[2], nx2[2];
    Splat gnext[2];
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        const uint32_t e = b0 + (uint32_t)(j + 16 * hh);
        nx[hh] = e < end ? list[e] : 0u;
        if (DEEP) {
            if (e < end) gnext[hh] = load_packed(a.pk, nx[hh] < a.n ? nx[hh] : 0u);
            const uint32_t e2 = e + kBatch;
            nx2[hh] = e2 < end ? list[e2] : 0u;
        }
    }
    for (; b0 < end; b0 += kBatch) {
        const uint64_t live = __ballot(!h.st.done);
        if (live == 0) break;
        uint32_t cur[2] = {nx[0], nx[1]};
        Splat gcur[2];
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const uint32_t e = b0 + kBatch + (uint32_t)(j + 16 * hh);
            if (DEEP) {
                gcur[hh] = gnext[hh];
                nx[hh] = nx2[hh];
                if (e < end) gnext[hh] = load_packed(a.pk, nx[hh] < a.n ? nx[hh] : 0u);
                const uint32_t e2 = e + kBatch;
                nx2[hh] = e2 < end ? list[e2] : 0u;
            } else {
                nx[hh] = e < end ? list[e] : 0u;
            }
        }
        const bool row_live = sub_ok && ((live >> (row * 16)) & 0xffffull) != 0;
        if (!row_live) continue;
        // Cull against the sub-tile and key along its centre ray.
        uint64_t k2[2] = {kInvalidKey, kInvalidKey};
        uint32_t i2[2] = {0, 0};
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const uint32_t e = b0 + (uint32_t)(j + 16 * hh);
            if (e < end) {
                uint32_t id = cur[hh];
                id = id < a.n ? id : 0u;
                i2[hh] = id;
                const Splat g = DEEP ? gcur[hh] : load_packed(a.pk, id);
                if (MODE == kFwdCount) ++h.work[kWorkTailTest];
                if ((a.flags & kAblateHierCull) || block_clears(g, S0, S1, S2, S3)) {
                    if (MODE == kFwdCount) ++h.work[kWorkTailKey];
                    k2[hh] = ((uint64_t)depth_bits(t_opt(g, dS)) << 32) | (uint64_t)(e - begin);
                }
            }
            q.nkey[row][j + 16 * hh] = k2[hh];
            q.nid[row][j + 16 * hh] = i2[hh];
        }
        const uint64_t v0 = __ballot(k2[0] != kInvalidKey), v1 = __ballot(k2[1] != kInvalidKey);
        const int nv = __popcll((v0 >> (row * 16)) & 0xffffull) + __popcll((v1 >> (row * 16)) & 0xffffull);
        wave_lds_sync();
        // Rank within the batch, then scatter into sorted order.
        int r2[2] = {0, 0};
        for (int m = 0; m < kBatch; ++m) {
            const uint64_t km = q.nkey[row][m];
            r2[0] += km < k2[0] ? 1 : 0;
            r2[1] += km < k2[1] ? 1 : 0;
        }
#pragma unroll
        for (int hh = 0; hh < 2; ++hh)
            if (k2[hh] != kInvalidKey) {
                q.skey[row][r2[hh]] = k2[hh];
                q.sid[row][r2[hh]] = i2[hh];
            }
        wave_lds_sync();
        // Merge with the tail (both sorted, keys distinct; tn <= 32 entries
        // from ts, two per lane) in place from position 0.
        uint64_t ek[2] = {kInvalidKey, kInvalidKey};
        uint32_t eid[2] = {0, 0};
        int pe[2] = {0, 0}, pn[2] = {0, 0};
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int idx = j + 16 * hh;
            if (idx < tn) {
                ek[hh] = q.tkey[row][ts + idx];
                eid[hh] = q.tid[row][ts + idx];
                pe[hh] = idx + count_below(q.skey[row], nv, ek[hh]);
            }
            if (k2[hh] != kInvalidKey) pn[hh] = r2[hh] + count_below(&q.tkey[row][ts], tn, k2[hh]);
        }
        wave_lds_sync();
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            if (j + 16 * hh < tn) {
                q.tkey[row][pe[hh]] = ek[hh];
                q.tid[row][pe[hh]] = eid[hh];
            }
            if (k2[hh] != kInvalidKey) {
                q.tkey[row][pn[hh]] = k2[hh];
                q.tid[row][pn[hh]] = i2[hh];
            }
        }
        wave_lds_sync();
        ts = 0;
        tn += nv;
        while (tn > kTailCap - kBatch) {
            h.push_mid(ts, kPop);
            ts += kPop;
            tn -= kPop;
        }
    }
    // A prefix that ran out while pixels of this strip are still live cannot
    // decide the tile: flag it for the full list.
    if (truncated && b0 >= end && __ballot(!h.st.done) != 0ull) {
        if (lane == 0) a.tile_flag[range_tile] = tl.n_all;  // same value from every strip
    }
    // Drain: the tail in chunks, then the mid queues, then the heads.
    {
        const uint64_t live = __ballot(!h.st.done);
        const bool row_live = sub_ok && ((live >> (row * 16)) & 0xffffull) != 0;
        if (row_live) {
            while (tn > 0) {
                const int c = tn < kPop ? tn : kPop;
                h.push_mid(ts, c);
                ts += c;
                tn -= c;
            }
            if (h.quad_ok) {
                while (h.mn > 0) {
                    const int c = h.mn < kMidBatch ? h.mn : kMidBatch;
                    h.push_head(c, h.ms);
                    h.ms += c;
                    h.mn -= c;
                }
            }
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (h.st.hn > 0) head_pop_blend<K, MODE>(a, h.st, h.pix, acc);
                quad_flush(a, h.st, acc);
            }
        }
    }
    flush_colour(h.st);
    if (MODE != kBwd && h.pix_ok) {
        const size_t P = (size_t)cam.W * cam.H;
        const size_t p = (size_t)h.pix;
        a.rgb[p] = h.st.C0 + h.st.T * a.bg0;
        a.rgb[P + p] = h.st.C1 + h.st.T * a.bg1;
        a.rgb[2 * P + p] = h.st.C2 + h.st.T * a.bg2;
        a.depth[p] = h.st.D;
        a.count[p] = h.st.n;
        a.T[p] = h.st.T;
        if (MODE == kFwdDebug) {
            for (int k = h.st.n; k < a.max_k; ++k) a.blend_ids[p * a.max_k + k] = -1;
            if (a.delta) a.delta[p] = h.st.dl;
        }
    }
    if (MODE == kFwdCount) {
        h.work[kWorkBlend] = h.pix_ok ? (uint32_t)h.st.n : 0u;
        for (int w = 0; w < kWorkN; ++w) {
            uint32_t v = h.work[w];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o);
            if (lane == 0 && v) atomicAdd(a.work + w, (unsigned long long)v);
        }
    }
    return (b0 < end ? b0 : end) - begin;
}

template <int K, int MODE>
__global__ __launch_bounds__(256, K <= 4 ? 3 : 2) void k_render_hier(RenderArgs a) {
    __shared__ WaveQueues s_q[4];
    __shared__ float s_pay[head_alpha_in_lds(K, MODE) ? 4 * 64 * K : 1];
    __shared__ uint32_t s_consumed[4];
    __shared__ float s_acc[MODE == kBwd ? 9 * kAccSlots : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (MODE == kBwd) {
        // The workspace must hold the forward of this scene, camera and
        // configuration (the same decision for every thread of the grid).
        if (a.fp) {
            bool same = true;
#pragma unroll
            for (int k = 0; k < kFingerprintWords; ++k) same = same && a.fp[k] == a.fp_expect[k];
            if (!same) {
                if (blockIdx.x == 0 && threadIdx.x == 0 && a.status) atomicOr(a.status, kStatusMismatch);
                return;
            }
        }
        for (int k = threadIdx.x; k < 9 * kAccSlots; k += 256) s_acc[k] = 0.0f;
        __syncthreads();
    }
    const uint32_t c = render_strip<K, MODE>(a, blockIdx.x, blockIdx.x, wave, s_q[wave],
                                             MODE == kBwd ? s_acc : nullptr, s_pay + wave * 64 * K);
    if (lane == 0) s_consumed[wave] = c;
    __syncthreads();
    if (MODE != kBwd && threadIdx.x == 0) {
        uint32_t m = s_consumed[0];
        for (int w = 1; w < 4; ++w) m = s_consumed[w] > m ? s_consumed[w] : m;
        if (m) atomicAdd(a.counters + 1, m);
    }
    if (MODE == kBwd) {
        // One global atomic per (tile, Gaussian, component) instead of one per blend.
        const TileList tl = tile_list(a, blockIdx.x);
        const uint32_t* list = tl.ids;
        const uint32_t n_list = tl.skip ? 0u : tl.len;
        const uint32_t len = n_list < (uint32_t)kAccSlots ? n_list : (uint32_t)kAccSlots;
        for (uint32_t r = threadIdx.x; r < len; r += 256) {
            uint32_t id = list[r];
            id = id < a.n ? id : 0u;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const float v = s_acc[k * kAccSlots + r];
                if (v != 0.0f) atomicAdd(a.grad2d + 9 * (size_t)id + k, v);
            }
        }
    }
}

// The forward with one wavefront per workgroup: a strip's queues are its
// own, so a finished wavefront frees its slot without waiting for the other
// strips of its tile.  Workgroup b renders strip (b mod 32) / 8 of tile
// 8 (b / 32) + b mod 8, so that the four strips of a tile run on one XCD
// (workgroups are dealt to the eight XCDs round robin) and share its L2.
// The entries a tile consumed (the most any of its strips read) are added
// to counters[1] by the tile's last strip, through two per-tile words after
// the flags (zeroed with them); the strips of a tile share an XCD, so their
// atomics meet in one L2.
template <int K, int MODE, bool DEEP>
__global__ __launch_bounds__(64) void k_render_hier1(RenderArgs a) {
    __shared__ WaveQueues s_q;
    __shared__ float s_pay[head_alpha_in_lds(K, MODE) ? 64 * K : 1];
    const uint32_t b = blockIdx.x, g = b / 32u, r = b % 32u;
    const int strip = (int)(r / 8u), tile = (int)(g * 8u + r % 8u);
    const int n_tiles = a.cam.tiles_x * a.cam.tiles_y;
    if (tile >= n_tiles) return;
    const uint32_t c = render_strip<K, MODE, DEEP>(a, tile, tile, strip, s_q, nullptr, s_pay);
    if (threadIdx.x == 0) {
        uint32_t* used = a.tile_flag + n_tiles;
        uint32_t* done = used + n_tiles;
        // The maximum is in place before this strip counts itself done: the
        // count waits for the returned value (no fence, which would write
        // back the L2).
        const uint32_t prev = atomicMax(&used[tile], c);
        asm volatile("" : : "v"(prev) : "memory");
        if ((atomicAdd(&done[tile], 1u) & 3u) == 3u) {
            const uint32_t m = atomicExch(&used[tile], 0u);
            if (m) atomicAdd(a.counters + 1, m);
        }
    }
}

// One (tile, strip) item of the batched render: slot `slot` of the work order.
template <int K>
__device__ __forceinline__ void render_batch_item(const BatchArgs& b, uint32_t slot, uint32_t strip, WaveQueues& q,
                                                  float* pay) {
    const uint32_t gt = b.order ? b.order[slot] : slot;
    // view of global tile gt: the last view whose first tile is <= gt
    int lo = 0, hi = b.n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (b.views[mid].tile_base <= gt)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int v = __builtin_amdgcn_readfirstlane(lo);
    const ViewDev& vd = b.views[v];
    RenderArgs a;
    a.cam = vd.cam;
    a.n = b.n_records;
    a.col = b.col;
    a.pk = b.pk;
    a.zd = b.zd;
    a.vals = b.vals;
    a.ranges = b.ranges;
    a.counters = nullptr;
    a.rgb = vd.rgb;
    a.depth = vd.depth;
    a.count = vd.count;
    a.T = vd.T;
    a.blend_ids = nullptr;
    a.max_k = 0;
    a.delta = nullptr;
    a.bg0 = b.bg0;
    a.bg1 = b.bg1;
    a.bg2 = b.bg2;
    a.dL = nullptr;
    a.rgb_in = nullptr;
    a.T_in = nullptr;
    a.grad2d = nullptr;
    a.list_mode = b.list_mode;
    a.pre_vals = b.pre_vals;
    a.pre_len = b.pre_len;
    a.tile_flag = b.tile_flag;
    a.flags = b.flags;
    a.work = nullptr;
    a.fp = nullptr;
    a.status = nullptr;
    render_strip<K, kFwdPlain>(a, (int)(gt - vd.tile_base), (int)gt, (int)strip, q, nullptr, pay);
}

// Persistent form over many views: wavefronts pull (tile, strip) work items
// from atomic queues until every queue is empty; tiles are taken in the order
// given by `order` (largest lists first when cost-ordered), so views of very
// different sizes share the machine.  Slot s of that order belongs to queue s
// % 8, which the workgroups of one XCD (blockIdx.x % 8, as workgroups are
// dealt to the 8 XCDs in turn) drain first: the four strips of a tile then
// meet in one L2.  A wavefront whose queue is empty moves on to the next
// queues in turn, and leaves once it has found all of them empty.
template <int K>
__global__ __launch_bounds__(256) void k_render_hier_batch(BatchArgs b) {
    __shared__ WaveQueues s_q[4];
    __shared__ float s_pay[head_alpha_in_lds(K, kFwdPlain) ? 4 * 64 * K : 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t n_slots = b.n_tiles_dev ? *b.n_tiles_dev : b.n_tiles;
    const uint32_t home = blockIdx.x % (uint32_t)kBatchQueues;
    for (uint32_t qi = 0; qi < (uint32_t)kBatchQueues; ++qi) {
        const uint32_t x = (home + qi) % (uint32_t)kBatchQueues;
        const uint32_t n_x = n_slots > x ? (n_slots - x + kBatchQueues - 1u) / (uint32_t)kBatchQueues : 0u;
        for (;;) {
            uint32_t item = 0;
            if (lane == 0) item = atomicAdd(b.queue + x, 1u);
            item = (uint32_t)__shfl((int)item, 0);
            item = __builtin_amdgcn_readfirstlane(item);
            if (item >= 4u * n_x) break;
            const uint32_t slot = (item >> 2) * (uint32_t)kBatchQueues + x;
            render_batch_item<K>(b, slot, item & 3u, s_q[wave], s_pay + wave * 64 * K);
        }
    }
}

template <bool DEBUG>
__global__ __launch_bounds__(256) void k_render_global(RenderArgs a) {
    __shared__ float4 s_xc[256];  // x, y, conic a, b
    __shared__ float2 s_co[256];  // conic c, opacity
    __shared__ float4 s_cd[256];  // colour, |mu - o|
    __shared__ uint32_t s_id[256];
    const DevCam& cam = a.cam;
    const int tile = blockIdx.x;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int px = tx * 16 + (threadIdx.x & 15), py = ty * 16 + (threadIdx.x >> 4);
    const bool inside = px < cam.W && py < cam.H;
    const int pix = py * cam.W + px;
    const TileList tl = tile_list(a, tile);
    if (tl.skip) return;
    const uint32_t begin = 0, end = tl.len;
    float T = 1.0f, C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, D = 0.0f;
    int n = 0;
    bool done = !inside;
    uint32_t consumed = 0;
    // debug: sort error along the pixel ray (the blend order is the list's)
    float se_sum = 0.0f, se_last = 0.0f;
    const float3 dP = DEBUG ? cam_ray(cam, (float)px, (float)py) : make_float3(0.0f, 0.0f, 0.0f);
    for (uint32_t start = begin; start < end; start += 256) {
        if (__syncthreads_count(done ? 1 : 0) == 256) break;
        const uint32_t idx = start + threadIdx.x;
        if (idx < end) {
            uint32_t id = tl.ids[idx];
            id = id < a.n ? id : 0u;
            s_id[threadIdx.x] = id;
            const float4 p0 = a.pk[4 * (size_t)id], p1 = a.pk[4 * (size_t)id + 1];
            s_xc[threadIdx.x] = p0;
            s_co[threadIdx.x] = make_float2(p1.x, p1.y);
            s_cd[threadIdx.x] = a.col[id];
        }
        __syncthreads();
        const uint32_t cnt = (end - start) < 256u ? (end - start) : 256u;
        consumed += cnt;
        for (uint32_t k = 0; k < cnt && !done; ++k) {
            Splat g;
            const float4 xc = s_xc[k];
            const float2 c = s_co[k];
            g.x = xc.x;
            g.y = xc.y;
            g.ca = xc.z;
            g.cb = xc.w;
            g.cc = c.x;
            g.op = c.y;
            g.lt = __int_as_float(0x7fc00000);
            float alpha;
            if (!pixel_alpha(g, (float)px, (float)py, alpha)) continue;
            const float Tn = T * (1.0f - alpha);
            if (Tn < kTMin) {
                done = true;
                break;
            }
            const float4 cd = s_cd[k];
            C0 = fmaf(cd.x * alpha, T, C0);
            C1 = fmaf(cd.y * alpha, T, C1);
            C2 = fmaf(cd.z * alpha, T, C2);
            D = fmaf(cd.w * alpha, T, D);
            if (DEBUG && n < a.max_k) a.blend_ids[(size_t)pix * a.max_k + n] = (int32_t)s_id[k];
            if (DEBUG && a.delta) {
                const float t = t_opt(load_packed(a.pk, s_id[k]), dP);
                if (n > 0 && se_last > t) se_sum = se_sum + (se_last - t);
                se_last = t;
            }
            n += 1;
            T = Tn;
        }
        __syncthreads();
    }
    // A prefix that ran out while pixels are still live cannot decide the
    // tile: flag it for its whole sorted list.
    if (tl.truncated && __syncthreads_or(done ? 0 : 1) && threadIdx.x == 0) a.tile_flag[tile] = tl.n_all;
    if (inside) {
        const size_t P = (size_t)cam.W * cam.H;
        a.rgb[pix] = C0 + T * a.bg0;
        a.rgb[P + pix] = C1 + T * a.bg1;
        a.rgb[2 * P + pix] = C2 + T * a.bg2;
        a.depth[pix] = D;
        a.count[pix] = n;
        a.T[pix] = T;
        if (DEBUG) {
            for (int k = n; k < a.max_k; ++k) a.blend_ids[(size_t)pix * a.max_k + k] = -1;
            if (a.delta) a.delta[pix] = se_sum;
        }
    }
    if (threadIdx.x == 0 && consumed) atomicAdd(a.counters + 1, consumed);
}

// One workgroup per tile; list entries staged through LDS 256 at a time; one
// lane per pixel with its window in registers (the head machinery of the
// hierarchical renderer).
template <int K, int MODE>
__global__ __launch_bounds__(256) void k_render_window(RenderArgs a) {
    __shared__ Splat s_g[256];
    __shared__ uint32_t s_id[256];
    __shared__ float s_pay[head_alpha_in_lds(K, MODE) ? 4 * 64 * K : 1];
    const DevCam& cam = a.cam;
    const int tile = blockIdx.x;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int px = tx * 16 + (threadIdx.x & 15), py = ty * 16 + (threadIdx.x >> 4);
    const bool inside = px < cam.W && py < cam.H;
    const int pix = py * cam.W + px;
    const TileList tl = tile_list(a, tile);
    if (tl.skip) return;
    const uint32_t begin = 0;
    // list ranks are keyed; a large window keeps them below kMaxPayloadRank
    const uint32_t end = head_alpha_in_lds(K, MODE) && tl.len > kMaxPayloadRank ? kMaxPayloadRank : tl.len;
    const float3 d = cam_ray(cam, (float)px, (float)py);
    PixelState<K, MODE> st;
    st.T = 1.0f;
    init_colour(st);
    st.D = 0.0f;
    st.dl = st.tl = 0.0f;
    st.n = 0;
    st.done = !inside;
    st.hn = 0;
    st.ids = tl.ids;
    st.n_ids = a.n;
    st.pay = s_pay + (threadIdx.x >> 6) * 64 * K + (threadIdx.x & 63);
#pragma unroll
    for (int i = 0; i < K; ++i) {
        st.hk[i] = kInvalidKey;
        if (!head_alpha_in_lds(K, MODE)) st.ha[i] = 0.0f;
        if (head_keeps_ids(K, MODE)) st.hid[i] = 0u;
    }
    uint32_t consumed = 0;
    for (uint32_t start = begin; start < end; start += 256) {
        if (__syncthreads_count(st.done ? 1 : 0) == 256) break;
        const uint32_t idx = start + threadIdx.x;
        if (idx < end) {
            uint32_t id = tl.ids[idx];
            id = id < a.n ? id : 0u;
            s_id[threadIdx.x] = id;
            s_g[threadIdx.x] = load_packed(a.pk, id);
        }
        __syncthreads();
        const uint32_t cnt = (end - start) < 256u ? (end - start) : 256u;
        consumed += cnt;
        for (uint32_t k = 0; k < cnt && !st.done; ++k) {
            const Splat& g = s_g[k];
            float alpha;
            if (!pixel_alpha(g, (float)px, (float)py, alpha)) continue;
            const uint64_t key = ((uint64_t)depth_bits(t_opt(g, d)) << 32) | (uint64_t)(start - begin + k);
            head_push<K, MODE>(a, st, pix, key, s_id[k], alpha, nullptr);
        }
        __syncthreads();
    }
    // A prefix that ran out while pixels are still live cannot decide the
    // tile: flag it for its whole sorted list (this pass's image is redone).
    if (tl.truncated && __syncthreads_or(st.done ? 0 : 1) && threadIdx.x == 0) a.tile_flag[tile] = tl.n_all;
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (st.hn > 0) head_pop_blend<K, MODE>(a, st, pix, nullptr);
    flush_colour(st);
    if (inside) {
        const size_t P = (size_t)cam.W * cam.H;
        a.rgb[pix] = st.C0 + st.T * a.bg0;
        a.rgb[P + pix] = st.C1 + st.T * a.bg1;
        a.rgb[2 * P + pix] = st.C2 + st.T * a.bg2;
        a.depth[pix] = st.D;
        a.count[pix] = st.n;
        a.T[pix] = st.T;
        if (MODE == kFwdDebug) {
            for (int k = st.n; k < a.max_k; ++k) a.blend_ids[(size_t)pix * a.max_k + k] = -1;
            if (a.delta) a.delta[pix] = st.dl;
        }
    }
    if (threadIdx.x == 0 && consumed) atomicAdd(a.counters + 1, consumed);
}

// Full per-pixel order without per-pixel storage: in rounds, every pixel
// scans its tile's list (exactly culled, so it holds every contributor) and
// keeps in registers the kFullSel smallest keys (t_opt bits << 32 | id) above
// the last key it blended, then blends them in order.  A round that finds
// fewer than kFullSel keys ends the pixel's list; a terminated pixel stops.
constexpr int kFullSel = 16;

template <int MODE>
__global__ __launch_bounds__(256) void k_render_full(RenderArgs a) {
    constexpr int K = kFullSel;
    __shared__ Splat s_g[256];
    __shared__ uint32_t s_id[256];
    const DevCam& cam = a.cam;
    const int tile = blockIdx.x;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int px = tx * 16 + (threadIdx.x & 15), py = ty * 16 + (threadIdx.x >> 4);
    const bool inside = px < cam.W && py < cam.H;
    const int pix = py * cam.W + px;
    const TileList tl = tile_list(a, tile);
    if (tl.skip) return;
    const uint32_t begin = 0, end = tl.len;
    const float3 d = cam_ray(cam, (float)px, (float)py);
    PixelState<K, MODE> st;
    st.T = 1.0f;
    init_colour(st);
    st.D = 0.0f;
    st.dl = st.tl = 0.0f;
    st.n = 0;
    st.done = !inside;
    st.hn = 0;
    st.ids = nullptr;
    st.n_ids = a.n;
    // the kFullSel smallest keys of a round: t_opt bits << 32 | Gaussian id
    uint64_t fk[K];
    float fa[K];
    bool more = true;
    uint64_t floor_key = 0;  // keys below this were blended in earlier rounds
    while (__syncthreads_or(!st.done && more)) {
        const bool active = !st.done && more;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            fk[i] = kInvalidKey;
            fa[i] = 0.0f;
        }
        int found = 0;
        for (uint32_t start = begin; start < end; start += 256) {
            const uint32_t idx = start + threadIdx.x;
            __syncthreads();
            if (idx < end) {
                uint32_t id = tl.ids[idx];
                id = id < a.n ? id : 0u;
                s_id[threadIdx.x] = id;
                s_g[threadIdx.x] = load_packed(a.pk, id);
            }
            __syncthreads();
            const uint32_t cnt = (end - start) < 256u ? (end - start) : 256u;
            if (!active) continue;
            for (uint32_t k = 0; k < cnt; ++k) {
                const Splat& g = s_g[k];
                float alpha;
                if (!pixel_alpha(g, (float)px, (float)py, alpha)) continue;
                const uint64_t key = ((uint64_t)depth_bits(t_opt(g, d)) << 32) | (uint64_t)s_id[k];
                if (key < floor_key || key >= fk[K - 1]) continue;
                // insertion into the sorted K smallest; the largest drops out
#pragma unroll
                for (int i = K - 1; i >= 1; --i) {
                    if (fk[i - 1] > key) {
                        fk[i] = fk[i - 1];
                        fa[i] = fa[i - 1];
                    } else if (fk[i] > key) {
                        fk[i] = key;
                        fa[i] = alpha;
                    }
                }
                if (fk[0] > key) {
                    fk[0] = key;
                    fa[0] = alpha;
                }
                found = found < K ? found + 1 : K;
            }
        }
        if (active) {
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < found) {
                    const uint32_t id = (uint32_t)fk[i];
                    blend_one<K, MODE>(a, st, pix, id < a.n ? id : 0u, fa[i], depth_from_bits((uint32_t)(fk[i] >> 32)),
                                       0u, nullptr);
                }
            more = found == K;
            floor_key = fk[K - 1] + 1ull;
        }
    }
    flush_colour(st);
    if (inside) {
        const size_t P = (size_t)cam.W * cam.H;
        a.rgb[pix] = st.C0 + st.T * a.bg0;
        a.rgb[P + pix] = st.C1 + st.T * a.bg1;
        a.rgb[2 * P + pix] = st.C2 + st.T * a.bg2;
        a.depth[pix] = st.D;
        a.count[pix] = st.n;
        a.T[pix] = st.T;
        if (MODE == kFwdDebug) {
            for (int k = st.n; k < a.max_k; ++k) a.blend_ids[(size_t)pix * a.max_k + k] = -1;
            if (a.delta) a.delta[pix] = st.dl;
        }
    }
}

template <int K>
hipError_t launch_window_k(const RenderArgs& a, hipStream_t s) {
    const unsigned tiles = (unsigned)(a.cam.tiles_x * a.cam.tiles_y);
    if (a.blend_ids || a.delta)
        hipLaunchKernelGGL((k_render_window<K, kFwdDebug>), dim3(tiles), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((k_render_window<K, kFwd>), dim3(tiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int K>
hipError_t launch_hier_k(const RenderArgs& a, hipStream_t s) {
    // the loads-ahead variant fits the registers (256 per lane, no spill) for heads up to 8
    constexpr bool kDeepBuilt = K <= 8;
    const unsigned tiles = (unsigned)(a.cam.tiles_x * a.cam.tiles_y);
    if (a.work) {
        if (K != 4) return hipErrorInvalidValue;  // the counting kernel is built for the default head
        hipLaunchKernelGGL((k_render_hier<4, kFwdCount>), dim3(tiles), dim3(256), 0, s, a);
    } else if (a.grad2d)
        hipLaunchKernelGGL((k_render_hier<K, kBwd>), dim3(tiles), dim3(256), 0, s, a);
    else if ((a.blend_ids || a.delta) && a.deep)
        hipLaunchKernelGGL((k_render_hier1<K, kFwdDebug, kDeepBuilt>), dim3((tiles + 7u) / 8u * 32u), dim3(64), 0, s,
                           a);
    else if (a.blend_ids || a.delta)
        hipLaunchKernelGGL((k_render_hier1<K, kFwdDebug, false>), dim3((tiles + 7u) / 8u * 32u), dim3(64), 0, s, a);
    else if (a.deep)
        hipLaunchKernelGGL((k_render_hier1<K, kFwd, kDeepBuilt>), dim3((tiles + 7u) / 8u * 32u), dim3(64), 0, s, a);
    else
        hipLaunchKernelGGL((k_render_hier1<K, kFwd, false>), dim3((tiles + 7u) / 8u * 32u), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace

bool hier_head_supported(int head) {
    switch (head) {
        case 1: case 2: case 3: case 4: case 6: case 8: case 12: case 16: case 20: case 24:
            return true;
        default:
            return false;
    }
}

hipError_t launch_render_hier(const RenderArgs& a, int head, hipStream_t s) {
    switch (head) {
        case 1: return launch_hier_k<1>(a, s);
        case 2: return launch_hier_k<2>(a, s);
        case 3: return launch_hier_k<3>(a, s);
        case 4: return launch_hier_k<4>(a, s);
        case 6: return launch_hier_k<6>(a, s);
        case 8: return launch_hier_k<8>(a, s);
        case 12: return launch_hier_k<12>(a, s);
        case 16: return launch_hier_k<16>(a, s);
        case 20: return launch_hier_k<20>(a, s);
        case 24: return launch_hier_k<24>(a, s);
        default: return hipErrorInvalidValue;
    }
}

template <int K>
hipError_t launch_hier_batch_k(const BatchArgs& b, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL(k_render_hier_batch<K>, dim3(grid), dim3(256), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_render_hier_batch(const BatchArgs& b, int head, unsigned grid, hipStream_t s) {
    switch (head) {
        case 1: return launch_hier_batch_k<1>(b, grid, s);
        case 2: return launch_hier_batch_k<2>(b, grid, s);
        case 3: return launch_hier_batch_k<3>(b, grid, s);
        case 4: return launch_hier_batch_k<4>(b, grid, s);
        case 6: return launch_hier_batch_k<6>(b, grid, s);
        case 8: return launch_hier_batch_k<8>(b, grid, s);
        case 12: return launch_hier_batch_k<12>(b, grid, s);
        case 16: return launch_hier_batch_k<16>(b, grid, s);
        case 20: return launch_hier_batch_k<20>(b, grid, s);
        case 24: return launch_hier_batch_k<24>(b, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_render_window(const RenderArgs& a, int head, hipStream_t s) {
    switch (head) {
        case 1: return launch_window_k<1>(a, s);
        case 2: return launch_window_k<2>(a, s);
        case 3: return launch_window_k<3>(a, s);
        case 4: return launch_window_k<4>(a, s);
        case 6: return launch_window_k<6>(a, s);
        case 8: return launch_window_k<8>(a, s);
        case 12: return launch_window_k<12>(a, s);
        case 16: return launch_window_k<16>(a, s);
        case 20: return launch_window_k<20>(a, s);
        case 24: return launch_window_k<24>(a, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_render_full(const RenderArgs& a, hipStream_t s) {
    const unsigned tiles = (unsigned)(a.cam.tiles_x * a.cam.tiles_y);
    if (a.blend_ids || a.delta)
        hipLaunchKernelGGL(k_render_full<kFwdDebug>, dim3(tiles), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_render_full<kFwd>, dim3(tiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_render_global(const RenderArgs& a, hipStream_t s) {
    const unsigned tiles = (unsigned)(a.cam.tiles_x * a.cam.tiles_y);
    if (a.blend_ids || a.delta)
        hipLaunchKernelGGL(k_render_global<true>, dim3(tiles), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(k_render_global<false>, dim3(tiles), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace gsr
