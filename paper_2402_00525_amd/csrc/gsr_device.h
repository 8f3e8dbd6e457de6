// Device arithmetic of the gfx950 rasterizer: exp/ln, ordered depth keys,
// camera rays, t_opt, the 2D Gaussian exponent, Algorithm 1 and the culling
// test.  Every floating-point expression is written in a fixed evaluation
// order and the library is built with -ffp-contract=off, so results are plain
// IEEE binary32 operations (division and square root correctly rounded).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gsr {

constexpr float kEpsO = 1.0f / 255.0f;   // opacity threshold eps_O (Sec. 3.4)
constexpr float kTMin = 0.0001f;         // transmittance stop
constexpr float kAlphaMax = 0.99f;       // alpha clamp
constexpr uint64_t kInvalidKey = ~0ull;

// Camera as handed to kernels.
struct DevCam {
    float R[9];
    float t[3];
    float o[3];
    float fx, fy, cx, cy, znear, limx, limy;
    float rfx, rfy;  // 1 / fx, 1 / fy, each rounded once
    int W, H, tiles_x, tiles_y;
};

__device__ __forceinline__ float sel_min(float a, float b) { return a < b ? a : b; }
__device__ __forceinline__ float sel_max(float a, float b) { return a > b ? a : b; }
__device__ __forceinline__ float sel_clamp(float v, float lo, float hi) { return v < lo ? lo : (v > hi ? hi : v); }

// e^x: x = k ln2 + r with k = rint(x log2 e) (Cody & Waite reduction, ln 2 in
// a 16-bit head and a tail), e^r by its Taylor series to degree 7 in Horner
// form with fused multiply-adds, result scaled by 2^k.  Below -80 (or NaN): 0.
__device__ __forceinline__ float exp_cw(float x) {
    if (!(x >= -80.0f)) return 0.0f;
    const float k = rintf(x * 1.44269504088896341f);
    float r = fmaf(-k, 0.693145751953125f, x);
    r = fmaf(-k, 1.42860676533018e-06f, r);
    float p = 1.0f / 5040.0f;
    p = fmaf(p, r, 1.0f / 720.0f);
    p = fmaf(p, r, 1.0f / 120.0f);
    p = fmaf(p, r, 1.0f / 24.0f);
    p = fmaf(p, r, 1.0f / 6.0f);
    p = fmaf(p, r, 0.5f);
    p = fmaf(p, r, 1.0f);
    p = fmaf(p, r, 1.0f);
    return ldexpf(p, (int)k);
}

// ln x for x >= 1: x = m 2^e, m in [1/sqrt 2, sqrt 2), ln m = 2 atanh((m-1)/(m+1))
// by its odd series through the 11th power.
__device__ __forceinline__ float ln_atanh(float x) {
    int e;
    float m = frexpf(x, &e);
    if (m < 0.70710678f) {
        m = m * 2.0f;
        e = e - 1;
    }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    float p = 1.0f / 11.0f;
    p = fmaf(p, z, 1.0f / 9.0f);
    p = fmaf(p, z, 1.0f / 7.0f);
    p = fmaf(p, z, 1.0f / 5.0f);
    p = fmaf(p, z, 1.0f / 3.0f);
    p = fmaf(p, z, 1.0f);
    const float lnm = (2.0f * s) * p;
    return fmaf((float)e, 0.693147180559945309f, lnm);
}

// Unsigned image of a float that orders like the float ('-0' before '+0').
__device__ __forceinline__ uint32_t depth_bits(float t) {
    const uint32_t u = __float_as_uint(t);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float depth_from_bits(uint32_t b) {
    return __uint_as_float((b & 0x80000000u) ? (b & 0x7fffffffu) : ~b);
}

// Unit world-space direction of the ray through image point (u, v): the
// camera-frame direction ((u - cx) rfx, (v - cy) rfy, 1) with rfx = 1 / fx,
// rfy = 1 / fy, rotated to the world by fused multiply-adds and scaled by the
// one reciprocal of its norm.
__device__ __forceinline__ float3 cam_ray(const DevCam& c, float u, float v) {
    const float a = (u - c.cx) * c.rfx;
    const float b = (v - c.cy) * c.rfy;
    const float w0 = fmaf(c.R[3], b, fmaf(c.R[0], a, c.R[6]));
    const float w1 = fmaf(c.R[4], b, fmaf(c.R[1], a, c.R[7]));
    const float w2 = fmaf(c.R[5], b, fmaf(c.R[2], a, c.R[8]));
    const float len = sqrtf(fmaf(w2, w2, fmaf(w1, w1, w0 * w0)));
    const float inv = 1.0f / len;
    return make_float3(w0 * inv, w1 * inv, w2 * inv);
}

// The per-Gaussian data the render levels use: 2D mean, conic, opacity,
// Sigma^-1 (6 unique entries), w = Sigma^-1 (mu - o), and lt = ln(eps_O /
// opacity) (NaN when not at hand), which lets culling skip exp (clears_eps).
struct Splat {
    float x, y, ca, cb, cc, op;
    float s00, s01, s02, s11, s12, s22, w0, w1, w2;
    float lt;
};

__device__ __forceinline__ Splat load_splat(const float2* __restrict__ xy, const float4* __restrict__ co,
                                            const float4* __restrict__ sw, uint32_t id) {
    Splat g;
    const float2 m = xy[id];
    const float4 c = co[id];
    const float4 a = sw[3 * id];
    const float4 b = sw[3 * id + 1];
    const float4 e = sw[3 * id + 2];
    g.x = m.x; g.y = m.y;
    g.ca = c.x; g.cb = c.y; g.cc = c.z; g.op = c.w;
    g.s00 = a.x; g.s01 = a.y; g.s02 = a.z; g.s11 = a.w;
    g.s12 = b.x; g.s22 = b.y; g.w0 = b.z; g.w1 = b.w;
    g.w2 = e.x;
    g.lt = __int_as_float(0x7fc00000);
    return g;
}

// The same splat from its packed 64-byte record (one cache line):
// (x, y, a, b), (c, opacity, s00, s01), (s02, s11, s12, s22), (w0, w1, w2, lt).
__device__ __forceinline__ Splat load_packed(const float4* __restrict__ pk, uint32_t id) {
    const float4 p0 = pk[4 * (size_t)id], p1 = pk[4 * (size_t)id + 1];
    const float4 p2 = pk[4 * (size_t)id + 2], p3 = pk[4 * (size_t)id + 3];
    Splat g;
    g.x = p0.x; g.y = p0.y; g.ca = p0.z; g.cb = p0.w;
    g.cc = p1.x; g.op = p1.y; g.s00 = p1.z; g.s01 = p1.w;
    g.s02 = p2.x; g.s11 = p2.y; g.s12 = p2.z; g.s22 = p2.w;
    g.w0 = p3.x; g.w1 = p3.y; g.w2 = p3.z;
    g.lt = p3.w;
    return g;
}

// Depth of maximum contribution along unit direction d (Eq. dopt):
// d^T Sigma^-1 (mu - o) / d^T Sigma^-1 d, each dot product one product and
// fused multiply-adds in index order; a NaN quotient reads as +inf.
__device__ __forceinline__ float t_opt(const Splat& g, float3 d) {
    const float sd0 = fmaf(g.s02, d.z, fmaf(g.s01, d.y, g.s00 * d.x));
    const float sd1 = fmaf(g.s12, d.z, fmaf(g.s11, d.y, g.s01 * d.x));
    const float sd2 = fmaf(g.s22, d.z, fmaf(g.s12, d.y, g.s02 * d.x));
    const float num = fmaf(d.z, g.w2, fmaf(d.y, g.w1, d.x * g.w0));
    const float den = fmaf(d.z, sd2, fmaf(d.y, sd1, d.x * sd0));
    const float t = num / den;
    return (t != t) ? __int_as_float(0x7f800000) : t;
}

// Exponent of G_2 at offset d = mu_2 - p: -1/2 (a dx^2 + c dy^2) - b dx dy,
// as -1/2 q - b dx dy with q = fma(c dy, dy, (a dx) dx), fused.
__device__ __forceinline__ float power_at_offset(float ca, float cb, float cc, float dx, float dy) {
    const float q = fmaf(cc * dy, dy, (ca * dx) * dx);
    return fmaf(-0.5f, q, -((cb * dx) * dy));
}
__device__ __forceinline__ float splat_power(const Splat& g, float px, float py) {
    return power_at_offset(g.ca, g.cb, g.cc, g.x - px, g.y - py);
}

// Algorithm 1 (App. B.1): the point of box [x0,x1] x [y0,y1] where the 2D
// Gaussian is largest, found on the two edges at the corner nearest the mean.
// FAST: the two edge parameters use a reciprocal instead of a correctly
// rounded division (for decisions that tolerate it, see block_clears).
template <bool FAST = false>
__device__ __forceinline__ float2 box_max_point(const Splat& g, float x0, float x1, float y0, float y1) {
    const float mx = g.x, my = g.y;
    const bool in_x = (x0 <= mx && mx <= x1);
    const bool in_y = (y0 <= my && my <= y1);
    if (in_x && in_y) return make_float2(mx, my);
    const float px = (mx < x0) ? x0 : ((mx > x1) ? x1 : ((mx - x0 <= x1 - mx) ? x0 : x1));
    const float py = (my < y0) ? y0 : ((my > y1) ? y1 : ((my - y0 <= y1 - my) ? y0 : y1));
    const float lx = ((px == x0) ? x1 : x0) - px;
    const float ly = ((py == y0) ? y1 : y0) - py;
    const float dx = mx - px, dy = my - py;
    float tx = 0.0f, ty = 0.0f;
    if (FAST) {
        if (!in_x && ly != 0.0f) ty = sel_clamp(__fdividef(fmaf(g.cb, dx, g.cc * dy), g.cc * ly), 0.0f, 1.0f);
        if (!in_y && lx != 0.0f) tx = sel_clamp(__fdividef(fmaf(g.ca, dx, g.cb * dy), g.ca * lx), 0.0f, 1.0f);
    } else {
        if (!in_x && ly != 0.0f) ty = sel_clamp(fmaf(g.cb, dx, g.cc * dy) / (g.cc * ly), 0.0f, 1.0f);
        if (!in_y && lx != 0.0f) tx = sel_clamp(fmaf(g.ca, dx, g.cb * dy) / (g.ca * lx), 0.0f, 1.0f);
    }
    return make_float2(fmaf(tx, lx, px), fmaf(ty, ly, py));
}

// opacity * exp(p) >= eps_O, decided as that comparison.  When the exponent
// is more than kCullMargin away from lt = ln(eps_O / opacity) the answer is
// settled without exp: exp, the logarithm and the products are accurate to
// about 1e-6, far inside the margin, so the result is the exact comparison's.
constexpr float kCullMargin = 1e-3f;

__device__ __forceinline__ bool clears_eps(const Splat& g, float p) {
    if (!(p <= 0.0f)) return false;
    if (p < g.lt - kCullMargin) return false;
    if (p > g.lt + kCullMargin) return true;
    return g.op * exp_cw(p) >= kEpsO;
}

// Exact culling: keep iff the maximum over the block clears eps_O; xh = the
// block's maximum point x^.
__device__ __forceinline__ bool keeps_block(const Splat& g, float x0, float x1, float y0, float y1, float2& xh) {
    xh = box_max_point(g, x0, x1, y0, y1);
    return clears_eps(g, splat_power(g, xh.x, xh.y));
}

// The same decision without x^.  The maximum point is first found with
// reciprocals; that moves the exponent by about 1e-5 (the 0.3 px^2 dilation
// bounds the conic), so an exponent more than kFastMargin from lt = ln(eps_O /
// opacity), and clearly below 0, settles the test; anything else is decided
// by keeps_block.
constexpr float kFastMargin = 2e-3f;

__device__ __forceinline__ bool block_clears(const Splat& g, float x0, float x1, float y0, float y1) {
    const float2 xa = box_max_point<true>(g, x0, x1, y0, y1);
    const float pa = splat_power(g, xa.x, xa.y);
    if (pa < g.lt - kFastMargin) return false;
    if (pa > g.lt + kFastMargin && pa < -kFastMargin) return true;
    float2 xh;
    return keeps_block(g, x0, x1, y0, y1, xh);
}

// alpha at a pixel centre; false when the Gaussian is skipped there (alpha is
// then not set).
__device__ __forceinline__ bool pixel_alpha(const Splat& g, float px, float py, float& alpha) {
    const float p = splat_power(g, px, py);
    if (p > 0.0f) return false;
    if (p < g.lt - kCullMargin) return false;
    const float a = g.op * exp_cw(p);
    alpha = a < kAlphaMax ? a : kAlphaMax;
    return !(alpha < kEpsO);
}

// ----- wavefront helpers (wave64) -----
__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Value of lane `src` (the same for every lane of the wavefront) in every
// lane, read into a scalar register.
__device__ __forceinline__ int lane_bcast(int v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ __forceinline__ uint32_t lane_bcast(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}
__device__ __forceinline__ float lane_bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// Orders this lane's LDS accesses against those of the other lanes of the
// same wavefront (compiler barrier plus wait for outstanding LDS operations).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this wave's LDS traffic has landed
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace gsr
