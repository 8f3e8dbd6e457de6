// Oracle for the sorted Gaussian-splatting frame -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, single-file CPU statement of what the frame pipeline of
// "StopThePop: Sorted Gaussian Splatting for View-Consistent Real-time
// Rendering" computes.  Only the test-suite, the smoke check and the CPU
// baseline of the benchmark load it; the product library never calls it, and
// the two share no code.
//
// The arithmetic is written as templates over the real type F:
//   * F = float  is the parity instantiation.  Every floating-point operation
//     is an IEEE-754 binary32 operation in the order written here (the file is
//     compiled with -ffp-contract=off and without fast math), so integer
//     decisions taken from floats (culling, sort keys, queue order, early
//     termination) are reproducible bit for bit.
//   * F = double is the reference instantiation used to pin the float one and
//     to check gradients against finite differences.
//
// Readings of points the paper leaves open are listed beside the code that
// takes them.  Parity status: every function here is pinned by the CPU tests
// (closed forms, brute force, invariants) except the exact interleaving of
// tail and mid pops at the default queue sizes, which is pinned only through
// the special cases described in hier_subtile().

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

typedef uint32_t u32;
typedef uint64_t u64;

// ---------------------------------------------------------------------------
// Scalar helpers.  Minimum, maximum and clamp are written as selections so
// that the chosen operand (including the sign of zero) is fixed.
// ---------------------------------------------------------------------------
template <class F> inline F smin(F a, F b) { return a < b ? a : b; }
template <class F> inline F smax(F a, F b) { return a > b ? a : b; }
template <class F> inline F sclamp(F v, F lo, F hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Order-preserving integer image of a float: u -> (u >= 2^31) ? ~u : u | 2^31.
// Unsigned comparison of the images equals '<' on the floats, with -0 < +0.
inline u64 ord_key(float t) {
    u32 u;
    std::memcpy(&u, &t, 4);
    return (u & 0x80000000u) ? (u64)(~u) : (u64)(u | 0x80000000u);
}
inline u64 ord_key(double t) {
    u64 u;
    std::memcpy(&u, &t, 8);
    return (u & 0x8000000000000000ull) ? ~u : (u | 0x8000000000000000ull);
}

// ---------------------------------------------------------------------------
// exp used for every opacity decision: Cody-Waite argument reduction
// x = k ln2 + r, |r| <= ln2/2, then the degree-7 Taylor polynomial of e^r in
// Horner form with fused multiply-adds, then scaling by 2^k.  ln2 is split as
// LN2_HI (the leading 16 bits of ln 2) + LN2_LO.  Arguments below -80 (and
// NaN) give 0.  The double instantiation uses the C library.
// ---------------------------------------------------------------------------
inline float expE(float x) {
    if (!(x >= -80.0f)) return 0.0f;
    const float LOG2E = 1.44269504088896341f;
    const float LN2_HI = 0.693145751953125f;
    const float LN2_LO = 1.42860676533018e-06f;
    float k = std::rint(x * LOG2E);
    float r = std::fma(-k, LN2_HI, x);
    r = std::fma(-k, LN2_LO, r);
    float p = 1.0f / 5040.0f;
    p = std::fma(p, r, 1.0f / 720.0f);
    p = std::fma(p, r, 1.0f / 120.0f);
    p = std::fma(p, r, 1.0f / 24.0f);
    p = std::fma(p, r, 1.0f / 6.0f);
    p = std::fma(p, r, 0.5f);
    p = std::fma(p, r, 1.0f);
    p = std::fma(p, r, 1.0f);
    return std::ldexp(p, (int)k);
}
inline double expE(double x) { return std::exp(x); }

// Natural logarithm for x >= 1 used only for the opacity-aware bound t_O:
// x = m 2^e with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s) with
// s = (m-1)/(m+1), series 2s(1 + s^2/3 + s^4/5 + ... + s^10/11).
inline float lnE(float x) {
    int e;
    float m = std::frexp(x, &e);
    if (m < 0.70710678f) {
        m = m * 2.0f;
        e = e - 1;
    }
    float s = (m - 1.0f) / (m + 1.0f);
    float z = s * s;
    float p = 1.0f / 11.0f;
    p = std::fma(p, z, 1.0f / 9.0f);
    p = std::fma(p, z, 1.0f / 7.0f);
    p = std::fma(p, z, 1.0f / 5.0f);
    p = std::fma(p, z, 1.0f / 3.0f);
    p = std::fma(p, z, 1.0f);
    float lnm = (2.0f * s) * p;
    return std::fma((float)e, 0.693147180559945309f, lnm);
}
inline double lnE(double x) { return std::log(x); }

// ---------------------------------------------------------------------------
// Real spherical harmonics up to degree 3 (colour, Sec. 1 / App. B.4): the
// orthonormal real basis, with the constants written from their closed forms
// sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) and the sign convention below.
// ---------------------------------------------------------------------------
template <class F> struct SHC {
    F c0, c1, c2[5], c3[7];
    SHC() {
        const double sp = std::sqrt(M_PI);
        c0 = (F)(0.5 / sp);
        c1 = (F)(std::sqrt(3.0) / (2.0 * sp));
        c2[0] = (F)(std::sqrt(15.0) / (2.0 * sp));
        c2[1] = (F)(-std::sqrt(15.0) / (2.0 * sp));
        c2[2] = (F)(std::sqrt(5.0) / (4.0 * sp));
        c2[3] = (F)(-std::sqrt(15.0) / (2.0 * sp));
        c2[4] = (F)(std::sqrt(15.0) / (4.0 * sp));
        c3[0] = (F)(-std::sqrt(17.5) / (4.0 * sp));
        c3[1] = (F)(std::sqrt(105.0) / (2.0 * sp));
        c3[2] = (F)(-std::sqrt(10.5) / (4.0 * sp));
        c3[3] = (F)(std::sqrt(7.0) / (4.0 * sp));
        c3[4] = (F)(-std::sqrt(10.5) / (4.0 * sp));
        c3[5] = (F)(std::sqrt(105.0) / (4.0 * sp));
        c3[6] = (F)(-std::sqrt(17.5) / (4.0 * sp));
    }
};

// Basis values b[0..(d+1)^2) at unit direction (x, y, z).
template <class F> void sh_basis(int deg, F x, F y, F z, F* b) {
    static const SHC<F> C;
    b[0] = C.c0;
    if (deg < 1) return;
    b[1] = (-C.c1) * y;
    b[2] = C.c1 * z;
    b[3] = (-C.c1) * x;
    if (deg < 2) return;
    F xx = x * x, yy = y * y, zz = z * z, xy = x * y, yz = y * z, xz = x * z;
    b[4] = C.c2[0] * xy;
    b[5] = C.c2[1] * yz;
    b[6] = C.c2[2] * ((F(2) * zz - xx) - yy);
    b[7] = C.c2[3] * xz;
    b[8] = C.c2[4] * (xx - yy);
    if (deg < 3) return;
    b[9] = C.c3[0] * (y * (F(3) * xx - yy));
    b[10] = C.c3[1] * (xy * z);
    b[11] = C.c3[2] * (y * ((F(4) * zz - xx) - yy));
    b[12] = C.c3[3] * (z * ((F(2) * zz - F(3) * xx) - F(3) * yy));
    b[13] = C.c3[4] * (x * ((F(4) * zz - xx) - yy));
    b[14] = C.c3[5] * (z * (xx - yy));
    b[15] = C.c3[6] * (x * (xx - F(3) * yy));
}

// Derivative of the basis with respect to the (unnormalised) unit direction
// components: db[k][0..2].
template <class F> void sh_basis_grad(int deg, F x, F y, F z, F db[16][3]) {
    static const SHC<F> C;
    for (int k = 0; k < 16; ++k) db[k][0] = db[k][1] = db[k][2] = F(0);
    if (deg < 1) return;
    db[1][1] = -C.c1;
    db[2][2] = C.c1;
    db[3][0] = -C.c1;
    if (deg < 2) return;
    db[4][0] = C.c2[0] * y; db[4][1] = C.c2[0] * x;
    db[5][1] = C.c2[1] * z; db[5][2] = C.c2[1] * y;
    db[6][0] = C.c2[2] * (-2 * x); db[6][1] = C.c2[2] * (-2 * y); db[6][2] = C.c2[2] * (4 * z);
    db[7][0] = C.c2[3] * z; db[7][2] = C.c2[3] * x;
    db[8][0] = C.c2[4] * (2 * x); db[8][1] = C.c2[4] * (-2 * y);
    if (deg < 3) return;
    F xx = x * x, yy = y * y, zz = z * z;
    db[9][0] = C.c3[0] * (6 * x * y); db[9][1] = C.c3[0] * (3 * xx - 3 * yy);
    db[10][0] = C.c3[1] * (y * z); db[10][1] = C.c3[1] * (x * z); db[10][2] = C.c3[1] * (x * y);
    db[11][0] = C.c3[2] * (-2 * x * y); db[11][1] = C.c3[2] * (4 * zz - xx - 3 * yy); db[11][2] = C.c3[2] * (8 * y * z);
    db[12][0] = C.c3[3] * (-6 * x * z); db[12][1] = C.c3[3] * (-6 * y * z); db[12][2] = C.c3[3] * (6 * zz - 3 * xx - 3 * yy);
    db[13][0] = C.c3[4] * (4 * zz - 3 * xx - yy); db[13][1] = C.c3[4] * (-2 * x * y); db[13][2] = C.c3[4] * (8 * x * z);
    db[14][0] = C.c3[5] * (2 * x * z); db[14][1] = C.c3[5] * (-2 * y * z); db[14][2] = C.c3[5] * (xx - yy);
    db[15][0] = C.c3[6] * (3 * xx - 3 * yy); db[15][1] = C.c3[6] * (-6 * x * y);
}

// ---------------------------------------------------------------------------
// Inputs.
// ---------------------------------------------------------------------------
struct OCam {  // mirrors the C struct handed in from Python (all float32)
    float R[9];       // world->camera rotation, row-major
    float t[3];       // translation: p_cam = R p + t
    float center[3];  // camera centre o in world space
    float fx, fy, cx, cy, znear;
    int32_t W, H;
};

struct OCfg {
    int32_t mode;       // 0 = global (3DGS) order, 1 = hierarchical, 2 = full per-pixel sort
    int32_t batch;      // tail batch B (32)
    int32_t tail;       // tail capacity (64)
    int32_t pop;        // tail -> mid chunk (16)
    int32_t mid;        // mid capacity (8)
    int32_t mid_batch;  // mid sub-batch b (4)
    int32_t head;       // head capacity K (4)
    float bg[3];
    int32_t flags;      // ablations of the hierarchical mode (ABL_*)
};

// Ablations of the hierarchical mode (Sec. 4.3, Table performance_ablation):
//   ABL_TILE_DEPTH  (B) no tile-depth adjustment: every key of a Gaussian
//                   uses its distance |mu - o| (t_opt along the ray through
//                   its own mean) instead of t_opt through the tile's x^;
//   ABL_TILE_CULL   (D) no tile-based culling: every rectangle tile is kept;
//   ABL_HIER_CULL   (E) no culling at the 4x4 and 2x2 levels of the render.
// Load balancing (C) changes no result and has no switch here.
// The global (3DGS) order has one variant (Sec. 3.3, Fig. pertiledepth):
//   TILE_CENTRE_DEPTH  every entry of a tile is keyed by t_opt along the ray
//                   through the tile's centre instead of the view depth.
enum { ABL_TILE_DEPTH = 1, ABL_TILE_CULL = 2, ABL_HIER_CULL = 4, TILE_CENTRE_DEPTH = 8 };

enum { MODE_GLOBAL = 0, MODE_HIER = 1, MODE_FULL = 2, MODE_WINDOW = 3 };

// Modes whose tile lists are those of 3DGS (3-sigma rectangle, every
// rectangle tile kept, view-space depth keys): the global order, and the
// per-ray resorting window of Sec. 3.3 that walks the same lists.
inline bool gs_lists(int mode) { return mode == MODE_GLOBAL || mode == MODE_WINDOW; }

template <class F> struct Cam {
    F R[9], t[3], o[3], fx, fy, cx, cy, znear, limx, limy, rfx, rfy;
    int W, H, tiles_x, tiles_y;
    explicit Cam(const OCam& c) {
        for (int i = 0; i < 9; ++i) R[i] = (F)c.R[i];
        for (int i = 0; i < 3; ++i) { t[i] = (F)c.t[i]; o[i] = (F)c.center[i]; }
        fx = c.fx; fy = c.fy; cx = c.cx; cy = c.cy; znear = c.znear;
        rfx = F(1) / fx;
        rfy = F(1) / fy;
        W = c.W; H = c.H;
        tiles_x = (W + 15) / 16;
        tiles_y = (H + 15) / 16;
        // Frustum clamp of the EWA Jacobian at 1.3 x the half field of view.
        limx = F(1.3) * ((F)W / (F(2) * fx));
        limy = F(1.3) * ((F)H / (F(2) * fy));
    }
    // Unit world-space ray direction through image point (u, v):
    // d_c = ((u-cx)/fx, (v-cy)/fy, 1), d_w = R^T d_c, d = d_w / |d_w|; the
    // divisions by the focal lengths as products with 1/fx and 1/fy (each
    // rounded once), each component of d_w and |d_w|^2 by fused
    // multiply-adds, and d_w scaled by the one reciprocal 1 / |d_w|.
    void ray(F u, F v, F d[3]) const {
        F a = (u - cx) * rfx, b = (v - cy) * rfy;
        F w0 = std::fma(R[3], b, std::fma(R[0], a, R[6]));
        F w1 = std::fma(R[4], b, std::fma(R[1], a, R[7]));
        F w2 = std::fma(R[5], b, std::fma(R[2], a, R[8]));
        F len = std::sqrt(std::fma(w2, w2, std::fma(w1, w1, w0 * w0)));
        F inv = F(1) / len;
        d[0] = w0 * inv; d[1] = w1 * inv; d[2] = w2 * inv;
    }
};

// Per-Gaussian record produced by preprocessing (App. B.4): 2D mean, conic and
// opacity, the six unique entries of the clamped inverse covariance, the
// vector w = Sigma^-1 (mu - o), the colour, and the global-mode depths.
template <class F> struct Rec {
    F x, y;           // 2D mean mu_2 (pixels)
    F ca, cb, cc, op; // conic (Sigma_2^-1 entries a, b, c) and opacity
    F s[6];           // Sigma^-1: s00 s01 s02 s11 s12 s22
    F w[3];           // Sigma^-1 (mu - o)
    F rgb[3];
    F z, dist;        // view-space depth and |mu - o| (global mode)
    int rect[4];      // tile rectangle x0, y0, x1, y1 (inclusive)
    bool vis;
    bool clamp_rgb[3];
    bool clamp_x, clamp_y;  // frustum clamp of the EWA Jacobian active
};

const float EPS_O_F = 1.0f / 255.0f;
template <class F> inline F eps_o() { return (F)1 / (F)255; }

// t_opt along unit direction d (Eq. dopt): d^T Sigma^-1 (mu - o) / d^T Sigma^-1 d.
// Each dot product is one multiplication followed by fused multiply-adds, in
// index order.  A NaN quotient (degenerate inverse covariance) is read as
// +infinity.
template <class F> inline F topt(const Rec<F>& g, const F d[3]) {
    F sd0 = std::fma(g.s[2], d[2], std::fma(g.s[1], d[1], g.s[0] * d[0]));
    F sd1 = std::fma(g.s[4], d[2], std::fma(g.s[3], d[1], g.s[1] * d[0]));
    F sd2 = std::fma(g.s[5], d[2], std::fma(g.s[4], d[1], g.s[2] * d[0]));
    F num = std::fma(d[2], g.w[2], std::fma(d[1], g.w[1], d[0] * g.w[0]));
    F den = std::fma(d[2], sd2, std::fma(d[1], sd1, d[0] * sd0));
    F t = num / den;
    if (t != t) t = (F)INFINITY;
    return t;
}

// Exponent of the 2D Gaussian at point (px, py):
// power = -1/2 (a dx^2 + c dy^2) - b dx dy, with d = mu_2 - p.
// (fused: -1/2 q - b dx dy with q = fma(c dy, dy, (a dx) dx) in one rounding)
template <class F> inline F power_at(const Rec<F>& g, F px, F py) {
    F dx = g.x - px, dy = g.y - py;
    F q = std::fma(g.cc * dy, dy, (g.ca * dx) * dx);
    return std::fma(F(-0.5), q, -((g.cb * dx) * dy));
}

// Algorithm 1 (App. B.1): point of the axis-aligned box [x0,x1]x[y0,y1] where
// the 2D Gaussian is largest.  If the mean is outside, the maximum lies on one
// of the two edges at the corner closest to the mean; a 1D line search along
// each edge (the 2D analogue of Eq. dopt), clamped to the edge, finds it.
template <class F> void alg1_max_point(const Rec<F>& g, F x0, F x1, F y0, F y1, F& hx, F& hy) {
    const F mx = g.x, my = g.y;
    const bool in_x = (x0 <= mx && mx <= x1), in_y = (y0 <= my && my <= y1);
    if (in_x && in_y) { hx = mx; hy = my; return; }
    // Closest corner p and the edge vectors towards the neighbouring corners.
    F px = (mx < x0) ? x0 : ((mx > x1) ? x1 : ((mx - x0 <= x1 - mx) ? x0 : x1));
    F py = (my < y0) ? y0 : ((my > y1) ? y1 : ((my - y0 <= y1 - my) ? y0 : y1));
    F lx = ((px == x0) ? x1 : x0) - px;   // d_x = (lx, 0)
    F ly = ((py == y0) ? y1 : y0) - py;   // d_y = (0, ly)
    F dx = mx - px, dy = my - py;         // mu_2 - p
    F tx = F(0), ty = F(0);
    if (!in_x && ly != F(0)) {
        // t_y = d_y^T C (mu - p) / d_y^T C d_y  with d_y = (0, ly)
        ty = sclamp(std::fma(g.cb, dx, g.cc * dy) / (g.cc * ly), F(0), F(1));
    }
    if (!in_y && lx != F(0)) {
        tx = sclamp(std::fma(g.ca, dx, g.cb * dy) / (g.ca * lx), F(0), F(1));
    }
    hx = std::fma(tx, lx, px);
    hy = std::fma(ty, ly, py);
}

// Culling test shared by every level: the Gaussian is kept for a region iff
// its largest value there clears the opacity threshold eps_O = 1/255 (Sec. 3.4).
template <class F> inline bool keep_at(const Rec<F>& g, F hx, F hy) {
    F p = power_at(g, hx, hy);
    return p <= F(0) && g.op * expE(p) >= eps_o<F>();
}

// Pixel-centre hull of a block: [x0, min(x0+size-1, W-1)] x [...].
template <class F> inline void hull(const Cam<F>& cam, int x0, int y0, int size, F& a, F& b, F& c, F& d) {
    a = (F)x0; b = (F)std::min(x0 + size - 1, cam.W - 1);
    c = (F)y0; d = (F)std::min(y0 + size - 1, cam.H - 1);
}

template <class F> inline bool keep_block(const Rec<F>& g, F x0, F x1, F y0, F y1, F& hx, F& hy) {
    alg1_max_point(g, x0, x1, y0, y1, hx, hy);
    return keep_at(g, hx, hy);
}

// ---------------------------------------------------------------------------
// Preprocess (Sec. 2.1 projection kept as in 3DGS, App. A inverse covariance,
// App. B.2 opacity-aware bound, App. B.4 packing).
// ---------------------------------------------------------------------------
template <class F>
void preprocess_one(const Cam<F>& cam, int mode, int deg, const float* mu_in, const float* s_in,
                    const float* q_in, float op_in, const float* sh_in, Rec<F>& g) {
    std::memset(&g, 0, sizeof(g));
    g.vis = false;
    F mu[3] = {(F)mu_in[0], (F)mu_in[1], (F)mu_in[2]};
    F s[3] = {(F)s_in[0], (F)s_in[1], (F)s_in[2]};
    F q[4] = {(F)q_in[0], (F)q_in[1], (F)q_in[2], (F)q_in[3]};
    F op = (F)op_in;
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(mu[i]) || !std::isfinite(s[i]) || !(s[i] > F(0))) return;
    for (int i = 0; i < 4; ++i)
        if (!std::isfinite(q[i])) return;
    if (!std::isfinite(op)) return;

    // Rotation from the quaternion (w, x, y, z); a zero quaternion is the identity.
    F n2 = ((q[0] * q[0] + q[1] * q[1]) + q[2] * q[2]) + q[3] * q[3];
    F qw = 1, qx = 0, qy = 0, qz = 0;
    if (n2 != F(0)) {
        F nrm = std::sqrt(n2);
        qw = q[0] / nrm; qx = q[1] / nrm; qy = q[2] / nrm; qz = q[3] / nrm;
    }
    F Rq[3][3];
    Rq[0][0] = F(1) - F(2) * (qy * qy + qz * qz);
    Rq[0][1] = F(2) * (qx * qy - qw * qz);
    Rq[0][2] = F(2) * (qx * qz + qw * qy);
    Rq[1][0] = F(2) * (qx * qy + qw * qz);
    Rq[1][1] = F(1) - F(2) * (qx * qx + qz * qz);
    Rq[1][2] = F(2) * (qy * qz - qw * qx);
    Rq[2][0] = F(2) * (qx * qz - qw * qy);
    Rq[2][1] = F(2) * (qy * qz + qw * qx);
    Rq[2][2] = F(1) - F(2) * (qx * qx + qy * qy);

    // Sigma = R S S^T R^T (Sec. 2.1).
    F s2[3] = {s[0] * s[0], s[1] * s[1], s[2] * s[2]};
    // Each symmetric matrix is formed on and above the diagonal and mirrored.
    F Sg[3][3];
    for (int j = 0; j < 3; ++j)
        for (int k = j; k < 3; ++k) {
            Sg[j][k] = ((Rq[j][0] * s2[0]) * Rq[k][0] + (Rq[j][1] * s2[1]) * Rq[k][1]) + (Rq[j][2] * s2[2]) * Rq[k][2];
            Sg[k][j] = Sg[j][k];
        }

    // Sigma^-1 = R S^-2 R^T with the entries of S^-1 bounded by 10^3 (Sec. 3.2, App. A).
    F si2[3];
    for (int l = 0; l < 3; ++l) {
        F si = F(1) / s[l];
        si = (si > F(1000)) ? F(1000) : si;
        si2[l] = si * si;
    }
    F Si[3][3];
    for (int j = 0; j < 3; ++j)
        for (int k = j; k < 3; ++k) {
            Si[j][k] = ((Rq[j][0] * si2[0]) * Rq[k][0] + (Rq[j][1] * si2[1]) * Rq[k][1]) + (Rq[j][2] * si2[2]) * Rq[k][2];
            Si[k][j] = Si[j][k];
        }

    F dm[3] = {mu[0] - cam.o[0], mu[1] - cam.o[1], mu[2] - cam.o[2]};
    F w[3];
    for (int j = 0; j < 3; ++j) w[j] = (Si[j][0] * dm[0] + Si[j][1] * dm[1]) + Si[j][2] * dm[2];

    // Camera space and near-plane cull.
    F p[3];
    for (int j = 0; j < 3; ++j)
        p[j] = ((cam.R[3 * j] * mu[0] + cam.R[3 * j + 1] * mu[1]) + cam.R[3 * j + 2] * mu[2]) + cam.t[j];
    if (!(p[2] > cam.znear)) return;

    // EWA splatting (Zwicker et al. 2002) as in 3DGS: Jacobian of the perspective
    // map with the frustum clamp, Sigma_2 = J W Sigma W^T J^T + 0.3 I.
    F txtz = p[0] / p[2], tytz = p[1] / p[2];
    F xcl = sclamp(txtz, -cam.limx, cam.limx) * p[2];
    F ycl = sclamp(tytz, -cam.limy, cam.limy) * p[2];
    F pz2 = p[2] * p[2];
    F J00 = cam.fx / p[2], J02 = -(cam.fx * xcl) / pz2;
    F J11 = cam.fy / p[2], J12 = -(cam.fy * ycl) / pz2;
    F T[2][3];
    for (int k = 0; k < 3; ++k) {
        T[0][k] = J00 * cam.R[k] + J02 * cam.R[6 + k];
        T[1][k] = J11 * cam.R[3 + k] + J12 * cam.R[6 + k];
    }
    F U[2][3];
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 3; ++k)
            U[j][k] = (T[j][0] * Sg[0][k] + T[j][1] * Sg[1][k]) + T[j][2] * Sg[2][k];
    F a = ((U[0][0] * T[0][0] + U[0][1] * T[0][1]) + U[0][2] * T[0][2]) + F(0.3);
    F b = (U[0][0] * T[1][0] + U[0][1] * T[1][1]) + U[0][2] * T[1][2];
    F c = ((U[1][0] * T[1][0] + U[1][1] * T[1][1]) + U[1][2] * T[1][2]) + F(0.3);
    F det = a * c - b * b;
    if (!(det > F(0))) return;
    const F ca = c / det, cb = (-b) / det, cc = a / det;
    const F mx = cam.fx * txtz + cam.cx;
    const F my = cam.fy * tytz + cam.cy;

    // Opacity below eps_O can never contribute.
    if (!(op >= eps_o<F>())) return;

    // Bounding radius from the largest eigenvalue of Sigma_2.
    F mid = F(0.5) * (a + c);
    F lam = mid + std::sqrt(smax(F(0.1), mid * mid - det));
    F rr;
    if (gs_lists(mode)) {
        // 3DGS: a 3-sigma circle.
        rr = std::ceil(F(3) * std::sqrt(lam));
    } else {
        // Opacity-aware bound t_O = sqrt(2 ln(o / eps_O)) (App. B.2), widened by
        // 1/256 and one pixel so that only exact culling decides the kept set.
        F tO = std::sqrt(F(2) * lnE(op / eps_o<F>()));
        F r = tO * std::sqrt(lam);  // radius
        rr = r * F(1.00390625) + F(1);
    }
    // Tiles whose pixel-centre hull meets [x - rr, x + rr] x [y - rr, y + rr].
    F fx0 = std::ceil(((mx - rr) - F(15)) / F(16));
    F fx1 = std::floor((mx + rr) / F(16));
    F fy0 = std::ceil(((my - rr) - F(15)) / F(16));
    F fy1 = std::floor((my + rr) / F(16));
    fx0 = sclamp(fx0, F(0), (F)cam.tiles_x);
    fy0 = sclamp(fy0, F(0), (F)cam.tiles_y);
    fx1 = sclamp(fx1, F(-1), (F)(cam.tiles_x - 1));
    fy1 = sclamp(fy1, F(-1), (F)(cam.tiles_y - 1));
    if (!(fx0 <= fx1) || !(fy0 <= fy1)) return;

    // View-dependent colour from SH with the direction camera -> mean (App. B.4).
    F len = std::sqrt((dm[0] * dm[0] + dm[1] * dm[1]) + dm[2] * dm[2]);
    F dir[3] = {dm[0] / len, dm[1] / len, dm[2] / len};
    F bas[16];
    sh_basis<F>(deg, dir[0], dir[1], dir[2], bas);
    int K = (deg + 1) * (deg + 1);
    F rgb[3];
    bool clamped[3];
    for (int ch = 0; ch < 3; ++ch) {
        F acc = bas[0] * (F)sh_in[ch];
        for (int k = 1; k < K; ++k) acc = acc + bas[k] * (F)sh_in[3 * k + ch];
        acc = acc + F(0.5);
        if (!std::isfinite(acc)) return;
        clamped[ch] = acc < F(0);
        rgb[ch] = acc < F(0) ? F(0) : acc;
    }
    // Visible: write the record.
    g.x = mx; g.y = my;
    g.ca = ca; g.cb = cb; g.cc = cc; g.op = op;
    g.clamp_x = !(-cam.limx <= txtz && txtz <= cam.limx);
    g.clamp_y = !(-cam.limy <= tytz && tytz <= cam.limy);
    g.rect[0] = (int)fx0; g.rect[1] = (int)fy0; g.rect[2] = (int)fx1; g.rect[3] = (int)fy1;
    for (int ch = 0; ch < 3; ++ch) { g.rgb[ch] = rgb[ch]; g.clamp_rgb[ch] = clamped[ch]; }
    g.s[0] = Si[0][0]; g.s[1] = Si[0][1]; g.s[2] = Si[0][2];
    g.s[3] = Si[1][1]; g.s[4] = Si[1][2]; g.s[5] = Si[2][2];
    g.w[0] = w[0]; g.w[1] = w[1]; g.w[2] = w[2];
    g.z = p[2];
    g.dist = len;
    g.vis = true;
}

// Number of rectangle tiles the Gaussian is kept for.  In hierarchical and
// full modes every rectangle tile goes through Algorithm 1; the global mode
// keeps every rectangle tile (3DGS).
template <class F> int count_tiles(const Cam<F>& cam, int mode, int flags, const Rec<F>& g) {
    if (!g.vis) return 0;
    int n = 0;
    for (int ty = g.rect[1]; ty <= g.rect[3]; ++ty)
        for (int tx = g.rect[0]; tx <= g.rect[2]; ++tx) {
            if (gs_lists(mode) || (flags & ABL_TILE_CULL)) { ++n; continue; }
            F a, b, c, d, hx, hy;
            hull(cam, tx * 16, ty * 16, 16, a, b, c, d);
            if (keep_block(g, a, b, c, d, hx, hy)) ++n;
        }
    return n;
}

// One (tile, Gaussian) sort entry: tile id, depth key, Gaussian id.
struct Entry {
    u32 tile;
    u64 dkey;
    u32 id;
    bool operator<(const Entry& o) const {
        if (tile != o.tile) return tile < o.tile;
        if (dkey != o.dkey) return dkey < o.dkey;
        return id < o.id;
    }
};

// Duplication (Sec. 2.1 keys; Sec. 3.4 tile-depth adjustment): for every kept
// tile the depth is t_opt along the ray through the tile's maximum point x^.
template <class F> void emit_entries(const Cam<F>& cam, int mode, int flags, const Rec<F>& g, u32 id,
                                     std::vector<Entry>& out) {
    if (!g.vis) return;
    for (int ty = g.rect[1]; ty <= g.rect[3]; ++ty)
        for (int tx = g.rect[0]; tx <= g.rect[2]; ++tx) {
            u32 tile = (u32)(ty * cam.tiles_x + tx);
            F a, b, c, d, hx, hy;
            hull(cam, tx * 16, ty * 16, 16, a, b, c, d);
            if (gs_lists(mode) && (flags & TILE_CENTRE_DEPTH)) {
                F dir[3];
                cam.ray(F(0.5) * (a + b), F(0.5) * (c + d), dir);
                out.push_back({tile, ord_key(topt(g, dir)), id});
                continue;
            }
            if (gs_lists(mode)) { out.push_back({tile, ord_key(g.z), id}); continue; }
            const bool keep = keep_block(g, a, b, c, d, hx, hy);
            if (!keep && !(flags & ABL_TILE_CULL)) continue;
            if (flags & ABL_TILE_DEPTH) { out.push_back({tile, ord_key(g.dist), id}); continue; }
            F dir[3];
            cam.ray(hx, hy, dir);
            out.push_back({tile, ord_key(topt(g, dir)), id});
        }
}

// ---------------------------------------------------------------------------
// Per-pixel blending state (Eq. volume_desc, front to back, with the 3DGS
// conventions: alpha = min(0.99, o G_2), skip alpha < 1/255, stop before the
// transmittance would fall below 10^-4).
// ---------------------------------------------------------------------------
template <class F> struct Pixel {
    F T = 1, C[3] = {0, 0, 0}, D = 0;
    int n = 0;
    bool done = false;
    std::vector<int> ids;     // blended ids in order
    std::vector<F> ts;        // their per-pixel depths (for the sort error)
    std::vector<F> alphas;    // their alphas (for the backward pass)
};

template <class F> inline void blend(Pixel<F>& px, const Rec<F>& g, F alpha, F t, int id, bool depth_is_dist) {
    if (px.done) return;
    F Tn = px.T * (F(1) - alpha);
    if (Tn < F(0.0001)) { px.done = true; return; }
    // front-to-back compositing (Eq. volume_desc), each term added by a fused multiply-add
    for (int ch = 0; ch < 3; ++ch) px.C[ch] = std::fma(g.rgb[ch] * alpha, px.T, px.C[ch]);
    F phi = depth_is_dist ? g.dist : t;
    px.D = std::fma(phi * alpha, px.T, px.D);
    px.n += 1;
    px.T = Tn;
    px.ids.push_back(id);
    px.ts.push_back(t);
    px.alphas.push_back(alpha);
}

// alpha of Gaussian g at pixel (u, v); returns false when it is skipped.
template <class F> inline bool pixel_alpha(const Rec<F>& g, F u, F v, F& alpha) {
    F p = power_at(g, u, v);
    if (p > F(0)) return false;
    F a = g.op * expE(p);
    alpha = a < F(0.99) ? a : F(0.99);
    return !(alpha < eps_o<F>());
}

// ---------------------------------------------------------------------------
// Hierarchical per-pixel resorting (Sec. 3.4, Fig. pipeline, App. B.4).
// Queue elements are ordered by (depth key, rank) where rank is the position
// in the tile's key-sorted list; this total order makes the result of every
// sort and merge unique.
// ---------------------------------------------------------------------------
struct QE {
    u64 k;
    u32 rank;
    int id;
    bool operator<(const QE& o) const { return k != o.k ? k < o.k : rank < o.rank; }
};
template <class F> struct HE {
    u64 k;
    u32 rank;
    int id;
    F alpha, t;
    bool before(const HE& o) const { return k != o.k ? k < o.k : rank < o.rank; }
};

struct HierStats {
    long long tail_in = 0, mid_in = 0, head_in = 0, blends = 0;
    int max_tail = 0, max_mid = 0, max_head = 0;
    int min_tail_after_pop = 1 << 30;
    bool sorted_ok = true;
};

template <class F> struct HierSubtile {
    const Cam<F>& cam;
    const OCfg& cfg;
    const std::vector<Rec<F>>& recs;
    int x0, y0;                 // sub-tile origin
    F sx0, sx1, sy0, sy1;       // sub-tile hull
    F dS[3];                    // sub-tile centre ray
    F qh[4][4];                 // quadrant hulls
    F dQ[4][3];                 // quadrant centre rays
    bool qexists[4];
    int pidx[4][4];             // pixel index (y*W+x) per quadrant lane, -1 if outside
    F pd[4][4][3];              // pixel rays
    std::vector<QE> tail;
    std::vector<QE> mid[4];
    std::vector<HE<F>> head[4][4];
    std::vector<Pixel<F>>& pix;
    HierStats& st;

    HierSubtile(const Cam<F>& c, const OCfg& cf, const std::vector<Rec<F>>& r, int ox, int oy,
                std::vector<Pixel<F>>& px, HierStats& s)
        : cam(c), cfg(cf), recs(r), x0(ox), y0(oy), pix(px), st(s) {
        hull(cam, x0, y0, 4, sx0, sx1, sy0, sy1);
        cam.ray(F(0.5) * (sx0 + sx1), F(0.5) * (sy0 + sy1), dS);
        for (int q = 0; q < 4; ++q) {
            int qx = x0 + 2 * (q & 1), qy = y0 + 2 * (q >> 1);
            qexists[q] = qx < cam.W && qy < cam.H;
            hull(cam, qx, qy, 2, qh[q][0], qh[q][1], qh[q][2], qh[q][3]);
            cam.ray(F(0.5) * (qh[q][0] + qh[q][1]), F(0.5) * (qh[q][2] + qh[q][3]), dQ[q]);
            for (int l = 0; l < 4; ++l) {
                int px_ = qx + (l & 1), py_ = qy + (l >> 1);
                pidx[q][l] = (px_ < cam.W && py_ < cam.H) ? py_ * cam.W + px_ : -1;
                if (pidx[q][l] >= 0) cam.ray((F)px_, (F)py_, pd[q][l]);
            }
        }
    }

    static std::vector<QE> merge_sorted(const std::vector<QE>& a, const std::vector<QE>& b) {
        std::vector<QE> out(a.size() + b.size());
        std::merge(a.begin(), a.end(), b.begin(), b.end(), out.begin());
        return out;
    }
    static std::vector<QE> pop_front(std::vector<QE>& q, size_t n) {
        std::vector<QE> out(q.begin(), q.begin() + n);
        q.erase(q.begin(), q.begin() + n);
        return out;
    }

    void blend_front(int q, int l) {
        HE<F> e = head[q][l].front();
        head[q][l].erase(head[q][l].begin());
        blend(pix[pidx[q][l]], recs[e.id], e.alpha, e.t, e.id, false);
        st.blends += 1;
    }

    // Head level: per pixel, alpha test, insertion by (t_pixel, rank), and
    // blending of the front element whenever the head holds more than K.
    void push_head(int q, const std::vector<QE>& elems) {
        for (const QE& e : elems) {
            const Rec<F>& g = recs[e.id];
            for (int l = 0; l < 4; ++l) {
                if (pidx[q][l] < 0) continue;
                Pixel<F>& P = pix[pidx[q][l]];
                if (P.done) continue;
                int px_ = x0 + 2 * (q & 1) + (l & 1), py_ = y0 + 2 * (q >> 1) + (l >> 1);
                F alpha;
                if (!pixel_alpha(g, (F)px_, (F)py_, alpha)) continue;
                F t = topt(g, pd[q][l]);
                HE<F> h{ord_key(t), e.rank, e.id, alpha, t};
                auto& H = head[q][l];
                size_t pos = 0;
                while (pos < H.size() && H[pos].before(h)) ++pos;
                H.insert(H.begin() + pos, h);
                st.head_in += 1;
                st.max_head = std::max(st.max_head, (int)H.size());
                if ((int)H.size() > cfg.head) blend_front(q, l);
            }
        }
    }

    // Mid level: sub-batches of b entries are culled against the 2x2 block,
    // keyed by t_opt along the block's centre ray, sorted and merged; while
    // the mid queue holds more than (capacity - b) elements, b go to the head.
    void push_mid(const std::vector<QE>& chunk) {
        for (int q = 0; q < 4; ++q) {
            if (!qexists[q]) continue;
            for (size_t r0 = 0; r0 < chunk.size(); r0 += cfg.mid_batch) {
                std::vector<QE> nv;
                for (size_t j = r0; j < std::min(chunk.size(), r0 + (size_t)cfg.mid_batch); ++j) {
                    const Rec<F>& g = recs[chunk[j].id];
                    F hx, hy;
                    if (!(cfg.flags & ABL_HIER_CULL) && !keep_block(g, qh[q][0], qh[q][1], qh[q][2], qh[q][3], hx, hy))
                        continue;
                    nv.push_back({ord_key(topt(g, dQ[q])), chunk[j].rank, chunk[j].id});
                }
                std::sort(nv.begin(), nv.end());
                st.mid_in += (long long)nv.size();
                mid[q] = merge_sorted(mid[q], nv);
                st.max_mid = std::max(st.max_mid, (int)mid[q].size());
                while ((int)mid[q].size() > cfg.mid - cfg.mid_batch) push_head(q, pop_front(mid[q], cfg.mid_batch));
            }
        }
    }

    // Tail level over the tile list [begin, end) of sorted ids.
    void run(const u32* ids, u32 begin, u32 end) {
        for (u32 b0 = begin; b0 < end; b0 += (u32)cfg.batch) {
            std::vector<QE> nv;
            for (u32 e = b0; e < std::min(end, b0 + (u32)cfg.batch); ++e) {
                const Rec<F>& g = recs[ids[e]];
                F hx, hy;
                if (!(cfg.flags & ABL_HIER_CULL) && !keep_block(g, sx0, sx1, sy0, sy1, hx, hy)) continue;
                nv.push_back({ord_key(topt(g, dS)), e - begin, (int)ids[e]});
            }
            std::sort(nv.begin(), nv.end());
            st.tail_in += (long long)nv.size();
            tail = merge_sorted(tail, nv);
            st.max_tail = std::max(st.max_tail, (int)tail.size());
            bool popped = false;
            while ((int)tail.size() > cfg.tail - cfg.batch) {
                push_mid(pop_front(tail, cfg.pop));
                popped = true;
            }
            if (popped) st.min_tail_after_pop = std::min(st.min_tail_after_pop, (int)tail.size());
        }
        // Drain: the rest of the tail in chunks, then every mid queue, then every head.
        while (!tail.empty()) push_mid(pop_front(tail, std::min((size_t)cfg.pop, tail.size())));
        for (int q = 0; q < 4; ++q) {
            if (!qexists[q]) continue;
            while (!mid[q].empty()) push_head(q, pop_front(mid[q], std::min((size_t)cfg.mid_batch, mid[q].size())));
            for (int l = 0; l < 4; ++l) {
                if (pidx[q][l] < 0) continue;
                while (!head[q][l].empty()) blend_front(q, l);
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Whole frame.
// ---------------------------------------------------------------------------
template <class F> struct Frame {
    Cam<F> cam;
    OCfg cfg;
    std::vector<Rec<F>> recs;
    std::vector<int> touched;
    std::vector<Entry> entries;   // sorted
    std::vector<u32> range_lo, range_hi;
    std::vector<Pixel<F>> pix;
    HierStats stats;
    double ms[4] = {0, 0, 0, 0};  // preprocess, duplicate, sort, render (wall clock)
    Frame(const OCam& c, const OCfg& f) : cam(c), cfg(f) {}
};

inline double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

template <class F>
void run_frame(Frame<F>& fr, int n, int deg, const float* means, const float* scales, const float* rots,
               const float* opac, const float* sh, const uint8_t* tile_mask) {
    const Cam<F>& cam = fr.cam;
    const int mode = fr.cfg.mode;
    const int K = (deg + 1) * (deg + 1);
    fr.recs.assign(n, Rec<F>());
    fr.touched.assign(n, 0);
    double t0 = now_ms();
#pragma omp parallel for schedule(dynamic, 256)
    for (int i = 0; i < n; ++i) {
        preprocess_one<F>(cam, mode, deg, means + 3 * i, scales + 3 * i, rots + 4 * i, opac[i], sh + 3 * K * i, fr.recs[i]);
        fr.touched[i] = (mode == MODE_FULL) ? 0 : count_tiles(cam, mode, fr.cfg.flags, fr.recs[i]);
    }
    const int ntiles = cam.tiles_x * cam.tiles_y;
    fr.ms[0] = now_ms() - t0;
    fr.pix.assign((size_t)cam.W * cam.H, Pixel<F>());
    if (mode == MODE_FULL) {
        // Brute force (Sec. 3.2): every visible Gaussian, per pixel, sorted by
        // (t_opt along the pixel ray, id), blended front to back.
#pragma omp parallel for schedule(dynamic, 1)
        for (int y = 0; y < cam.H; ++y)
            for (int x = 0; x < cam.W; ++x) {
                F d[3];
                cam.ray((F)x, (F)y, d);
                std::vector<std::pair<std::pair<u64, int>, F>> c;
                std::vector<F> al;
                for (int i = 0; i < n; ++i) {
                    const Rec<F>& g = fr.recs[i];
                    if (!g.vis) continue;
                    F a;
                    if (!pixel_alpha(g, (F)x, (F)y, a)) continue;
                    F t = topt(g, d);
                    c.push_back({{ord_key(t), i}, t});
                }
                std::sort(c.begin(), c.end(), [](const auto& A, const auto& B) { return A.first < B.first; });
                Pixel<F>& P = fr.pix[(size_t)y * cam.W + x];
                for (auto& e : c) {
                    if (P.done) break;
                    F a;
                    pixel_alpha(fr.recs[e.first.second], (F)x, (F)y, a);
                    blend(P, fr.recs[e.first.second], a, e.second, e.first.second, false);
                }
            }
        return;
    }
    // Duplicate in Gaussian order, then sort by (tile, depth key, id).
    t0 = now_ms();
    std::vector<std::vector<Entry>> per(n);
#pragma omp parallel for schedule(dynamic, 256)
    for (int i = 0; i < n; ++i) emit_entries(cam, mode, fr.cfg.flags, fr.recs[i], (u32)i, per[i]);
    fr.entries.clear();
    for (int i = 0; i < n; ++i) {
        fr.entries.insert(fr.entries.end(), per[i].begin(), per[i].end());
        std::vector<Entry>().swap(per[i]);
    }
    fr.ms[1] = now_ms() - t0;
    t0 = now_ms();
    std::sort(fr.entries.begin(), fr.entries.end());
    fr.range_lo.assign(ntiles, 0);
    fr.range_hi.assign(ntiles, 0);
    for (size_t e = 0; e < fr.entries.size(); ++e) {
        u32 t = fr.entries[e].tile;
        if (e == 0 || fr.entries[e - 1].tile != t) fr.range_lo[t] = (u32)e;
        if (e + 1 == fr.entries.size() || fr.entries[e + 1].tile != t) fr.range_hi[t] = (u32)(e + 1);
    }
    std::vector<u32> ids(fr.entries.size());
    for (size_t e = 0; e < ids.size(); ++e) ids[e] = fr.entries[e].id;
    fr.ms[2] = now_ms() - t0;
    t0 = now_ms();

    if (mode == MODE_GLOBAL) {
        // Each pixel blends its tile's list in key order (3DGS).
#pragma omp parallel for schedule(dynamic, 1)
        for (int tile = 0; tile < ntiles; ++tile) {
            if (tile_mask && !tile_mask[tile]) continue;
            int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
            for (int y = ty * 16; y < std::min(ty * 16 + 16, cam.H); ++y)
                for (int x = tx * 16; x < std::min(tx * 16 + 16, cam.W); ++x) {
                    Pixel<F>& P = fr.pix[(size_t)y * cam.W + x];
                    F d[3];
                    cam.ray((F)x, (F)y, d);
                    for (u32 e = fr.range_lo[tile]; e < fr.range_hi[tile] && !P.done; ++e) {
                        const Rec<F>& g = fr.recs[ids[e]];
                        F a;
                        if (!pixel_alpha(g, (F)x, (F)y, a)) continue;
                        // Depth output uses |mu - o|; the per-pixel t_opt is kept for the sort error.
                        blend(P, g, a, topt(g, d), (int)ids[e], true);
                    }
                }
        }
        fr.ms[3] = now_ms() - t0;
        return;
    }
    if (mode == MODE_WINDOW) {
        // Per-ray resorting (Sec. 3.3): each pixel walks its tile's 3DGS list;
        // a sample that passes the alpha test is placed by insertion into a
        // window ordered by (t_opt along the pixel ray, rank in the list); when
        // the window holds more than cfg.head samples its front is blended.
        // The walk stops once the pixel has terminated; at the end of the list
        // the window is blended in order.
#pragma omp parallel for schedule(dynamic, 1)
        for (int tile = 0; tile < ntiles; ++tile) {
            if (tile_mask && !tile_mask[tile]) continue;
            int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
            const u32 lo = fr.range_lo[tile], hi = fr.range_hi[tile];
            for (int y = ty * 16; y < std::min(ty * 16 + 16, cam.H); ++y)
                for (int x = tx * 16; x < std::min(tx * 16 + 16, cam.W); ++x) {
                    Pixel<F>& P = fr.pix[(size_t)y * cam.W + x];
                    F d[3];
                    cam.ray((F)x, (F)y, d);
                    std::vector<HE<F>> win;
                    for (u32 e = lo; e < hi && !P.done; ++e) {
                        const Rec<F>& g = fr.recs[ids[e]];
                        F a;
                        if (!pixel_alpha(g, (F)x, (F)y, a)) continue;
                        const F t = topt(g, d);
                        HE<F> h{ord_key(t), e - lo, (int)ids[e], a, t};
                        size_t pos = 0;
                        while (pos < win.size() && win[pos].before(h)) ++pos;
                        win.insert(win.begin() + pos, h);
                        if ((int)win.size() > fr.cfg.head) {
                            const HE<F> f = win.front();
                            win.erase(win.begin());
                            blend(P, fr.recs[f.id], f.alpha, f.t, f.id, false);
                        }
                    }
                    for (const HE<F>& f : win) blend(P, fr.recs[f.id], f.alpha, f.t, f.id, false);
                }
        }
        fr.ms[3] = now_ms() - t0;
        return;
    }
    // Hierarchical: every 4x4 sub-tile runs its queues independently.
    const int sub_x = (cam.W + 3) / 4, sub_y = (cam.H + 3) / 4;
    std::vector<HierStats> sts((size_t)sub_x * sub_y);
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < sub_x * sub_y; ++s) {
        int sx = s % sub_x, sy = s / sub_x;
        int tile = (sy / 4) * cam.tiles_x + (sx / 4);
        if (tile_mask && !tile_mask[tile]) continue;
        HierSubtile<F> H(cam, fr.cfg, fr.recs, sx * 4, sy * 4, fr.pix, sts[s]);
        H.run(ids.data(), fr.range_lo[tile], fr.range_hi[tile]);
    }
    fr.ms[3] = now_ms() - t0;
    for (auto& s : sts) {
        fr.stats.tail_in += s.tail_in; fr.stats.mid_in += s.mid_in; fr.stats.head_in += s.head_in;
        fr.stats.blends += s.blends;
        fr.stats.max_tail = std::max(fr.stats.max_tail, s.max_tail);
        fr.stats.max_mid = std::max(fr.stats.max_mid, s.max_mid);
        fr.stats.max_head = std::max(fr.stats.max_head, s.max_head);
        fr.stats.min_tail_after_pop = std::min(fr.stats.min_tail_after_pop, s.min_tail_after_pop);
    }
}


// ---------------------------------------------------------------------------
// Backward pass (Sec. 3.5).  The image is C = sum_i c_i alpha_i T_i + T_N bg
// over each pixel's blend sequence (Eq. volume_desc).  Front to back, the
// colour of everything behind Gaussian i is C - C_i (C_i: accumulated colour
// including i) and the transmittance behind it is T_N / T_{i+1}, so
//   dC/dc_i     = alpha_i T_i
//   dC/dalpha_i = c_i T_i - (C - C_i + T_N bg) / (1 - alpha_i).
// The order (t_opt, culling, termination) is piecewise constant and carries
// no gradient; clamped quantities (alpha at 0.99, colour at 0, the frustum
// clamp of the Jacobian) pass none through the clamped variable.
// ---------------------------------------------------------------------------
template <class F> struct G2 {
    F mx = 0, my = 0, ca = 0, cb = 0, cc = 0, op = 0, rgb[3] = {0, 0, 0};
};

// With `bound` given, each 2D component also accumulates a bound on the
// magnitudes its terms are computed from (every difference and sum of the
// term taken with absolute values), and `nterms` counts the Gaussian's blends:
// a float32 evaluation of the same sums in any order differs from the exact
// ones by at most about (nterms + ops per term) * 2^-24 * bound (first-order
// running-error analysis).  The bound carries no gradient information.
//
// The terms are evaluated in F from a frame rendered in FD: the blend
// sequences, alphas, records, final colours and transmittances are the FD
// frame's, and so are the decisions (whether the alpha clamp was active), so
// that F = double over an FD = float frame differentiates exactly the branch
// that the float32 forward took (the order, culling and termination are
// piecewise constant, Sec. 3.5); only the arithmetic of the terms is F.
template <class F, class FD> Rec<F> rec_as(const Rec<FD>& r) {
    Rec<F> g;
    g.x = (F)r.x; g.y = (F)r.y;
    g.ca = (F)r.ca; g.cb = (F)r.cb; g.cc = (F)r.cc; g.op = (F)r.op;
    for (int k = 0; k < 6; ++k) g.s[k] = (F)r.s[k];
    for (int k = 0; k < 3; ++k) { g.w[k] = (F)r.w[k]; g.rgb[k] = (F)r.rgb[k]; g.clamp_rgb[k] = r.clamp_rgb[k]; }
    g.z = (F)r.z; g.dist = (F)r.dist;
    for (int k = 0; k < 4; ++k) g.rect[k] = r.rect[k];
    g.vis = r.vis; g.clamp_x = r.clamp_x; g.clamp_y = r.clamp_y;
    return g;
}

template <class F, class FD = F>
void backward_blends(const Frame<FD>& fr, const F* dL, const float bg[3], std::vector<G2<F>>& g2,
                     std::vector<G2<F>>* bound = nullptr, std::vector<int>* nterms = nullptr) {
    const Cam<FD>& cam = fr.cam;
    const size_t P = (size_t)cam.W * cam.H;
    for (int y = 0; y < cam.H; ++y)
        for (int x = 0; x < cam.W; ++x) {
            const size_t p = (size_t)y * cam.W + x;
            const Pixel<FD>& px = fr.pix[p];
            const F TN = (F)px.T;
            const F Cfin[3] = {(F)px.C[0], (F)px.C[1], (F)px.C[2]};
            F T = 1, Cacc[3] = {0, 0, 0};
            for (size_t k = 0; k < px.ids.size(); ++k) {
                const int id = px.ids[k];
                const F a = (F)px.alphas[k];
                const Rec<FD>& gd = fr.recs[id];
                const Rec<F> g = rec_as<F>(gd);
                for (int ch = 0; ch < 3; ++ch) Cacc[ch] = std::fma(g.rgb[ch] * a, T, Cacc[ch]);
                F ga = 0, ga_m = 0;
                for (int ch = 0; ch < 3; ++ch) {
                    const F dl = dL[ch * P + p];
                    g2[id].rgb[ch] += dl * a * T;
                    ga += dl * (g.rgb[ch] * T - (Cfin[ch] - Cacc[ch] + TN * (F)bg[ch]) / (F(1) - a));
                    if (bound) {
                        (*bound)[id].rgb[ch] += std::abs(dl) * a * T;
                        ga_m += std::abs(dl) * (std::abs(g.rgb[ch]) * T +
                                                (std::abs(Cfin[ch]) + std::abs(Cacc[ch]) + TN * std::abs((F)bg[ch])) /
                                                    (F(1) - a));
                    }
                }
                if (nterms) (*nterms)[id] += 1;
                const F pw = power_at(g, (F)x, (F)y);
                const F G = expE(pw);
                // the clamp decision of the forward's arithmetic
                if (gd.op * expE(power_at(gd, (FD)x, (FD)y)) < FD(0.99)) {
                    g2[id].op += ga * G;
                    const F gp = ga * a;  // d alpha / d power = o G = alpha
                    const F dx = g.x - (F)x, dy = g.y - (F)y;
                    g2[id].mx += gp * (-g.ca * dx - g.cb * dy);
                    g2[id].my += gp * (-g.cc * dy - g.cb * dx);
                    g2[id].ca += gp * (F(-0.5) * dx * dx);
                    g2[id].cb += gp * (-dx * dy);
                    g2[id].cc += gp * (F(-0.5) * dy * dy);
                    if (bound) {
                        G2<F>& b = (*bound)[id];
                        const F gm = ga_m * a, adx = std::abs(dx), ady = std::abs(dy);
                        b.op += ga_m * G;
                        b.mx += gm * (std::abs(g.ca) * adx + std::abs(g.cb) * ady);
                        b.my += gm * (std::abs(g.cc) * ady + std::abs(g.cb) * adx);
                        b.ca += gm * (F(0.5) * adx * adx);
                        b.cb += gm * (adx * ady);
                        b.cc += gm * (F(0.5) * ady * ady);
                    }
                }
                T = T * (F(1) - a);
            }
        }
}

// Chain rule from the 2D quantities back to the Gaussian parameters through
// the colour (SH), the conic (EWA, Sigma = R S S^T R^T) and the 2D mean.
template <class F>
void backward_gaussian(const Cam<F>& cam, int deg, const float* mu_in, const float* s_in, const float* q_in,
                       const float* sh_in, const Rec<F>& rec, const G2<F>& g, F* dmu, F* ds, F* dq, F* dop, F* dsh) {
    const int K = (deg + 1) * (deg + 1);
    for (int j = 0; j < 3; ++j) dmu[j] = ds[j] = 0;
    for (int j = 0; j < 4; ++j) dq[j] = 0;
    *dop = 0;
    for (int k = 0; k < 3 * K; ++k) dsh[k] = 0;
    if (!rec.vis) return;
    const F mu[3] = {(F)mu_in[0], (F)mu_in[1], (F)mu_in[2]};
    const F s[3] = {(F)s_in[0], (F)s_in[1], (F)s_in[2]};
    const F n2 = ((F)q_in[0] * q_in[0] + (F)q_in[1] * q_in[1]) + (F)q_in[2] * q_in[2] + (F)q_in[3] * q_in[3];
    F qn[4] = {1, 0, 0, 0}, nrm = 0;
    if (n2 != F(0)) {
        nrm = std::sqrt(n2);
        for (int j = 0; j < 4; ++j) qn[j] = (F)q_in[j] / nrm;
    }
    const F w = qn[0], x = qn[1], y = qn[2], z = qn[3];
    F Rq[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                  {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                  {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    F M[3][3], Sg[3][3];
    for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) M[j][l] = Rq[j][l] * s[l];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) Sg[j][k] = M[j][0] * M[k][0] + M[j][1] * M[k][1] + M[j][2] * M[k][2];
    F p[3];
    for (int j = 0; j < 3; ++j) p[j] = cam.R[3 * j] * mu[0] + cam.R[3 * j + 1] * mu[1] + cam.R[3 * j + 2] * mu[2] + cam.t[j];
    const F pz = p[2], pz2 = pz * pz, pz3 = pz2 * pz;
    const F txtz = p[0] / pz, tytz = p[1] / pz;
    const F Lx = sclamp(txtz, -cam.limx, cam.limx), Ly = sclamp(tytz, -cam.limy, cam.limy);
    const F J00 = cam.fx / pz, J02 = -(cam.fx * Lx * pz) / pz2;
    const F J11 = cam.fy / pz, J12 = -(cam.fy * Ly * pz) / pz2;
    F T[2][3];
    for (int k = 0; k < 3; ++k) {
        T[0][k] = J00 * cam.R[k] + J02 * cam.R[6 + k];
        T[1][k] = J11 * cam.R[3 + k] + J12 * cam.R[6 + k];
    }
    F TS[2][3];
    for (int j = 0; j < 2; ++j)
        for (int k = 0; k < 3; ++k) TS[j][k] = T[j][0] * Sg[0][k] + T[j][1] * Sg[1][k] + T[j][2] * Sg[2][k];
    const F a = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2] + F(0.3);
    const F b = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
    const F c = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2] + F(0.3);
    const F D = a * c - b * b, D2 = D * D;

    // Colour: rgb = max(0, sum_k b_k(dir) sh_k + 1/2), dir = (mu - o) / |mu - o|.
    F dm[3] = {mu[0] - cam.o[0], mu[1] - cam.o[1], mu[2] - cam.o[2]};
    const F len = std::sqrt(dm[0] * dm[0] + dm[1] * dm[1] + dm[2] * dm[2]);
    const F dir[3] = {dm[0] / len, dm[1] / len, dm[2] / len};
    F bas[16], db[16][3];
    sh_basis<F>(deg, dir[0], dir[1], dir[2], bas);
    sh_basis_grad<F>(deg, dir[0], dir[1], dir[2], db);
    F gacc[3];
    for (int ch = 0; ch < 3; ++ch) gacc[ch] = rec.clamp_rgb[ch] ? F(0) : g.rgb[ch];
    F gdir[3] = {0, 0, 0};
    for (int k = 0; k < K; ++k)
        for (int ch = 0; ch < 3; ++ch) {
            dsh[3 * k + ch] = bas[k] * gacc[ch];
            for (int j = 0; j < 3; ++j) gdir[j] += gacc[ch] * (F)sh_in[3 * k + ch] * db[k][j];
        }
    const F dd = dir[0] * gdir[0] + dir[1] * gdir[1] + dir[2] * gdir[2];
    for (int j = 0; j < 3; ++j) dmu[j] += (gdir[j] - dir[j] * dd) / len;

    // Conic (c, -b, a) / D of the 2D covariance (a, b, c).
    const F ga = g.ca * (-c * c / D2) + g.cb * (b * c / D2) + g.cc * (-b * b / D2);
    const F gb = g.ca * (2 * b * c / D2) + g.cb * (-F(1) / D - 2 * b * b / D2) + g.cc * (2 * a * b / D2);
    const F gc = g.ca * (-b * b / D2) + g.cb * (a * b / D2) + g.cc * (-a * a / D2);
    const F G2m[2][2] = {{ga, gb / 2}, {gb / 2, gc}};
    // Sigma_2 = T Sigma T^T: dSigma = T^T G T, dT = 2 G T Sigma.
    F dSg[3][3], dT[2][3];
    for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) {
            F acc = 0;
            for (int u = 0; u < 2; ++u)
                for (int v = 0; v < 2; ++v) acc += T[u][j] * G2m[u][v] * T[v][k];
            dSg[j][k] = acc;
        }
    for (int u = 0; u < 2; ++u)
        for (int k = 0; k < 3; ++k) {
            F acc = 0;
            for (int v = 0; v < 2; ++v) acc += G2m[u][v] * TS[v][k];
            dT[u][k] = 2 * acc;
        }
    // T = J W with W the camera rotation.
    F dJ00 = 0, dJ02 = 0, dJ11 = 0, dJ12 = 0;
    for (int k = 0; k < 3; ++k) {
        dJ00 += dT[0][k] * cam.R[k];
        dJ02 += dT[0][k] * cam.R[6 + k];
        dJ11 += dT[1][k] * cam.R[3 + k];
        dJ12 += dT[1][k] * cam.R[6 + k];
    }
    F gp[3] = {0, 0, 0};
    gp[0] += g.mx * cam.fx / pz;
    gp[1] += g.my * cam.fy / pz;
    gp[2] += -g.mx * cam.fx * p[0] / pz2 - g.my * cam.fy * p[1] / pz2;
    gp[2] += dJ00 * (-cam.fx / pz2) + dJ11 * (-cam.fy / pz2);
    if (!rec.clamp_x) {
        gp[0] += dJ02 * (-cam.fx / pz2);
        gp[2] += dJ02 * (2 * cam.fx * p[0] / pz3);
    } else {
        gp[2] += dJ02 * (cam.fx * Lx / pz2);
    }
    if (!rec.clamp_y) {
        gp[1] += dJ12 * (-cam.fy / pz2);
        gp[2] += dJ12 * (2 * cam.fy * p[1] / pz3);
    } else {
        gp[2] += dJ12 * (cam.fy * Ly / pz2);
    }
    for (int j = 0; j < 3; ++j) dmu[j] += cam.R[j] * gp[0] + cam.R[3 + j] * gp[1] + cam.R[6 + j] * gp[2];

    // Sigma = M M^T with M = R_q diag(s).
    F dM[3][3];
    for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) dM[j][l] = 2 * (dSg[j][0] * M[0][l] + dSg[j][1] * M[1][l] + dSg[j][2] * M[2][l]);
    F dR[3][3];
    for (int l = 0; l < 3; ++l) {
        ds[l] = dM[0][l] * Rq[0][l] + dM[1][l] * Rq[1][l] + dM[2][l] * Rq[2][l];
        for (int j = 0; j < 3; ++j) dR[j][l] = dM[j][l] * s[l];
    }
    // Rotation from the unit quaternion, then the normalisation.
    F dqn[4];
    dqn[0] = 2 * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
    dqn[1] = 2 * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2 * x * dR[1][1] - w * dR[1][2] + z * dR[2][0] +
                  w * dR[2][1] - 2 * x * dR[2][2]);
    dqn[2] = 2 * (-2 * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] - w * dR[2][0] +
                  z * dR[2][1] - 2 * y * dR[2][2]);
    dqn[3] = 2 * (-2 * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2 * z * dR[1][1] + y * dR[1][2] +
                  x * dR[2][0] + y * dR[2][1]);
    if (n2 != F(0)) {
        const F qd = qn[0] * dqn[0] + qn[1] * dqn[1] + qn[2] * dqn[2] + qn[3] * dqn[3];
        for (int j = 0; j < 4; ++j) dq[j] = (dqn[j] - qn[j] * qd) / nrm;
    }
    *dop = g.op;
}

// FNV-1a hash of every discrete decision of a frame: visibility, rectangles,
// kept-tile counts, clamps, and each pixel's blend sequence.  Two parameter
// vectors with equal signatures lie on the same smooth piece of the image.
template <class F> u64 decision_signature(const Frame<F>& fr) {
    u64 h = 1469598103934665603ull;
    auto mix = [&](u64 v) {
        for (int b = 0; b < 8; ++b) {
            h ^= (v >> (8 * b)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    for (size_t i = 0; i < fr.recs.size(); ++i) {
        const Rec<F>& g = fr.recs[i];
        mix(g.vis);
        if (!g.vis) continue;
        for (int k = 0; k < 4; ++k) mix((u64)(int64_t)g.rect[k]);
        mix(fr.touched[i]);
        mix(g.clamp_rgb[0] | (g.clamp_rgb[1] << 1) | (g.clamp_rgb[2] << 2) | (g.clamp_x << 3) | (g.clamp_y << 4));
    }
    for (size_t p = 0; p < fr.pix.size(); ++p) {
        const Pixel<F>& px = fr.pix[p];
        mix(px.ids.size());
        for (size_t k = 0; k < px.ids.size(); ++k) {
            mix((u64)px.ids[k]);
            mix(px.alphas[k] >= F(0.99));
        }
    }
    return h;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI (ctypes).  All arrays are host arrays owned by the caller.
// ---------------------------------------------------------------------------
struct OFrameOut {
    // optional outputs (NULL to skip)
    float* xy;           // [N,2]
    float* conic_o;      // [N,4]
    float* sw;           // [N,12]  Sigma^-1 (6), w (3), rgb (3)
    float* zd;           // [N,2]   view depth, distance
    int32_t* rect;       // [N,4]
    int32_t* touched;    // [N]
    uint64_t* keys;      // [capacity]  (tile << 32) | depth key
    uint32_t* values;    // [capacity]
    int64_t capacity;
    int64_t n_entries;   // out
    uint32_t* ranges;    // [tiles,2]
    float* rgb;          // [3,H,W]
    float* depth;        // [H,W]
    int32_t* count;      // [H,W]
    float* T;            // [H,W]
    int32_t* blend_ids;  // [H,W,max_k], -1 padded
    int32_t max_k;
    float* delta;        // [H,W] per-pixel sort error
    int64_t stats[12];   // out: tail_in, mid_in, head_in, blends, max_tail, max_mid, max_head, min_tail_after_pop, entries
    const uint8_t* tile_mask;  // optional [tiles]: render only these tiles
    double ms[4];              // out: preprocess, duplicate, sort, render wall-clock times
    int32_t threads;           // out: OpenMP threads used
    uint64_t signature;        // out: hash of every discrete decision of the frame
};

template <class F, class OUT>
static int frame_impl(int n, int deg, const float* means, const float* scales, const float* rots,
                      const float* opac, const float* sh, const OCam* cam, const OCfg* cfg, OFrameOut* o,
                      OUT* rgb_out, OUT* depth_out, OUT* T_out) {
    if (n < 0 || deg < 0 || deg > 3 || cam->W <= 0 || cam->H <= 0) return -1;
    Frame<F> fr(*cam, *cfg);
    run_frame<F>(fr, n, deg, means, scales, rots, opac, sh, o->tile_mask);
    for (int i = 0; i < n; ++i) {
        const Rec<F>& g = fr.recs[i];
        if (o->xy) { o->xy[2 * i] = (float)g.x; o->xy[2 * i + 1] = (float)g.y; }
        if (o->conic_o) {
            o->conic_o[4 * i] = (float)g.ca; o->conic_o[4 * i + 1] = (float)g.cb;
            o->conic_o[4 * i + 2] = (float)g.cc; o->conic_o[4 * i + 3] = (float)g.op;
        }
        if (o->sw) {
            for (int k = 0; k < 6; ++k) o->sw[12 * i + k] = (float)g.s[k];
            for (int k = 0; k < 3; ++k) o->sw[12 * i + 6 + k] = (float)g.w[k];
            for (int k = 0; k < 3; ++k) o->sw[12 * i + 9 + k] = (float)g.rgb[k];
        }
        if (o->zd) { o->zd[2 * i] = (float)g.z; o->zd[2 * i + 1] = (float)g.dist; }
        if (o->rect) for (int k = 0; k < 4; ++k) o->rect[4 * i + k] = g.vis ? g.rect[k] : 0;
        if (o->touched) o->touched[i] = fr.touched[i];
    }
    o->n_entries = (int64_t)fr.entries.size();
    if (o->keys || o->values) {
        if ((int64_t)fr.entries.size() > o->capacity) return -2;
        for (size_t e = 0; e < fr.entries.size(); ++e) {
            const Entry& E = fr.entries[e];
            if (o->keys) o->keys[e] = ((uint64_t)E.tile << 32) | (E.dkey & 0xffffffffull);
            if (o->values) o->values[e] = E.id;
        }
    }
    if (o->ranges)
        for (size_t t = 0; t < fr.range_lo.size(); ++t) { o->ranges[2 * t] = fr.range_lo[t]; o->ranges[2 * t + 1] = fr.range_hi[t]; }
    const size_t P = (size_t)cam->W * cam->H;
    for (size_t p = 0; p < P; ++p) {
        const Pixel<F>& px = fr.pix[p];
        if (rgb_out) for (int ch = 0; ch < 3; ++ch) rgb_out[ch * P + p] = (OUT)(px.C[ch] + px.T * (F)cfg->bg[ch]);
        if (depth_out) depth_out[p] = (OUT)px.D;
        if (o->count) o->count[p] = px.n;
        if (T_out) T_out[p] = (OUT)px.T;
        if (o->blend_ids)
            for (int k = 0; k < o->max_k; ++k) o->blend_ids[p * o->max_k + k] = k < (int)px.ids.size() ? px.ids[k] : -1;
        if (o->delta) {
            // Sort error (Sec. 3.3): sum over consecutive blended pairs that are
            // out of order of their difference in t_opt.
            F d = 0;
            for (size_t k = 0; k + 1 < px.ts.size(); ++k)
                if (px.ts[k] > px.ts[k + 1]) d = d + (px.ts[k] - px.ts[k + 1]);
            o->delta[p] = (float)d;
        }
    }
    o->stats[0] = fr.stats.tail_in; o->stats[1] = fr.stats.mid_in; o->stats[2] = fr.stats.head_in;
    o->stats[3] = fr.stats.blends; o->stats[4] = fr.stats.max_tail; o->stats[5] = fr.stats.max_mid;
    o->stats[6] = fr.stats.max_head; o->stats[7] = fr.stats.min_tail_after_pop; o->stats[8] = (int64_t)fr.entries.size();
    for (int k = 0; k < 4; ++k) o->ms[k] = fr.ms[k];
    o->signature = decision_signature(fr);
#ifdef _OPENMP
    o->threads = omp_get_max_threads();
#else
    o->threads = 1;
#endif
    return 0;
}


// Forward and backward of one frame: dL_drgb [3,H,W]; gradients per Gaussian
// (means [N,3], scales [N,3], rots [N,4], opacities [N], sh [N,(d+1)^2,3]);
// also writes the forward image and the decision signature.
template <class F>
static int backward_impl(int n, int deg, const float* means, const float* scales, const float* rots,
                         const float* opac, const float* sh, const OCam* cam, const OCfg* cfg, const F* dL, F* dmeans,
                         F* dscales, F* drots, F* dopac, F* dsh, F* rgb_out, uint64_t* signature) {
    if (n < 0 || deg < 0 || deg > 3) return -1;
    Frame<F> fr(*cam, *cfg);
    run_frame<F>(fr, n, deg, means, scales, rots, opac, sh, nullptr);
    std::vector<G2<F>> g2(n);
    backward_blends(fr, dL, cfg->bg, g2);
    const int K = (deg + 1) * (deg + 1);
    for (int i = 0; i < n; ++i)
        backward_gaussian<F>(fr.cam, deg, means + 3 * i, scales + 3 * i, rots + 4 * i, sh + 3 * K * i, fr.recs[i], g2[i],
                             dmeans + 3 * i, dscales + 3 * i, drots + 4 * i, dopac + i, dsh + 3 * K * i);
    const size_t P = (size_t)cam->W * cam->H;
    if (rgb_out)
        for (size_t p = 0; p < P; ++p)
            for (int ch = 0; ch < 3; ++ch) rgb_out[ch * P + p] = fr.pix[p].C[ch] + fr.pix[p].T * (F)cfg->bg[ch];
    if (signature) *signature = decision_signature(fr);
    return 0;
}

// Chain rule alone: parameter gradients of every Gaussian from given 2D
// gradients g2_in [N,9] (same component order as oracle_grad2d_f64), in
// float64 or float32 arithmetic.
template <class F>
static int chain_impl(int n, int deg, const float* means, const float* scales, const float* rots, const float* opac,
                      const float* sh, const OCam* cam, const OCfg* cfg, const double* g2_in, double* dmeans,
                      double* dscales, double* drots, double* dopac, double* dsh) {
    if (n < 0 || deg < 0 || deg > 3) return -1;
    const Cam<F> C(*cam);
    const int K = (deg + 1) * (deg + 1);
    for (int i = 0; i < n; ++i) {
        Rec<F> r;
        preprocess_one<F>(C, cfg->mode, deg, means + 3 * i, scales + 3 * i, rots + 4 * i, opac[i], sh + 3 * K * i, r);
        G2<F> g;
        const double* q = g2_in + 9 * i;
        g.mx = (F)q[0]; g.my = (F)q[1]; g.ca = (F)q[2]; g.cb = (F)q[3]; g.cc = (F)q[4]; g.op = (F)q[5];
        g.rgb[0] = (F)q[6]; g.rgb[1] = (F)q[7]; g.rgb[2] = (F)q[8];
        F dm[3], ds[3], dq[4], dop, dsh_[48];
        backward_gaussian<F>(C, deg, means + 3 * i, scales + 3 * i, rots + 4 * i, sh + 3 * K * i, r, g, dm, ds, dq,
                             &dop, dsh_);
        for (int j = 0; j < 3; ++j) { dmeans[3 * i + j] = dm[j]; dscales[3 * i + j] = ds[j]; }
        for (int j = 0; j < 4; ++j) drots[4 * i + j] = dq[j];
        dopac[i] = dop;
        for (int k = 0; k < 3 * K; ++k) dsh[3 * K * i + k] = dsh_[k];
    }
    return 0;
}

extern "C" {

int oracle_frame_f32(int n, int deg, const float* means, const float* scales, const float* rots, const float* opac,
                     const float* sh, const OCam* cam, const OCfg* cfg, OFrameOut* out) {
    return frame_impl<float, float>(n, deg, means, scales, rots, opac, sh, cam, cfg, out, out->rgb, out->depth, out->T);
}

// Double instantiation: images in double.
int oracle_frame_f64(int n, int deg, const float* means, const float* scales, const float* rots, const float* opac,
                     const float* sh, const OCam* cam, const OCfg* cfg, OFrameOut* out, double* rgb, double* depth,
                     double* T) {
    return frame_impl<double, double>(n, deg, means, scales, rots, opac, sh, cam, cfg, out, rgb, depth, T);
}

int oracle_backward_f64(int n, int deg, const float* means, const float* scales, const float* rots, const float* opac,
                        const float* sh, const OCam* cam, const OCfg* cfg, const double* dL, double* dmeans,
                        double* dscales, double* drots, double* dopac, double* dsh, double* rgb, uint64_t* sig) {
    return backward_impl<double>(n, deg, means, scales, rots, opac, sh, cam, cfg, dL, dmeans, dscales, drots, dopac, dsh,
                                 rgb, sig);
}

int oracle_backward_f32(int n, int deg, const float* means, const float* scales, const float* rots, const float* opac,
                        const float* sh, const OCam* cam, const OCfg* cfg, const float* dL, float* dmeans,
                        float* dscales, float* drots, float* dopac, float* dsh, float* rgb, uint64_t* sig) {
    return backward_impl<float>(n, deg, means, scales, rots, opac, sh, cam, cfg, dL, dmeans, dscales, drots, dopac, dsh,
                                rgb, sig);
}

// 2D gradients of one frame, float64 terms over the float32 forward's blend
// sequences and decisions: per Gaussian the 9 components
// (mean x, mean y, conic a, b, c, opacity, r, g, b) of d(sum dL * rgb), the
// magnitude bound of each (see backward_blends) and the number of blends.
int oracle_grad2d_f64(int n, int deg, const float* means, const float* scales, const float* rots, const float* opac,
                      const float* sh, const OCam* cam, const OCfg* cfg, const double* dL, double* g2_out,
                      double* bound_out, int32_t* nterms_out) {
    if (n < 0 || deg < 0 || deg > 3) return -1;
    // the float32 forward's blends and decisions, terms in float64
    Frame<float> fr(*cam, *cfg);
    run_frame<float>(fr, n, deg, means, scales, rots, opac, sh, nullptr);
    std::vector<G2<double>> g2(n), bd(n);
    std::vector<int> nt(n, 0);
    backward_blends<double, float>(fr, dL, cfg->bg, g2, &bd, &nt);
    auto put = [](const G2<double>& g, double* o) {
        o[0] = g.mx; o[1] = g.my; o[2] = g.ca; o[3] = g.cb; o[4] = g.cc; o[5] = g.op;
        o[6] = g.rgb[0]; o[7] = g.rgb[1]; o[8] = g.rgb[2];
    };
    for (int i = 0; i < n; ++i) {
        put(g2[i], g2_out + 9 * i);
        put(bd[i], bound_out + 9 * i);
        nterms_out[i] = nt[i];
    }
    return 0;
}

int oracle_chain_f64(int n, int deg, const float* means, const float* scales, const float* rots, const float* opac,
                     const float* sh, const OCam* cam, const OCfg* cfg, const double* g2_in, double* dmeans,
                     double* dscales, double* drots, double* dopac, double* dsh) {
    return chain_impl<double>(n, deg, means, scales, rots, opac, sh, cam, cfg, g2_in, dmeans, dscales, drots, dopac,
                              dsh);
}

int oracle_chain_f32(int n, int deg, const float* means, const float* scales, const float* rots, const float* opac,
                     const float* sh, const OCam* cam, const OCfg* cfg, const double* g2_in, double* dmeans,
                     double* dscales, double* drots, double* dopac, double* dsh) {
    return chain_impl<float>(n, deg, means, scales, rots, opac, sh, cam, cfg, g2_in, dmeans, dscales, drots, dopac,
                             dsh);
}

// ----- element functions exposed for the pins -----
float oracle_exp_f32(float x) { return expE(x); }
float oracle_ln_f32(float x) { return lnE(x); }

void oracle_sh_basis(int deg, double x, double y, double z, double* b) { sh_basis<double>(deg, x, y, z, b); }
void oracle_sh_basis_f32(int deg, float x, float y, float z, float* b) { sh_basis<float>(deg, x, y, z, b); }

// Algorithm 1 on one box for a 2D Gaussian given by mean and conic.
void oracle_alg1(double mx, double my, double ca, double cb, double cc, double x0, double x1, double y0, double y1,
                 double* out) {
    Rec<double> g;
    std::memset(&g, 0, sizeof(g));
    g.x = mx; g.y = my; g.ca = ca; g.cb = cb; g.cc = cc;
    alg1_max_point(g, x0, x1, y0, y1, out[0], out[1]);
}

// t_opt of one Gaussian (mean, scale, quaternion) for a camera centre and a
// unit direction, through the same preprocessing as the frame (double).
int oracle_topt_f64(const float* mu, const float* s, const float* q, const OCam* cam, const double* d, double* t,
                    double* sinv) {
    Cam<double> C(*cam);
    Rec<double> g;
    float sh[48] = {0};
    float op = 1.0f;
    preprocess_one<double>(C, MODE_HIER, 0, mu, s, q, op, sh, g);
    if (!g.vis) return -1;
    for (int k = 0; k < 6; ++k) sinv[k] = g.s[k];
    *t = topt(g, d);
    return 0;
}

// Unit ray of the camera through image point (u, v).
void oracle_ray_f64(const OCam* cam, double u, double v, double* d) { Cam<double>(*cam).ray(u, v, d); }
void oracle_ray_f32(const OCam* cam, float u, float v, float* d) { Cam<float>(*cam).ray(u, v, d); }

}  // extern "C"
