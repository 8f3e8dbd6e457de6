// Per-Gaussian stages of a frame: preprocessing (EWA splat, SH colour,
// clamped inverse covariance, opacity-aware bound, exact tile count),
// prefix sum of the counts, duplication into (tile, depth) keys, and tile
// ranges of the sorted keys.
#include "gsr_internal.h"

namespace gsr {

namespace {

// Real SH constants sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) with signs.
constexpr float kC0 = 0.28209479177387814f;
constexpr float kC1 = 0.4886025119029199f;
constexpr float kC2a = 1.0925484305920792f;   // xy, yz (neg), xz (neg)
constexpr float kC2b = 0.31539156525252005f;  // 2zz - xx - yy
constexpr float kC2c = 0.5462742152960396f;   // xx - yy
constexpr float kC3a = 0.5900435899266435f;
constexpr float kC3b = 2.8906114426405543f;
constexpr float kC3c = 0.4570457994644658f;
constexpr float kC3d = 0.37317633259011546f;
constexpr float kC3e = 1.4453057213202771f;

// Real SH basis b[0..(deg+1)^2) at the unit direction (x, y, z).
__device__ __forceinline__ void sh_basis(int deg, float x, float y, float z, float* bas) {
    bas[0] = kC0;
    if (deg >= 1) {
        bas[1] = (-kC1) * y;
        bas[2] = kC1 * z;
        bas[3] = (-kC1) * x;
    }
    if (deg >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, yz = y * z, xz = x * z;
        bas[4] = kC2a * xy;
        bas[5] = (-kC2a) * yz;
        bas[6] = kC2b * ((2.0f * zz - xx) - yy);
        bas[7] = (-kC2a) * xz;
        bas[8] = kC2c * (xx - yy);
        if (deg >= 3) {
            bas[9] = (-kC3a) * (y * (3.0f * xx - yy));
            bas[10] = kC3b * (xy * z);
            bas[11] = (-kC3c) * (y * ((4.0f * zz - xx) - yy));
            bas[12] = kC3d * (z * ((2.0f * zz - 3.0f * xx) - 3.0f * yy));
            bas[13] = (-kC3c) * (x * ((4.0f * zz - xx) - yy));
            bas[14] = kC3e * (z * (xx - yy));
            bas[15] = (-kC3a) * (x * (xx - 3.0f * yy));
        }
    }
}

// Gradient of sum_k w_k b_k(dir) with respect to dir, for weights w_k.
__device__ __forceinline__ float3 sh_basis_vjp(int deg, float x, float y, float z, const float* w) {
    float gx = 0.0f, gy = 0.0f, gz = 0.0f;
    if (deg >= 1) {
        gy += -kC1 * w[1];
        gz += kC1 * w[2];
        gx += -kC1 * w[3];
    }
    if (deg >= 2) {
        gx += kC2a * y * w[4];
        gy += kC2a * x * w[4];
        gy += -kC2a * z * w[5];
        gz += -kC2a * y * w[5];
        gx += kC2b * (-2.0f * x) * w[6];
        gy += kC2b * (-2.0f * y) * w[6];
        gz += kC2b * (4.0f * z) * w[6];
        gx += -kC2a * z * w[7];
        gz += -kC2a * x * w[7];
        gx += kC2c * (2.0f * x) * w[8];
        gy += kC2c * (-2.0f * y) * w[8];
    }
    if (deg >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        gx += -kC3a * (6.0f * x * y) * w[9];
        gy += -kC3a * (3.0f * xx - 3.0f * yy) * w[9];
        gx += kC3b * (y * z) * w[10];
        gy += kC3b * (x * z) * w[10];
        gz += kC3b * (x * y) * w[10];
        gx += -kC3c * (-2.0f * x * y) * w[11];
        gy += -kC3c * (4.0f * zz - xx - 3.0f * yy) * w[11];
        gz += -kC3c * (8.0f * y * z) * w[11];
        gx += kC3d * (-6.0f * x * z) * w[12];
        gy += kC3d * (-6.0f * y * z) * w[12];
        gz += kC3d * (6.0f * zz - 3.0f * xx - 3.0f * yy) * w[12];
        gx += -kC3c * (4.0f * zz - 3.0f * xx - yy) * w[13];
        gy += -kC3c * (-2.0f * x * y) * w[13];
        gz += -kC3c * (8.0f * x * z) * w[13];
        gx += kC3e * (2.0f * x * z) * w[14];
        gy += kC3e * (-2.0f * y * z) * w[14];
        gz += kC3e * (xx - yy) * w[14];
        gx += -kC3a * (3.0f * xx - 3.0f * yy) * w[15];
        gy += -kC3a * (-6.0f * x * y) * w[15];
    }
    return make_float3(gx, gy, gz);
}

__device__ __forceinline__ uint32_t wave_reduce_add(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

struct PreOut {
    float4* pk;
    float4* col;
    float2* zd;
    int4* rect;
};

// Per-Gaussian results of projection, kept until the colour is known.
struct ProjOut {
    float mx, my, ca, cb, cc, op;
    float Si[6];     // s00 s01 s02 s11 s12 s22
    float w[3];
    float pz, dist;
    float lno;       // ln(opacity / eps_O)
    float dir[3];    // unit direction camera -> mean (colour)
    int4 rc;
};

// Projection of Gaussian i (Sec. 2.1, App. A, App. B.2, App. B.4), all but
// the colour.  Returns false when the Gaussian is culled.  `tight`: the tile
// rectangle is cut down to the box of the alpha ellipse.
__device__ bool project_geom(const SceneArgs& sc, const DevCam& cam, int mode, bool tight, int i, ProjOut& po) {
    const float mu0 = sc.means[3 * i], mu1 = sc.means[3 * i + 1], mu2 = sc.means[3 * i + 2];
    const float s0 = sc.scales[3 * i], s1 = sc.scales[3 * i + 1], s2 = sc.scales[3 * i + 2];
    const float4 qv = reinterpret_cast<const float4*>(sc.rots)[i];
    const float op = sc.opac[i];
    bool ok = isfinite(mu0) && isfinite(mu1) && isfinite(mu2) && isfinite(s0) && isfinite(s1) && isfinite(s2) &&
              s0 > 0.0f && s1 > 0.0f && s2 > 0.0f && isfinite(qv.x) && isfinite(qv.y) && isfinite(qv.z) &&
              isfinite(qv.w) && isfinite(op);
    float Si[3][3];
    float w[3];
    float pz = 0.0f, dist = 0.0f;
    float ca = 0.0f, cb = 0.0f, cc = 0.0f, mx = 0.0f, my = 0.0f;
    float fx0 = 0.0f, fy0 = 0.0f, fx1 = 0.0f, fy1 = 0.0f;
    if (ok) {
        // Unit quaternion (w, x, y, z) -> rotation; zero -> identity.
        const float n2 = ((qv.x * qv.x + qv.y * qv.y) + qv.z * qv.z) + qv.w * qv.w;
        float qw = 1.0f, qx = 0.0f, qy = 0.0f, qz = 0.0f;
        if (n2 != 0.0f) {
            const float nrm = sqrtf(n2);
            qw = qv.x / nrm; qx = qv.y / nrm; qy = qv.z / nrm; qz = qv.w / nrm;
        }
        float Rq[3][3];
        Rq[0][0] = 1.0f - 2.0f * (qy * qy + qz * qz);
        Rq[0][1] = 2.0f * (qx * qy - qw * qz);
        Rq[0][2] = 2.0f * (qx * qz + qw * qy);
        Rq[1][0] = 2.0f * (qx * qy + qw * qz);
        Rq[1][1] = 1.0f - 2.0f * (qx * qx + qz * qz);
        Rq[1][2] = 2.0f * (qy * qz - qw * qx);
        Rq[2][0] = 2.0f * (qx * qz - qw * qy);
        Rq[2][1] = 2.0f * (qy * qz + qw * qx);
        Rq[2][2] = 1.0f - 2.0f * (qx * qx + qy * qy);

        // Sigma = R S^2 R^T and Sigma^-1 = R min(S^-1, 10^3)^2 R^T, upper
        // triangle formed and mirrored.
        const float sq[3] = {s0 * s0, s1 * s1, s2 * s2};
        float si2[3];
        const float sv[3] = {s0, s1, s2};
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            float si = 1.0f / sv[l];
            si = (si > 1000.0f) ? 1000.0f : si;
            si2[l] = si * si;
        }
        float Sg[3][3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int k = j; k < 3; ++k) {
                Sg[j][k] = ((Rq[j][0] * sq[0]) * Rq[k][0] + (Rq[j][1] * sq[1]) * Rq[k][1]) + (Rq[j][2] * sq[2]) * Rq[k][2];
                Sg[k][j] = Sg[j][k];
                Si[j][k] = ((Rq[j][0] * si2[0]) * Rq[k][0] + (Rq[j][1] * si2[1]) * Rq[k][1]) +
                           (Rq[j][2] * si2[2]) * Rq[k][2];
                Si[k][j] = Si[j][k];
            }
        const float dm[3] = {mu0 - cam.o[0], mu1 - cam.o[1], mu2 - cam.o[2]};
#pragma unroll
        for (int j = 0; j < 3; ++j) w[j] = (Si[j][0] * dm[0] + Si[j][1] * dm[1]) + Si[j][2] * dm[2];

        float p[3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
            p[j] = ((cam.R[3 * j] * mu0 + cam.R[3 * j + 1] * mu1) + cam.R[3 * j + 2] * mu2) + cam.t[j];
        ok = p[2] > cam.znear;
        if (ok) {
            // EWA: Jacobian of the perspective map with the 1.3x frustum clamp.
            const float txtz = p[0] / p[2], tytz = p[1] / p[2];
            const float xcl = sel_clamp(txtz, -cam.limx, cam.limx) * p[2];
            const float ycl = sel_clamp(tytz, -cam.limy, cam.limy) * p[2];
            const float pz2 = p[2] * p[2];
            const float J00 = cam.fx / p[2], J02 = -(cam.fx * xcl) / pz2;
            const float J11 = cam.fy / p[2], J12 = -(cam.fy * ycl) / pz2;
            float T[2][3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T[0][k] = J00 * cam.R[k] + J02 * cam.R[6 + k];
                T[1][k] = J11 * cam.R[3 + k] + J12 * cam.R[6 + k];
            }
            float U[2][3];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int k = 0; k < 3; ++k) U[j][k] = (T[j][0] * Sg[0][k] + T[j][1] * Sg[1][k]) + T[j][2] * Sg[2][k];
            const float a = ((U[0][0] * T[0][0] + U[0][1] * T[0][1]) + U[0][2] * T[0][2]) + 0.3f;
            const float b = (U[0][0] * T[1][0] + U[0][1] * T[1][1]) + U[0][2] * T[1][2];
            const float c = ((U[1][0] * T[1][0] + U[1][1] * T[1][1]) + U[1][2] * T[1][2]) + 0.3f;
            const float det = a * c - b * b;
            ok = det > 0.0f;
            if (ok) {
                ca = c / det;
                cb = (-b) / det;
                cc = a / det;
                mx = cam.fx * txtz + cam.cx;
                my = cam.fy * tytz + cam.cy;
                ok = op >= kEpsO;
            }
            float lno = 0.0f;
            if (ok) {
                lno = ln_atanh(op / kEpsO);
                po.lno = lno;
                const float mid = 0.5f * (a + c);
                const float disc = mid * mid - det;
                const float lam = mid + sqrtf(0.1f > disc ? 0.1f : disc);
                float rr;
                if (mode == kModeGlobal) {
                    rr = ceilf(3.0f * sqrtf(lam));
                } else {
                    // Opacity-aware bound t_O = sqrt(2 ln(o / eps_O)), widened by
                    // 1/256 and a pixel so that only exact culling decides.
                    const float tO = sqrtf(2.0f * lno);
                    const float r = tO * sqrtf(lam);
                    rr = r * 1.00390625f + 1.0f;
                }
                fx0 = ceilf(((mx - rr) - 15.0f) / 16.0f);
                fx1 = floorf((mx + rr) / 16.0f);
                fy0 = ceilf(((my - rr) - 15.0f) / 16.0f);
                fy1 = floorf((my + rr) / 16.0f);
                fx0 = sel_clamp(fx0, 0.0f, (float)cam.tiles_x);
                fy0 = sel_clamp(fy0, 0.0f, (float)cam.tiles_y);
                fx1 = sel_clamp(fx1, -1.0f, (float)(cam.tiles_x - 1));
                fy1 = sel_clamp(fy1, -1.0f, (float)(cam.tiles_y - 1));
                ok = (fx0 <= fx1) && (fy0 <= fy1);
                if (ok && tight) {
                    // The tiles tested are those of the alpha ellipse's box:
                    // q <= t_O^2 has half-widths t_O sqrt(Sigma_2 diagonal), at
                    // most the radius above; widened the same way (the box may
                    // be empty when the square is not).
                    const float tO = sqrtf(2.0f * lno);
                    const float rx = (tO * sqrtf(a)) * 1.00390625f + 1.0f;
                    const float ry = (tO * sqrtf(c)) * 1.00390625f + 1.0f;
                    fx0 = sel_max(fx0, ceilf(((mx - rx) - 15.0f) / 16.0f));
                    fx1 = sel_min(fx1, floorf((mx + rx) / 16.0f));
                    fy0 = sel_max(fy0, ceilf(((my - ry) - 15.0f) / 16.0f));
                    fy1 = sel_min(fy1, floorf((my + ry) / 16.0f));
                }
            }
            if (ok) {
                // Colour direction: camera -> mean (App. B.4).
                const float len = sqrtf((dm[0] * dm[0] + dm[1] * dm[1]) + dm[2] * dm[2]);
                po.dir[0] = dm[0] / len;
                po.dir[1] = dm[1] / len;
                po.dir[2] = dm[2] / len;
                dist = len;
                pz = p[2];
            }
        }
    }
    if (ok) {
        po.mx = mx; po.my = my; po.ca = ca; po.cb = cb; po.cc = cc; po.op = op;
        po.Si[0] = Si[0][0]; po.Si[1] = Si[0][1]; po.Si[2] = Si[0][2];
        po.Si[3] = Si[1][1]; po.Si[4] = Si[1][2]; po.Si[5] = Si[2][2];
        po.w[0] = w[0]; po.w[1] = w[1]; po.w[2] = w[2];
        po.pz = pz; po.dist = dist;
        po.rc = make_int4((int)fx0, (int)fy0, (int)fx1, (int)fy1);
    }
    return ok;
}

// Writes Gaussian i's records (a zero record when culled) and its splat.
__device__ void write_records(const PreOut& out, int i, bool ok, const ProjOut& po, const float* rgb, Splat& g,
                              int4& rc) {
    if (ok) {
        g.x = po.mx; g.y = po.my; g.ca = po.ca; g.cb = po.cb; g.cc = po.cc; g.op = po.op;
        g.lt = -po.lno;
        g.s00 = po.Si[0]; g.s01 = po.Si[1]; g.s02 = po.Si[2]; g.s11 = po.Si[3]; g.s12 = po.Si[4]; g.s22 = po.Si[5];
        g.w0 = po.w[0]; g.w1 = po.w[1]; g.w2 = po.w[2];
        rc = po.rc;
        out.pk[4 * i] = make_float4(po.mx, po.my, po.ca, po.cb);
        out.pk[4 * i + 1] = make_float4(po.cc, po.op, po.Si[0], po.Si[1]);
        out.pk[4 * i + 2] = make_float4(po.Si[2], po.Si[3], po.Si[4], po.Si[5]);
        out.pk[4 * i + 3] = make_float4(po.w[0], po.w[1], po.w[2], g.lt);
        out.col[i] = make_float4(rgb[0], rgb[1], rgb[2], po.dist);
        out.zd[i] = make_float2(po.pz, po.dist);
        out.rect[i] = rc;
    } else {
        const float4 z4 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        out.pk[4 * i] = z4;
        out.pk[4 * i + 1] = z4;
        out.pk[4 * i + 2] = z4;
        out.pk[4 * i + 3] = z4;
        out.col[i] = z4;
        out.zd[i] = make_float2(0.0f, 0.0f);
        out.rect[i] = make_int4(0, 0, 0, 0);
    }
}

__device__ __forceinline__ void tile_hull(const DevCam& cam, int tx, int ty, float& x0, float& x1, float& y0,
                                          float& y1) {
    x0 = (float)(tx * 16);
    x1 = (float)min(tx * 16 + 15, cam.W - 1);
    y0 = (float)(ty * 16);
    y1 = (float)min(ty * 16 + 15, cam.H - 1);
}

// Exact tile culling decision (Sec. 3.4) for tile (tx, ty).
__device__ __forceinline__ bool tile_kept(const Splat& g, const DevCam& cam, int tx, int ty) {
    float x0, x1, y0, y1;
    tile_hull(cam, tx, ty, x0, x1, y0, y1);
    return block_clears(g, x0, x1, y0, y1);
}

struct PreArgs {
    SceneArgs sc;
    DevCam cam;
    int mode, lb, flags;
    PreOut out;
    uint32_t* touched;
    uint64_t* kmask;
    // Grouped duplication (see launch_preprocess): per-workgroup counts of
    // kept tiles by the low kDupDigitBits bits of the (batch-global) tile id,
    // digit-major: dhist[d * dh_stride + wg_base + workgroup].
    uint32_t* dhist;
    uint32_t dh_stride, wg_base, tile_base;
};

__device__ __forceinline__ uint32_t dup_digit(const DevCam& cam, uint32_t tile_base, int tx, int ty) {
    return ((uint32_t)(ty * cam.tiles_x + tx) + tile_base) & (uint32_t)(kDupBins - 1);
}

// Column of the counts (and order of the buckets' runs) of workgroup w of a
// launch of nw workgroups: workgroups go to the 8 XCDs round robin, and the
// runs of workgroups of one XCD are made adjacent, so that a cache line on the
// boundary of two runs is written through one L2.  A bijection of [0, nw).
__device__ __forceinline__ uint32_t xcd_column(uint32_t w, uint32_t nw) {
    const uint32_t q = nw / 8u, r = nw % 8u, x = w % 8u;
    return x * q + (x < r ? x : r) + w / 8u;
}

// Work classes of a visible Gaussian in preprocessing and duplication
// (load balancing, Sec. 3.4), by the number of tiles of its rectangle:
//   masked    <= min(lb, 64): its (Gaussian, tile) pairs are spread over the
//             wavefront as one flat list; preprocessing records its kept
//             tiles as a 64-bit mask;
//   deferred  > lb: the whole wavefront works on it, one Gaussian at a time;
//   serial    the rest (64 < tiles <= lb), and every Gaussian when lb is
//             kNoLoadBalance: its own lane walks its rectangle.
__device__ __forceinline__ int lane_tile_limit(int lb) { return lb < 64 ? lb : 64; }
__device__ __forceinline__ bool class_masked(int area, int lb) { return lb < kNoLoadBalance && area <= lane_tile_limit(lb); }
__device__ __forceinline__ bool class_deferred(int area, int lb) { return lb < kNoLoadBalance && area > lb; }

// floor(k / w) for 0 <= k < 64 and 1 <= w <= 64 as (k * r16) >> 16 with
// r16 = ceil(2^16 / w): the product overshoots k / w by less than k / 2^16 <
// 1 / w, which never reaches the next integer.
__device__ __forceinline__ uint32_t small_recip(int w) { return (65536u + (uint32_t)w - 1u) / (uint32_t)w; }
__device__ __forceinline__ int small_div(int k, uint32_t r16) { return (int)(((uint32_t)k * r16) >> 16); }

// Index of the r-th lowest set bit of m (r < popcount(m)), by halving.
__device__ __forceinline__ int nth_set_bit(uint64_t m, uint32_t r) {
    uint32_t w = (uint32_t)m;
    int pos = 0;
    const uint32_t c32 = (uint32_t)__popc(w);
    if (r >= c32) {
        r -= c32;
        w = (uint32_t)(m >> 32);
        pos = 32;
    }
#pragma unroll
    for (int sh = 16; sh > 0; sh >>= 1) {
        const uint32_t c = (uint32_t)__popc(w & ((1u << sh) - 1u));
        if (r >= c) {
            r -= c;
            w >>= sh;
            pos += sh;
        }
    }
    return pos;
}

// Walks rectangle tiles k = lane, lane + 64, ... of a rectangle of width w
// without a division per step.
struct RectWalk {
    int cx, cy, sx, sy, w;
    __device__ __forceinline__ RectWalk(int lane, int w_) : w(w_) {
        cy = lane / w;
        cx = lane - cy * w;
        sy = 64 / w;
        sx = 64 - sy * w;
    }
    __device__ __forceinline__ void next() {
        cx += sx;
        cy += sy;
        if (cx >= w) {
            cx -= w;
            ++cy;
        }
    }
};

// Owner lookup for a flat list of the pairs of a wavefront's lanes: lane L
// owns positions [start_L, start_L + len_L), starts in lane order, every
// list at most 64 long (so at most 64 x 64 positions).  The owner of
// position p is the r-th non-empty list, r = (number of list starts <= p) -
// 1; the starts are kept as one 64-bit word per 64 positions, so a step of
// 64 positions needs one word and a popcount instead of a search.
struct FlatStarts {
    uint64_t bits[64];
    uint32_t lane_of[64];  // lane of the r-th non-empty list
};

__device__ __forceinline__ void flat_starts_init(FlatStarts& f, uint32_t start, uint32_t len) {
    const int lane = __lane_id();
    f.bits[lane] = 0ull;
    wave_lds_sync();
    const uint64_t ne = __ballot(len > 0);
    if (len > 0) {
        atomicOr((unsigned long long*)&f.bits[start >> 6], 1ull << (start & 63u));
        f.lane_of[__popcll(ne & lanemask_lt())] = (uint32_t)lane;
    }
    wave_lds_sync();
}

// Owner lane of position 64 j + lane (valid when that position exists);
// `seen` counts the starts of the steps before j and is advanced.
__device__ __forceinline__ int flat_owner(const FlatStarts& f, uint32_t j, uint32_t& seen) {
    const int lane = __lane_id();
    const uint64_t m = f.bits[j];
    const uint32_t upto = (uint32_t)__popcll(m & lanemask_lt()) + (uint32_t)((m >> lane) & 1ull);
    const uint32_t r = seen + upto;
    seen += (uint32_t)__popcll(m);
    return r > 0 ? (int)f.lane_of[(r - 1u) & 63u] : 0;
}

// SH coefficients of a workgroup's Gaussians are staged in LDS as whole rows
// (3 (deg + 1)^2 floats per Gaussian), kShRows Gaussians per round, so that
// every cache line of the coefficients is read once; rows are kShStride
// floats apart at most, with an odd stride so that lanes reading their own
// rows hit distinct banks.
constexpr int kShRows = 128;
constexpr int kShStride = 3 * 16 + 1;

// Per-wavefront staging for the flat kept-tile test (reuses the SH memory).
struct CountStage {
    float x[64], y[64], ca[64], cb[64], cc[64], op[64], lt[64];
    int rx0[64], ry0[64], rw[64];
    uint32_t pfx[64], r16[64];
    uint64_t mask[64];
    FlatStarts fs;
};
static_assert(4 * sizeof(CountStage) <= kShRows * kShStride * sizeof(float), "staging fits the SH area");

// One lane per Gaussian.  Gaussians whose rectangle holds more than
// lane_tile_limit(lb) tiles are counted in a second phase by the whole
// wavefront (Sec. 3.4, load balancing), one Gaussian at a time, tiles spread
// over the lanes; the others record which rectangle tiles they keep.
__global__ __launch_bounds__(256) void k_preprocess(PreArgs a) {
    __shared__ __align__(16) float s_sh[kShRows * kShStride];
    __shared__ uint32_t s_dh[kDupBins];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = __lane_id();
    const bool grouped = a.dhist != nullptr;
    for (int d = threadIdx.x; d < kDupBins; d += blockDim.x) s_dh[d] = 0u;
    ProjOut po;
    bool vis = false;
    if (i < a.sc.n) vis = project_geom(a.sc, a.cam, a.mode, a.mode == kModeHier && !(a.flags & kAblateTileCull), i, po);
    // Colour: SH along the direction camera -> mean (App. B.4), the
    // coefficients of the workgroup's Gaussians staged through LDS, kShRows
    // whole rows per round with coalesced loads; each channel sums its terms
    // in order k = 0, 1, ..., K - 1.
    const int K = (a.sc.deg + 1) * (a.sc.deg + 1), row = 3 * K, S = row | 1;
    const int b0 = blockIdx.x * blockDim.x;
    const int nloc = min((int)blockDim.x, a.sc.n - b0);
    float rgb[3] = {0.0f, 0.0f, 0.0f};
    float bas[16];
    if (vis) sh_basis(a.sc.deg, po.dir[0], po.dir[1], po.dir[2], bas);
    for (int r0 = 0; r0 < nloc; r0 += kShRows) {
        const int nr = min(kShRows, nloc - r0);
        {
            // (Gaussian, column) of element f, advanced by blockDim.x per step
            const float* src = a.sc.sh + (size_t)(b0 + r0) * row;
            int gidx = (int)threadIdx.x / row, col = (int)threadIdx.x - gidx * row;
            const int sq = (int)blockDim.x / row, sr = (int)blockDim.x - sq * row;
            for (int f = threadIdx.x; f < nr * row; f += blockDim.x) {
                s_sh[gidx * S + col] = src[f];
                gidx += sq;
                col += sr;
                if (col >= row) {
                    col -= row;
                    ++gidx;
                }
            }
        }
        __syncthreads();
        const int li = (int)threadIdx.x - r0;
        if (vis && li >= 0 && li < kShRows) {
            const float* shp = s_sh + li * S;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = bas[0] * shp[ch];
#pragma unroll
                for (int k = 1; k < 16; ++k)
                    if (k < K) acc = acc + bas[k] * shp[3 * k + ch];
                rgb[ch] = acc;
            }
        }
        __syncthreads();  // the rows are consumed before the next are staged
    }
    if (vis) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float acc = rgb[ch] + 0.5f;
            if (!isfinite(acc)) vis = false;
            rgb[ch] = acc < 0.0f ? 0.0f : acc;
        }
    }
    Splat g;
    int4 rc = make_int4(0, 0, -1, -1);
    if (i < a.sc.n) write_records(a.out, i, vis, po, rgb, g, rc);
    const int wdt = rc.z - rc.x + 1, hgt = rc.w - rc.y + 1;
    const int area = (vis && wdt > 0 && hgt > 0) ? wdt * hgt : 0;  // the ellipse box may be empty
    uint32_t cnt = 0;
    uint64_t mask = 0;
    const bool no_cull = (a.flags & kAblateTileCull) != 0;
    const bool masked = vis && class_masked(area, a.lb);
    const bool deferred = vis && a.mode == kModeHier && class_deferred(area, a.lb);
    const bool serial = vis && a.mode == kModeHier && !masked && !deferred;
    if (a.mode == kModeGlobal) {
        cnt = (uint32_t)area;
    } else {
        // Kept-tile test of all (Gaussian, rectangle tile) pairs of the masked
        // Gaussians of this wavefront as one flat list, one pair per lane per
        // step; kept tiles set bits of their Gaussian's mask in LDS.
        __syncthreads();  // the SH rows are no longer needed: reuse the memory
        CountStage& st = reinterpret_cast<CountStage*>(s_sh)[threadIdx.x >> 6];
        const uint32_t my = masked ? (uint32_t)area : 0u;
        uint32_t incl = my;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
            if (lane >= o) incl += y;
        }
        const uint32_t total = (uint32_t)__shfl((int)incl, 63);
        st.x[lane] = g.x; st.y[lane] = g.y; st.ca[lane] = g.ca; st.cb[lane] = g.cb; st.cc[lane] = g.cc;
        st.op[lane] = g.op; st.lt[lane] = g.lt;
        st.rx0[lane] = rc.x; st.ry0[lane] = rc.y; st.rw[lane] = wdt;
        st.r16[lane] = masked ? small_recip(wdt) : 0u;
        st.pfx[lane] = incl - my;
        st.mask[lane] = 0ull;
        flat_starts_init(st.fs, incl - my, my);
        uint32_t seen = 0;
        for (uint32_t j = 0; 64u * j < total; ++j) {
            const int lo = flat_owner(st.fs, j, seen);
            const uint32_t q = 64u * j + (uint32_t)lane;
            if (q >= total) continue;
            const int k = (int)(q - st.pfx[lo]);
            const int dy = small_div(k, st.r16[lo]);
            Splat h;
            h.x = st.x[lo]; h.y = st.y[lo]; h.ca = st.ca[lo]; h.cb = st.cb[lo]; h.cc = st.cc[lo]; h.op = st.op[lo];
            h.lt = st.lt[lo];
            const int tx = st.rx0[lo] + (k - dy * st.rw[lo]), ty = st.ry0[lo] + dy;
            if (no_cull || tile_kept(h, a.cam, tx, ty)) {
                atomicOr((unsigned long long*)&st.mask[lo], 1ull << k);
                if (grouped) atomicAdd(&s_dh[dup_digit(a.cam, a.tile_base, tx, ty)], 1u);
            }
        }
        wave_lds_sync();
        mask = st.mask[lane];
        cnt = (uint32_t)__popcll(mask);
        if (serial) {
            for (int k = 0; k < area; ++k) {
                const int tx = rc.x + k % wdt, ty = rc.y + k / wdt;
                if (no_cull || tile_kept(g, a.cam, tx, ty)) {
                    ++cnt;
                    if (grouped) atomicAdd(&s_dh[dup_digit(a.cam, a.tile_base, tx, ty)], 1u);
                }
            }
        }
    }
    uint64_t pend = __ballot(deferred);
    while (pend) {
        const int src_lane = __builtin_ctzll(pend);
        pend &= pend - 1;
        Splat h;
        h.x = lane_bcast(g.x, src_lane); h.y = lane_bcast(g.y, src_lane);
        h.ca = lane_bcast(g.ca, src_lane); h.cb = lane_bcast(g.cb, src_lane); h.cc = lane_bcast(g.cc, src_lane);
        h.op = lane_bcast(g.op, src_lane); h.lt = lane_bcast(g.lt, src_lane);
        const int rx0 = lane_bcast(rc.x, src_lane), ry0 = lane_bcast(rc.y, src_lane);
        const int rw = lane_bcast(wdt, src_lane), rarea = lane_bcast(area, src_lane);
        uint32_t c = 0;
        RectWalk wk(lane, rw);
        for (int k = lane; k < rarea; k += 64, wk.next()) {
            const int tx = rx0 + wk.cx, ty = ry0 + wk.cy;
            if (no_cull || tile_kept(h, a.cam, tx, ty)) {
                ++c;
                if (grouped) atomicAdd(&s_dh[dup_digit(a.cam, a.tile_base, tx, ty)], 1u);
            }
        }
        c = wave_reduce_add(c);
        if (lane == src_lane) cnt = c;
    }
    if (i < a.sc.n) {
        a.touched[i] = cnt;
        a.kmask[i] = mask;
    }
    if (grouped) {
        __syncthreads();
        const uint32_t col = a.wg_base + xcd_column(blockIdx.x, gridDim.x);
        for (int d = threadIdx.x; d < kDupBins; d += blockDim.x) a.dhist[(size_t)d * a.dh_stride + col] = s_dh[d];
    }
}

struct DupArgs {
    DevCam cam;
    int n, mode, lb, flags;
    const float4* pk;
    const float2* zd;
    const int4* rect;
    const uint32_t* touched;
    const uint64_t* kmask;
    const uint32_t* offsets;
    uint64_t* keys;
    uint32_t* vals;
    uint32_t capacity;
    int32_t* status;
    uint32_t tile_base, id_base;
    // Grouped duplication: the scanned per-workgroup digit counts of
    // preprocessing; entries go to their digit's bucket (in no particular
    // order inside it) instead of their Gaussian's offsets.
    const uint32_t* dhist;
    uint32_t dh_stride, wg_base;
};

__device__ __forceinline__ void put_entry(const DupArgs& a, uint32_t pos, uint32_t tile, uint32_t dbits, uint32_t id) {
    if (pos < a.capacity) {
        a.keys[pos] = ((uint64_t)(tile + a.tile_base) << 32) | (uint64_t)dbits;
        a.vals[pos] = id + a.id_base;
    } else {
        atomicOr(a.status, 1);
    }
}

// Key depth of a kept tile: the view depth z (global order), t_opt along the
// tile-centre ray (global order with naive per-tile depth, Sec. 3.3), the Gaussian's
// distance (ablation without tile-depth adjustment), or t_opt along the ray
// through the tile's maximum point x^ (Sec. 3.4).
__device__ __forceinline__ uint32_t key_depth(const DupArgs& a, const Splat& h, float z, int tx, int ty) {
    float x0, x1, y0, y1;
    if (a.mode == kModeGlobal && (a.flags & kTileCentreDepth)) {
        tile_hull(a.cam, tx, ty, x0, x1, y0, y1);
        return depth_bits(t_opt(h, cam_ray(a.cam, 0.5f * (x0 + x1), 0.5f * (y0 + y1))));
    }
    if (a.mode == kModeGlobal || (a.flags & kAblateTileDepth)) return depth_bits(z);
    tile_hull(a.cam, tx, ty, x0, x1, y0, y1);
    const float2 xh = box_max_point(h, x0, x1, y0, y1);
    return depth_bits(t_opt(h, cam_ray(a.cam, xh.x, xh.y)));
}

// Keep test and key depth of one rectangle tile (every tile is kept in the
// global order and in the ablation without tile-based culling).  With
// tile-depth adjustment the exact maximum point x^ decides the culling
// (o exp(power(x^)) against eps_O) and gives the key's ray.
__device__ __forceinline__ bool keep_and_depth(const DupArgs& a, const Splat& h, float z, int tx, int ty,
                                               uint32_t& dbits) {
    const bool keep_all = a.mode == kModeGlobal || (a.flags & kAblateTileCull);
    const bool flat_depth = a.mode == kModeGlobal || (a.flags & kAblateTileDepth);
    float x0, x1, y0, y1;
    if (flat_depth) {
        if (!keep_all) {
            tile_hull(a.cam, tx, ty, x0, x1, y0, y1);
            if (!block_clears(h, x0, x1, y0, y1)) return false;
        }
        if (a.mode == kModeGlobal && (a.flags & kTileCentreDepth)) {
            tile_hull(a.cam, tx, ty, x0, x1, y0, y1);
            dbits = depth_bits(t_opt(h, cam_ray(a.cam, 0.5f * (x0 + x1), 0.5f * (y0 + y1))));
        } else {
            dbits = depth_bits(z);
        }
        return true;
    }
    tile_hull(a.cam, tx, ty, x0, x1, y0, y1);
    const float2 xh = box_max_point(h, x0, x1, y0, y1);
    if (!keep_all && !clears_eps(h, splat_power(h, xh.x, xh.y))) return false;
    dbits = depth_bits(t_opt(h, cam_ray(a.cam, xh.x, xh.y)));
    return true;
}

// Per-wavefront staging of the 64 Gaussians whose kept tiles are enumerated.
struct DupStage {
    float x[64], y[64], ca[64], cb[64], cc[64], op[64];
    float s00[64], s01[64], s02[64], s11[64], s12[64], s22[64], w0[64], w1[64], w2[64];
    float z[64];
    int rx0[64], ry0[64], rw[64];
    uint32_t off[64], pfx[64], r16[64];
    uint64_t mask[64];
    FlatStarts fs;
};

// Duplication: every kept tile becomes a key (tile << 32 | depth bits) with
// depth = t_opt along the ray through the tile's maximum point (tile-depth
// adjustment, Sec. 3.4), or the view depth in the global mode.  A wavefront
// enumerates the kept (Gaussian, tile) pairs of its lane-handled Gaussians
// as one flat list, one pair per lane per step (balanced work; consecutive
// lanes write consecutive entries of a Gaussian); Gaussians with large
// rectangles go through the cooperative phase with ballot-compacted writes
// (App. B.4).
__global__ __launch_bounds__(256) void k_duplicate(DupArgs a) {
    __shared__ DupStage s_st[4];
    __shared__ uint32_t s_cur[kDupBins];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    DupStage& st = s_st[wave];
    const bool grouped = a.dhist != nullptr;
    if (grouped) {
        const uint32_t col = a.wg_base + xcd_column(blockIdx.x, gridDim.x);
        for (int d = threadIdx.x; d < kDupBins; d += blockDim.x) s_cur[d] = a.dhist[(size_t)d * a.dh_stride + col];
        __syncthreads();
    }
    // Slot of the next entry of tile (tx, ty) in its bucket.
    auto bucket_slot = [&](int tx, int ty) -> uint32_t {
        return atomicAdd(&s_cur[dup_digit(a.cam, a.tile_base, tx, ty)], 1u);
    };
    uint32_t cnt = 0;
    if (i < a.n) cnt = a.touched[i];
    Splat g;
    int4 rc = make_int4(0, 0, -1, -1);
    uint32_t off = 0;
    float zdepth = 0.0f;  // the depth used by keys without tile-depth adjustment
    if (cnt > 0) {
        g = load_packed(a.pk, (uint32_t)i);
        rc = a.rect[i];
        off = grouped ? 0u : a.offsets[i];
        const float2 zd = a.zd[i];
        zdepth = a.mode == kModeGlobal ? zd.x : zd.y;
    }
    const int wdt = rc.z - rc.x + 1, hgt = rc.w - rc.y + 1;
    const int area = cnt > 0 ? wdt * hgt : 0;
    const bool small = cnt > 0 && class_masked(area, a.lb);
    const bool deferred = cnt > 0 && class_deferred(area, a.lb);
    const bool serial = cnt > 0 && !small && !deferred;
    uint64_t mask = 0;
    if (small) mask = a.mode == kModeHier ? a.kmask[i] : (area >= 64 ? ~0ull : ((1ull << area) - 1ull));
    const uint32_t my = small ? cnt : 0u;
    uint32_t incl = my;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= o) incl += y;
    }
    const uint32_t total = (uint32_t)__shfl((int)incl, 63);
    st.x[lane] = g.x; st.y[lane] = g.y; st.ca[lane] = g.ca; st.cb[lane] = g.cb; st.cc[lane] = g.cc;
    st.op[lane] = g.op; st.s00[lane] = g.s00; st.s01[lane] = g.s01; st.s02[lane] = g.s02; st.s11[lane] = g.s11;
    st.s12[lane] = g.s12; st.s22[lane] = g.s22; st.w0[lane] = g.w0; st.w1[lane] = g.w1; st.w2[lane] = g.w2;
    st.z[lane] = zdepth;
    st.rx0[lane] = rc.x; st.ry0[lane] = rc.y; st.rw[lane] = wdt;
    st.mask[lane] = mask; st.off[lane] = off; st.pfx[lane] = incl - my;
    st.r16[lane] = small ? small_recip(wdt) : 0u;
    flat_starts_init(st.fs, incl - my, my);  // also orders the stores above
    const uint32_t id_wave = (uint32_t)(blockIdx.x * blockDim.x + wave * 64);
    uint32_t seen = 0;
    for (uint32_t j = 0; 64u * j < total; ++j) {
        const int lo = flat_owner(st.fs, j, seen);
        const uint32_t q = 64u * j + (uint32_t)lane;
        if (q >= total) continue;
        const uint32_t r = q - st.pfx[lo];
        const int k = nth_set_bit(st.mask[lo], r);  // the r-th kept tile
        const int dy = small_div(k, st.r16[lo]);
        const int tx = st.rx0[lo] + (k - dy * st.rw[lo]), ty = st.ry0[lo] + dy;
        Splat h;
        h.x = st.x[lo]; h.y = st.y[lo]; h.ca = st.ca[lo]; h.cb = st.cb[lo]; h.cc = st.cc[lo]; h.op = st.op[lo];
        h.s00 = st.s00[lo]; h.s01 = st.s01[lo]; h.s02 = st.s02[lo]; h.s11 = st.s11[lo]; h.s12 = st.s12[lo];
        h.s22 = st.s22[lo]; h.w0 = st.w0[lo]; h.w1 = st.w1[lo]; h.w2 = st.w2[lo];
        h.lt = __int_as_float(0x7fc00000);  // no culling here: the mask decided
        const uint32_t dbits = key_depth(a, h, st.z[lo], tx, ty);
        put_entry(a, grouped ? bucket_slot(tx, ty) : st.off[lo] + r, (uint32_t)(ty * a.cam.tiles_x + tx), dbits,
                  id_wave + (uint32_t)lo);
    }
    if (serial) {
        // No load balancing for this Gaussian: its lane walks its rectangle.
        uint32_t r = 0;
        for (int k = 0; k < area; ++k) {
            const int tx = rc.x + k % wdt, ty = rc.y + k / wdt;
            uint32_t dbits;
            if (keep_and_depth(a, g, zdepth, tx, ty, dbits)) {
                put_entry(a, grouped ? bucket_slot(tx, ty) : off + r, (uint32_t)(ty * a.cam.tiles_x + tx), dbits,
                          (uint32_t)i);
                ++r;
            }
        }
    }
    uint64_t pend = __ballot(deferred);
    while (pend) {
        const int src = __builtin_ctzll(pend);
        pend &= pend - 1;
        Splat h;
        h.x = lane_bcast(g.x, src); h.y = lane_bcast(g.y, src);
        h.ca = lane_bcast(g.ca, src); h.cb = lane_bcast(g.cb, src); h.cc = lane_bcast(g.cc, src);
        h.op = lane_bcast(g.op, src);
        h.s00 = lane_bcast(g.s00, src); h.s01 = lane_bcast(g.s01, src); h.s02 = lane_bcast(g.s02, src);
        h.s11 = lane_bcast(g.s11, src); h.s12 = lane_bcast(g.s12, src); h.s22 = lane_bcast(g.s22, src);
        h.w0 = lane_bcast(g.w0, src); h.w1 = lane_bcast(g.w1, src); h.w2 = lane_bcast(g.w2, src);
        h.lt = lane_bcast(g.lt, src);
        const float hz = lane_bcast(zdepth, src);
        const int rx0 = lane_bcast(rc.x, src), ry0 = lane_bcast(rc.y, src);
        const int rw = lane_bcast(wdt, src), rarea = lane_bcast(area, src);
        uint32_t base = lane_bcast(off, src);
        const uint32_t id = lane_bcast((uint32_t)i, src);
        RectWalk wk(lane, rw);
        for (int k0 = 0; k0 < rarea; k0 += 64, wk.next()) {
            const int k = k0 + lane;
            bool keep = false;
            uint32_t dbits = 0;
            const int tx = rx0 + wk.cx, ty = ry0 + wk.cy;
            if (k < rarea) keep = keep_and_depth(a, h, hz, tx, ty, dbits);
            const uint64_t m = __ballot(keep);
            if (keep) put_entry(a, grouped ? bucket_slot(tx, ty) : base + (uint32_t)__popcll(m & lanemask_lt()),
                                (uint32_t)(ty * a.cam.tiles_x + tx),
                                dbits, id);
            base += (uint32_t)__popcll(m);
        }
    }
}

// ----- exclusive scan -----
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds_waves, uint32_t& total) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds_waves[wave] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) {
        const uint32_t s = lds_waves[w];
        if (w < wave) before += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + x - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* __restrict__ in, size_t n,
                                                              uint32_t* __restrict__ partial) {
    __shared__ uint32_t lw[kScanThreads / 64];
    const size_t base = (size_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        const size_t j = base + (size_t)r * kScanThreads + threadIdx.x;
        if (j < n) s += in[j];
    }
    uint32_t tot;
    block_exclusive_scan(s, lw, tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One block: exclusive scan of the partial sums (64-bit running total).
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* partial, size_t np, uint32_t* total_out,
                                                        uint32_t clamp, int32_t* status, uint32_t* raw_total) {
    __shared__ uint32_t lw[16];
    unsigned long long carry = 0;
    for (size_t b0 = 0; b0 < np; b0 += blockDim.x) {
        const size_t j = b0 + threadIdx.x;
        const uint32_t v = j < np ? partial[j] : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, lw, tot);
        if (j < np) partial[j] = (uint32_t)(carry + ex);
        carry += tot;
    }
    if (threadIdx.x == 0 && raw_total) *raw_total = carry > 0xffffffffull ? 0xffffffffu : (uint32_t)carry;
    if (threadIdx.x == 0 && total_out) {
        if (carry > (unsigned long long)clamp) {
            if (status) atomicOr(status, 1);
            *total_out = clamp;
        } else {
            *total_out = (uint32_t)carry;
        }
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const uint32_t* __restrict__ in, uint32_t* __restrict__ out,
                                                            size_t n, const uint32_t* __restrict__ partial) {
    __shared__ uint32_t lw[kScanThreads / 64];
    const size_t base = (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        v[r] = (base + r < n) ? in[base + r] : 0u;
        s += v[r];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, lw, tot) + partial[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        if (base + r < n) out[base + r] = run;
        run += v[r];
    }
}

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

struct BwdArgs {
    SceneArgs sc;
    DevCam cam;
    const float4* pk;
    const float* g2;
    float* dmeans;
    float* dscales;
    float* drots;
    float* dopac;
    float* dsh;
};

// Backward of preprocessing (Sec. 3.5 chain rule): from the accumulated
// gradients of the 2D mean, conic, opacity and colour to the mean, scales,
// quaternion, opacity and SH coefficients.  The forward quantities are
// recomputed; clamped colour channels and a clamped frustum coordinate pass
// no gradient through the clamped variable.
// SH coefficients of a wavefront's 64 Gaussians staged in LDS, kBwdShStride
// floats per Gaussian (odd, so that the lanes' rows fall in distinct banks):
// the coefficients are read and their gradients written in whole contiguous
// runs rather than one 4-byte word per lane every 3 (d + 1)^2 words.
constexpr int kBwdShStride = 49;  // >= 48 = 3 (3 + 1)^2

// Copies the S coefficients of `cnt` consecutive Gaussians between global
// memory (g, contiguous) and the staging (rows of kBwdShStride floats).
__device__ __forceinline__ void sh_stage_in(float* stage, const float* __restrict__ g, int cnt, int S) {
    if (cnt <= 0 || S <= 0) return;
    const int lane = __lane_id(), total = cnt * S, dg = 64 / S, dk = 64 % S;
    int gi = lane / S, k = lane - gi * S;
    for (int j = lane; j < total; j += 64) {
        stage[gi * kBwdShStride + k] = g[j];
        gi += dg;
        k += dk;
        if (k >= S) {
            k -= S;
            ++gi;
        }
    }
}
__device__ __forceinline__ void sh_stage_out(const float* stage, float* __restrict__ g, int cnt, int S) {
    if (cnt <= 0 || S <= 0) return;
    const int lane = __lane_id(), total = cnt * S, dg = 64 / S, dk = 64 % S;
    int gi = lane / S, k = lane - gi * S;
    for (int j = lane; j < total; j += 64) {
        g[j] = stage[gi * kBwdShStride + k];
        gi += dg;
        k += dk;
        if (k >= S) {
            k -= S;
            ++gi;
        }
    }
}

// One Gaussian; sh holds its coefficients on entry and their gradients on
// return (both in the staging).
__device__ __forceinline__ void preprocess_bwd_one(const BwdArgs& a, int i, float* sh) {
    const int deg = a.sc.deg, K = (deg + 1) * (deg + 1);
    const bool vis = a.pk[4 * (size_t)i + 1].y > 0.0f;  // opacity; zero when culled
    if (!vis) {
        for (int k = 0; k < 3 * K; ++k) sh[k] = 0.0f;
        for (int j = 0; j < 3; ++j) a.dmeans[3 * i + j] = a.dscales[3 * i + j] = 0.0f;
        for (int j = 0; j < 4; ++j) a.drots[4 * i + j] = 0.0f;
        a.dopac[i] = 0.0f;
        return;
    }
    const DevCam& cam = a.cam;
    const float* gg = a.g2 + 9 * (size_t)i;
    const float gmx = gg[0], gmy = gg[1], gca = gg[2], gcb = gg[3], gcc = gg[4], gop = gg[5];
    const float grgb[3] = {gg[6], gg[7], gg[8]};
    const float mu[3] = {a.sc.means[3 * i], a.sc.means[3 * i + 1], a.sc.means[3 * i + 2]};
    const float s[3] = {a.sc.scales[3 * i], a.sc.scales[3 * i + 1], a.sc.scales[3 * i + 2]};
    const float4 qv = reinterpret_cast<const float4*>(a.sc.rots)[i];
    const float n2 = ((qv.x * qv.x + qv.y * qv.y) + qv.z * qv.z) + qv.w * qv.w;
    float nrm = 0.0f, w = 1.0f, x = 0.0f, y = 0.0f, z = 0.0f;
    if (n2 != 0.0f) {
        nrm = sqrtf(n2);
        w = qv.x / nrm; x = qv.y / nrm; y = qv.z / nrm; z = qv.w / nrm;
    }
    const float Rq[3][3] = {{1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y)},
                            {2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x)},
                            {2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)}};
    float M[3][3], Sg[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int l = 0; l < 3; ++l) M[j][l] = Rq[j][l] * s[l];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k) Sg[j][k] = M[j][0] * M[k][0] + M[j][1] * M[k][1] + M[j][2] * M[k][2];
    float p[3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
        p[j] = ((cam.R[3 * j] * mu[0] + cam.R[3 * j + 1] * mu[1]) + cam.R[3 * j + 2] * mu[2]) + cam.t[j];
    const float pz = p[2], pz2 = pz * pz, pz3 = pz2 * pz;
    const float txtz = p[0] / pz, tytz = p[1] / pz;
    const bool cx_ = !(-cam.limx <= txtz && txtz <= cam.limx);
    const bool cy_ = !(-cam.limy <= tytz && tytz <= cam.limy);
    const float Lx = sel_clamp(txtz, -cam.limx, cam.limx), Ly = sel_clamp(tytz, -cam.limy, cam.limy);
    const float J00 = cam.fx / pz, J02 = -(cam.fx * Lx) / pz;
    const float J11 = cam.fy / pz, J12 = -(cam.fy * Ly) / pz;
    float T[2][3], TS[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T[0][k] = J00 * cam.R[k] + J02 * cam.R[6 + k];
        T[1][k] = J11 * cam.R[3 + k] + J12 * cam.R[6 + k];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k) TS[j][k] = T[j][0] * Sg[0][k] + T[j][1] * Sg[1][k] + T[j][2] * Sg[2][k];
    const float ea = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2] + 0.3f;
    const float eb = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
    const float ec = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2] + 0.3f;
    const float D = ea * ec - eb * eb, D2 = D * D;

    // Colour.  The clamp decision repeats the forward arithmetic exactly.
    const float dm[3] = {mu[0] - cam.o[0], mu[1] - cam.o[1], mu[2] - cam.o[2]};
    const float len = sqrtf((dm[0] * dm[0] + dm[1] * dm[1]) + dm[2] * dm[2]);
    const float dx_ = dm[0] / len, dy_ = dm[1] / len, dz_ = dm[2] / len;
    float bas[16];
    sh_basis(deg, dx_, dy_, dz_, bas);
    float* shp = sh;
    float gacc[3];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float acc = bas[0] * shp[ch];
        for (int k = 1; k < K; ++k) acc = acc + bas[k] * shp[3 * k + ch];
        acc = acc + 0.5f;
        gacc[ch] = acc < 0.0f ? 0.0f : grgb[ch];
    }
    float wk[16];
    for (int k = 0; k < K; ++k) {
        wk[k] = gacc[0] * shp[3 * k] + gacc[1] * shp[3 * k + 1] + gacc[2] * shp[3 * k + 2];
        shp[3 * k] = bas[k] * gacc[0];  // the coefficient's gradient replaces it
        shp[3 * k + 1] = bas[k] * gacc[1];
        shp[3 * k + 2] = bas[k] * gacc[2];
    }
    const float3 gd = sh_basis_vjp(deg, dx_, dy_, dz_, wk);
    const float dd = dx_ * gd.x + dy_ * gd.y + dz_ * gd.z;
    float dmu[3] = {(gd.x - dx_ * dd) / len, (gd.y - dy_ * dd) / len, (gd.z - dz_ * dd) / len};

    // Conic (c, -b, a) / D of the 2D covariance (a, b, c).
    const float ga = gca * (-ec * ec / D2) + gcb * (eb * ec / D2) + gcc * (-eb * eb / D2);
    const float gb = gca * (2.0f * eb * ec / D2) + gcb * (-1.0f / D - 2.0f * eb * eb / D2) + gcc * (2.0f * ea * eb / D2);
    const float gc = gca * (-eb * eb / D2) + gcb * (ea * eb / D2) + gcc * (-ea * ea / D2);
    const float G00 = ga, G01 = 0.5f * gb, G11 = gc;
    // Sigma_2 = T Sigma T^T: dSigma = T^T G T, dT = 2 G T Sigma.
    float dSg[3][3], dT[2][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k)
            dSg[j][k] = T[0][j] * (G00 * T[0][k] + G01 * T[1][k]) + T[1][j] * (G01 * T[0][k] + G11 * T[1][k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dT[0][k] = 2.0f * (G00 * TS[0][k] + G01 * TS[1][k]);
        dT[1][k] = 2.0f * (G01 * TS[0][k] + G11 * TS[1][k]);
    }
    float dJ00 = 0.0f, dJ02 = 0.0f, dJ11 = 0.0f, dJ12 = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dJ00 += dT[0][k] * cam.R[k];
        dJ02 += dT[0][k] * cam.R[6 + k];
        dJ11 += dT[1][k] * cam.R[3 + k];
        dJ12 += dT[1][k] * cam.R[6 + k];
    }
    float gp0 = gmx * cam.fx / pz, gp1 = gmy * cam.fy / pz;
    float gp2 = -gmx * cam.fx * p[0] / pz2 - gmy * cam.fy * p[1] / pz2;
    gp2 += dJ00 * (-cam.fx / pz2) + dJ11 * (-cam.fy / pz2);
    if (!cx_) {
        gp0 += dJ02 * (-cam.fx / pz2);
        gp2 += dJ02 * (2.0f * cam.fx * p[0] / pz3);
    } else {
        gp2 += dJ02 * (cam.fx * Lx / pz2);
    }
    if (!cy_) {
        gp1 += dJ12 * (-cam.fy / pz2);
        gp2 += dJ12 * (2.0f * cam.fy * p[1] / pz3);
    } else {
        gp2 += dJ12 * (cam.fy * Ly / pz2);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) dmu[j] += cam.R[j] * gp0 + cam.R[3 + j] * gp1 + cam.R[6 + j] * gp2;

    // Sigma = M M^T with M = R_q diag(s); then the unit quaternion.
    float dR[3][3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        float dsl = 0.0f;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const float dM = 2.0f * (dSg[j][0] * M[0][l] + dSg[j][1] * M[1][l] + dSg[j][2] * M[2][l]);
            dsl += dM * Rq[j][l];
            dR[j][l] = dM * s[l];
        }
        a.dscales[3 * i + l] = dsl;
    }
    float dq[4];
    dq[0] = 2.0f * (-z * dR[0][1] + y * dR[0][2] + z * dR[1][0] - x * dR[1][2] - y * dR[2][0] + x * dR[2][1]);
    dq[1] = 2.0f * (y * dR[0][1] + z * dR[0][2] + y * dR[1][0] - 2.0f * x * dR[1][1] - w * dR[1][2] + z * dR[2][0] +
                    w * dR[2][1] - 2.0f * x * dR[2][2]);
    dq[2] = 2.0f * (-2.0f * y * dR[0][0] + x * dR[0][1] + w * dR[0][2] + x * dR[1][0] + z * dR[1][2] - w * dR[2][0] +
                    z * dR[2][1] - 2.0f * y * dR[2][2]);
    dq[3] = 2.0f * (-2.0f * z * dR[0][0] - w * dR[0][1] + x * dR[0][2] + w * dR[1][0] - 2.0f * z * dR[1][1] +
                    y * dR[1][2] + x * dR[2][0] + y * dR[2][1]);
    if (n2 != 0.0f) {
        const float qd = w * dq[0] + x * dq[1] + y * dq[2] + z * dq[3];
        a.drots[4 * i] = (dq[0] - w * qd) / nrm;
        a.drots[4 * i + 1] = (dq[1] - x * qd) / nrm;
        a.drots[4 * i + 2] = (dq[2] - y * qd) / nrm;
        a.drots[4 * i + 3] = (dq[3] - z * qd) / nrm;
    } else {
        for (int j = 0; j < 4; ++j) a.drots[4 * i + j] = 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) a.dmeans[3 * i + j] = dmu[j];
    a.dopac[i] = gop;
}

__global__ __launch_bounds__(256) void k_preprocess_bwd(BwdArgs a) {
    __shared__ float s_sh[4][64 * kBwdShStride];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i0 = blockIdx.x * blockDim.x + wave * 64;
    const int S = 3 * (a.sc.deg + 1) * (a.sc.deg + 1);
    const int cnt = a.sc.n - i0 < 64 ? a.sc.n - i0 : 64;
    float* st = s_sh[wave];
    sh_stage_in(st, a.sc.sh + (size_t)(i0 > 0 ? i0 : 0) * S, cnt, S);
    wave_lds_sync();
    if (lane < cnt) preprocess_bwd_one(a, i0 + lane, st + lane * kBwdShStride);
    wave_lds_sync();
    sh_stage_out(st, a.dsh + (size_t)(i0 > 0 ? i0 : 0) * S, cnt, S);
}

__global__ void k_probe_math(const float* a, const float* b, int n, float* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = a[i], y = b[i];
    out[i] = x / y;
    out[n + i] = sqrtf(x);
    out[2 * n + i] = exp_cw(x);
    out[3 * n + i] = x >= 1.0f ? ln_atanh(x) : 0.0f;
    out[4 * n + i] = rintf(x);
    out[5 * n + i] = x * y + x;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)div_up(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_preprocess(const SceneArgs& sc, const DevCam& cam, int mode, int lb, int flags, const FrameBufs& b,
                             hipStream_t s, const DupGroups* groups) {
    if (sc.n == 0) return hipSuccess;
    PreArgs a;
    a.sc = sc;
    a.cam = cam;
    a.mode = mode;
    a.lb = lb;
    a.flags = flags;
    a.out = PreOut{b.pk, b.col, b.zd, b.rect};
    a.touched = b.touched;
    a.kmask = b.kmask;
    a.dhist = groups ? groups->hist : nullptr;
    a.dh_stride = groups ? groups->stride : 0u;
    a.wg_base = groups ? groups->wg_base : 0u;
    a.tile_base = groups ? groups->tile_base : 0u;
    hipLaunchKernelGGL(k_preprocess, dim3((unsigned)div_up(sc.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scan(const uint32_t* in, uint32_t* out, size_t n, uint32_t* partial, uint32_t* total,
                       uint32_t clamp, int32_t* status, hipStream_t s, uint32_t* raw_total) {
    const size_t nb = scan_partial_len(n);
    if (n == 0) {
        if (total) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, total, (size_t)1, 0u);
        if (raw_total) hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(1), 0, s, raw_total, (size_t)1, 0u);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partial);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partial, nb, total, clamp, status, raw_total);
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n, (const uint32_t*)partial);
    return hipGetLastError();
}

hipError_t launch_duplicate(int n, const DevCam& cam, int mode, int lb, int flags, const FrameBufs& b, int buf,
                            int32_t* status, hipStream_t s, uint32_t tile_base, uint32_t id_base,
                            const DupGroups* groups) {
    if (n == 0) return hipSuccess;
    DupArgs a;
    a.cam = cam;
    a.n = n;
    a.mode = mode;
    a.lb = lb;
    a.flags = flags;
    a.pk = b.pk;
    a.zd = b.zd;
    a.rect = b.rect;
    a.touched = b.touched;
    a.kmask = b.kmask;
    a.offsets = b.offsets;
    a.keys = b.keys[buf];
    a.vals = b.vals[buf];
    a.capacity = b.capacity;
    a.status = status;
    a.tile_base = tile_base;
    a.id_base = id_base;
    a.dhist = groups ? groups->hist : nullptr;
    a.dh_stride = groups ? groups->stride : 0u;
    a.wg_base = groups ? groups->wg_base : 0u;
    hipLaunchKernelGGL(k_duplicate, dim3((unsigned)div_up(n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}


hipError_t launch_preprocess_backward(const SceneArgs& sc, const DevCam& cam, const float4* pk, const float* grad2d,
                                      float* dmeans, float* dscales, float* drots, float* dopac, float* dsh,
                                      hipStream_t s) {
    if (sc.n == 0) return hipSuccess;
    BwdArgs a{sc, cam, pk, grad2d, dmeans, dscales, drots, dopac, dsh};
    hipLaunchKernelGGL(k_preprocess_bwd, dim3((unsigned)div_up(sc.n, 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_probe_math(const float* a, const float* b, int n, float* out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_probe_math, dim3((unsigned)div_up(n, 256)), dim3(256), 0, s, a, b, n, out);
    return hipGetLastError();
}

}  // namespace gsr
