// Device-side building blocks shared by the DGSM kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "dgsm.h"

namespace dgsm {

constexpr int kWave = 64;
constexpr int kTile = 8;          // atlas tile side in texels (Sec. 3.2 buckets 8x8 tiles)
constexpr int kSuperTiles = 8;    // supertile side in tiles (a supertile holds <= 64 tiles)
constexpr int kMaxSuper = 256;    // supertiles per light: atlases up to 1024 x 1024 texels
constexpr int kMaskWords = kMaxSuper / 64;
constexpr int kPrepThreads = 256;
constexpr int kMaxAtlasSide = kTile * kSuperTiles * 16;   // 1024

// Tiling of one atlas: tiles of kTile x kTile texels, grouped into supertiles
// of up to kSuperTiles x kSuperTiles tiles (the coarse level of the two-level
// light-space binning).
struct Geom {
    int H, W, K, spacing, dtype;
    int param;       // dgsm_param
    int F;           // cube-map face side (H / 2); unused for the octahedral map
    float r0, r1;
    int TH, TW;      // tiles per column / row
    int SGH, SGW;    // supertile grid
    int STH, STW;    // tiles per supertile side
    int S;           // SGH * SGW
    int ntiles;
};

inline Geom make_geom(const dgsm_atlas_desc_t& d) {
    Geom g{};
    g.H = d.H; g.W = d.W; g.K = d.K; g.spacing = d.spacing; g.dtype = d.dtype;
    g.param = d.param;
    g.F = d.H / 2;
    g.r0 = d.r0; g.r1 = d.r1;
    g.TH = (d.H + kTile - 1) / kTile;
    g.TW = (d.W + kTile - 1) / kTile;
    g.STH = g.TH < kSuperTiles ? g.TH : kSuperTiles;
    g.STW = g.TW < kSuperTiles ? g.TW : kSuperTiles;
    g.SGH = (g.TH + g.STH - 1) / g.STH;
    g.SGW = (g.TW + g.STW - 1) / g.STW;
    g.S = g.SGH * g.SGW;
    g.ntiles = g.TH * g.TW;
    return g;
}

// Per-(light, Gaussian) record read by the tile build with wave-uniform
// (scalar) loads.  w_j = R e_j / s_j are the rows of the whitening W with
// A = W^T W; c_j = R e_j / (s_k s_l) are the rows of adj(A)^(1/2).  Padded to
// 128 bytes: with the record array 128-byte aligned, every record is exactly
// one L2 line (a 112-byte record straddles two lines seven times in eight).
struct __attribute__((aligned(16))) GRec {
    double mx, my, mz;   // o_L - mu, exact in FP64
    float w[9];
    float c[9];
    float bp;            // beta * sqrt(pi / 2)
    float r2;            // squared ray-to-mean distance beyond which no texel is active
    float lg;            // e0 = |adj(A)^(1/2) (m x d)|^2 / a at or beyond which no texel is active
    float r0;            // culling-cone numerator s_max sqrt(2 ln(U / eps)); -1: contributes nothing
    float pad[4];        // [0] the tile test's plane scale (per light and frame), [1] det(Sigma),
                         // [2] s_max / s_min, [3] 0
};
static_assert(sizeof(GRec) == 128, "GRec layout");

// Tile of tile-build block b (b < ntiles) in an XCD-aware order.  Workgroups
// are dealt to the eight XCDs round-robin, so blocks b = x, x + 8, ... share
// XCD x and its L2.  Runs of C = 8 consecutive tiles of the supertile-major
// order (all tiles of supertile 0, then supertile 1, ...) go to one XCD, and
// the XCDs take turns run by run: tiles in flight on one XCD are neighbours
// in the atlas and walk largely the same Gaussian records (L2 hits), while
// every XCD still gets tiles from all over the atlas (balanced work).  Blocks
// past the last whole group of 64 take the rest of the order in block order.
__host__ __device__ inline int xcd_tile(const Geom& g, int b) {
    const int n = g.ntiles, C = 8, full = n / (8 * C) * (8 * C);
    const int x = b % 8, r = b / 8;
    const int o = b < full ? ((r / C) * 8 + x) * C + r % C : b;   // position in supertile-major order
    const int sy = o / (g.STH * g.TW);                   // supertile row (full rows before it)
    const int o1 = o - sy * g.STH * g.TW;
    const int hy = g.TH - sy * g.STH < g.STH ? g.TH - sy * g.STH : g.STH;
    const int sx = o1 / (hy * g.STW);                    // supertile in that row (full ones before it)
    const int o2 = o1 - sx * hy * g.STW;
    const int ntx = g.TW - sx * g.STW < g.STW ? g.TW - sx * g.STW : g.STW;
    const int ly = o2 / ntx;
    return (sy * g.STH + ly) * g.TW + sx * g.STW + (o2 - ly * ntx);
}

// Octahedral decode of the texel centre (i, j) of an H x W atlas (Sec. 3.2).
__device__ inline void octa_texel_dir(int i, int j, int H, int W, double& x, double& y, double& z) {
    const double u = -1.0 + (2.0 * j + 1.0) / W;
    const double v = -1.0 + (2.0 * i + 1.0) / H;
    const double au = fabs(u), av = fabs(v);
    z = 1.0 - au - av;
    if (z < 0.0) {
        x = (u >= 0.0 ? 1.0 : -1.0) * (1.0 - av);
        y = (v >= 0.0 ? 1.0 : -1.0) * (1.0 - au);
    } else {
        x = u;
        y = v;
    }
    const double inv = 1.0 / sqrt(x * x + y * y + z * z);
    x *= inv; y *= inv; z *= inv;
}

// Cube-map decode (Ablation C) of the texel centre (i, j) of a 2F x 3F atlas:
// face f = 3 (i / F) + j / F, m = f / 2, d[m] = +-1, d[(m+1) % 3] = s,
// d[(m+2) % 3] = t with the face coordinates (s, t) of the texel centre.
__device__ inline void cube_texel_dir(int i, int j, int F, double& x, double& y, double& z) {
    const int bi = i / F, bj = j / F;
    const int f = 3 * bi + bj, m = f >> 1;
    const double s = -1.0 + (2.0 * (j - bj * F) + 1.0) / F;
    const double t = -1.0 + (2.0 * (i - bi * F) + 1.0) / F;
    const double inv = 1.0 / sqrt(1.0 + s * s + t * t);
    const double a = ((f & 1) ? -1.0 : 1.0) * inv, b = s * inv, c = t * inv;
    if (m == 0) { x = a; y = b; z = c; }
    else if (m == 1) { y = a; z = b; x = c; }
    else { z = a; x = b; y = c; }
}

// Unit direction of the texel centre (i, j) of either parameterisation.
__device__ inline void texel_dir(const Geom& g, int i, int j, double& x, double& y, double& z) {
    if (g.param == DGSM_PARAM_CUBEMAP)
        cube_texel_dir(i, j, g.F, x, y, z);
    else
        octa_texel_dir(i, j, g.H, g.W, x, y, z);
}

// Two cones (unit axis, sin of half the half-angle) can share a direction iff
// the angle between the axes is at most the sum of the half-angles.  Tested
// with the chord |a - b| = 2 sin(angle / 2), which stays accurate for small
// angles.  sh < 0 marks an empty cone.
// cos of half the half-angle of a cone, as the cone tests use it.
__device__ inline float cone_cos(float4 c) { return sqrtf(fmaxf(0.f, 1.f - c.w * c.w)); }

// The same test with both cosines given (cone_cos of each): the form for
// loops that test one cone against many whose cosines are stored.
__device__ inline bool cones_touch_c(float4 a, float ca, float4 b, float cb) {
    const float sh = a.w * cb + ca * b.w;        // sin((ta + tb) / 2)
    const float chh = ca * cb - a.w * b.w;       // cos((ta + tb) / 2)
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    return a.w >= 0.f && b.w >= 0.f && (chh <= 0.f || dx * dx + dy * dy + dz * dz <= 4.f * sh * sh);
}

__device__ inline bool cones_touch(float4 a, float4 b) {
    if (a.w < 0.f || b.w < 0.f) return false;
    const float ca = cone_cos(a);
    const float cb = cone_cos(b);
    const float sh = a.w * cb + ca * b.w;        // sin((ta + tb) / 2)
    const float chh = ca * cb - a.w * b.w;       // cos((ta + tb) / 2)
    if (chh <= 0.f) return true;                 // half-angles sum to >= pi
    const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
    return dx * dx + dy * dy + dz * dz <= 4.f * sh * sh;
}

// Shell radius t_k in FP64.
__device__ inline double shell_radius(int k, int K, int spacing, float r0, float r1) {
    if (spacing == DGSM_SHELLS_GEOMETRIC)
        return (double)r0 * pow((double)r1 / (double)r0, (double)k / (double)(K - 1));
    return ((double)k + 0.5) * (double)r1 / (double)K;
}

// Trilinear cell of a world point seen from a light (Sec. 3.3): the floor
// texel (i0, j0), the lower shell k0 and the fractions.  lr0, kscale: shell
// coordinate (log2 r - lr0) * kscale (geometric) or r * kscale - 1/2 (uniform).
// Clamped (NaN-safe) so that every texel and shell the lookup touches exists.
struct Cell {
    int i0, j0, k0;
    float fi, fj, fk;
};

// In-face cell of one cube-map axis: coordinate (c+1) F/2 - 1/2 clamped to
// [0, F-1], floor held at <= F-2 so that both neighbours lie in the face.
__device__ inline void cube_axis(float c, int F, int& c0, float& fc) {
    const float cf = fminf(fmaxf((c + 1.f) * (0.5f * (float)F) - 0.5f, 0.f), (float)(F - 1));
    c0 = min((int)cf, F - 2);
    fc = cf - (float)c0;
}

__device__ inline Cell query_cell(const Geom& g, float lr0, float kscale, const float* light, float x, float y,
                                  float z) {
    const float dx = x - light[0], dy = y - light[1], dz = z - light[2];
    const float l1 = fabsf(dx) + fabsf(dy) + fabsf(dz);
    Cell c;
    if (g.param == DGSM_PARAM_CUBEMAP) {
        const float ax = fabsf(dx), ay = fabsf(dy), az = fabsf(dz);
        float ma = dz, sa = dx, ta = dy;            // r = 0 looks along +z
        int m = 2;
        if (l1 > 0.f) {
            if (ax >= ay && ax >= az) { m = 0; ma = dx; sa = dy; ta = dz; }
            else if (ay >= az) { m = 1; ma = dy; sa = dz; ta = dx; }
        } else {
            ma = 1.f; sa = 0.f; ta = 0.f;
        }
        const int f = 2 * m + (ma < 0.f ? 1 : 0);
        const float im = 1.f / fabsf(ma);
        int a0, b0;
        cube_axis(sa * im, g.F, a0, c.fj);
        cube_axis(ta * im, g.F, b0, c.fi);
        c.i0 = (f / 3) * g.F + b0;
        c.j0 = (f % 3) * g.F + a0;
    } else {
        float qx = 0.f, qy = 0.f, qz = 1.f;
        if (l1 > 0.f) {
            const float il = 1.f / l1;
            qx = dx * il; qy = dy * il; qz = dz * il;
        }
        float u = qx, v = qy;
        if (qz < 0.f) {
            u = copysignf(1.f - fabsf(qy), qx >= 0.f ? 1.f : -1.f);
            v = copysignf(1.f - fabsf(qx), qy >= 0.f ? 1.f : -1.f);
        }
        const float jf = fminf(fmaxf((u + 1.f) * (0.5f * (float)g.W) - 0.5f, -0.5f), (float)g.W - 0.5f);
        const float fi_ = fminf(fmaxf((v + 1.f) * (0.5f * (float)g.H) - 0.5f, -0.5f), (float)g.H - 0.5f);
        const float j0f = floorf(jf), i0f = floorf(fi_);
        c.j0 = (int)j0f;
        c.i0 = (int)i0f;
        c.fj = jf - j0f;
        c.fi = fi_ - i0f;
    }
    const float r = sqrtf(dx * dx + dy * dy + dz * dz);
    float kf = g.spacing == DGSM_SHELLS_GEOMETRIC ? (__log2f(r) - lr0) * kscale : r * kscale - 0.5f;
    kf = fminf(fmaxf(kf, 0.f), (float)(g.K - 1));   // log2(0) = -inf clamps to shell 0
    c.k0 = min((int)kf, g.K - 2);
    c.fk = kf - (float)c.k0;
    return c;
}

// A texel one step outside the grid, through the octahedral mirror wrap:
// across the left/right edge (u = -1/+1) the map identifies (u, v) with
// (u, -v), across the top/bottom edge (v = -1/+1) (u, v) with (-u, v).
__device__ inline void wrap_texel(int& i, int& j, int H, int W) {
    if (j < 0) { j = 0; i = H - 1 - i; }
    else if (j >= W) { j = W - 1; i = H - 1 - i; }
    if (i < 0) { i = 0; j = W - 1 - j; }
    else if (i >= H) { i = H - 1; j = W - 1 - j; }
}

// Real orthonormal SH up to degree 3 without the Condon-Shortley phase,
// index k = l^2 + l + m; writes the first kp values.
__device__ inline void real_sh16(float x, float y, float z, int kp, float* Y) {
    Y[0] = 0.28209479177387814f;
    if (kp <= 1) return;
    const float c1 = 0.48860251190291992f;           // sqrt(3 / (4 pi))
    Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
    if (kp <= 4) return;
    const float c2a = 1.0925484305920792f;           // sqrt(15 / pi) / 2
    const float c2b = 0.31539156525252005f;          // sqrt(5 / pi) / 4
    const float c2c = 0.54627421529603959f;          // sqrt(15 / pi) / 4
    Y[4] = c2a * x * y; Y[5] = c2a * y * z; Y[6] = c2b * (3.f * z * z - 1.f);
    Y[7] = c2a * x * z; Y[8] = c2c * (x * x - y * y);
    if (kp <= 9) return;
    const float c3a = 0.59004358992664352f;          // sqrt(35 / (2 pi)) / 4
    const float c3b = 2.8906114426405538f;           // sqrt(105 / pi) / 2
    const float c3c = 0.45704579946446572f;          // sqrt(21 / (2 pi)) / 4
    const float c3d = 0.37317633259011540f;          // sqrt(7 / pi) / 4
    const float c3e = 1.4453057213202769f;           // sqrt(105 / pi) / 4
    Y[9] = c3a * y * (3.f * x * x - y * y);
    Y[10] = c3b * x * y * z;
    Y[11] = c3c * y * (5.f * z * z - 1.f);
    Y[12] = c3d * z * (5.f * z * z - 3.f);
    Y[13] = c3c * x * (5.f * z * z - 1.f);
    Y[14] = c3e * z * (x * x - y * y);
    Y[15] = c3a * x * (x * x - 3.f * y * y);
}

// Wave ballot of a lane predicate straight into a scalar mask (no detour
// through a 0/1 vector register and a second compare).
__device__ inline uint64_t ballot(bool b) { return __builtin_amdgcn_ballot_w64(b); }

extern "C" __device__ int __ockl_wfred_min_i32(int);
extern "C" __device__ unsigned int __ockl_wfred_or_u32(unsigned int);
extern "C" __device__ int __ockl_wfred_max_i32(int);

// Wave-wide integer min / max (DPP row reductions); call with all lanes active.
__device__ inline int wave_min(int v) { return __ockl_wfred_min_i32(v); }
__device__ inline int wave_max(int v) { return __ockl_wfred_max_i32(v); }
__device__ inline uint64_t wave_or(uint64_t v) {
    return ((uint64_t)__ockl_wfred_or_u32((unsigned int)(v >> 32)) << 32) | __ockl_wfred_or_u32((unsigned int)v);
}

// erf(x) by Abramowitz and Stegun, Handbook of Mathematical Functions, 7.1.28
// (after Hastings): for z = |x| >= 0, erf(z) = 1 - (1 + a1 z + ... + a6 z^6)^-16,
// absolute error below 3e-7.  One reciprocal and no exponential; the
// 16th power overflows to +inf for large z, which saturates to +-1 exactly.
__device__ inline float erf_as(float x) {
    const float z = fabsf(x);
    float p = 0.0000430638f;
    p = fmaf(z, p, 0.0002765672f);
    p = fmaf(z, p, 0.0001520143f);
    p = fmaf(z, p, 0.0092705272f);
    p = fmaf(z, p, 0.0422820123f);
    p = fmaf(z, p, 0.0705230784f);
    p = fmaf(z, p, 1.f);
    p *= p; p *= p; p *= p; p *= p;
    return copysignf(1.f - __builtin_amdgcn_rcpf(p), x);
}

__device__ inline int lane_id() { return __lane_id(); }

// Rank of this lane among the lanes set in a wave ballot.
__device__ inline int ballot_rank(uint64_t bal) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}

template <typename T> struct Store;
template <> struct Store<float> {
    __device__ static inline void put(float* p, float v) { *p = v; }
    __device__ static inline float get(const float* p) { return *p; }
};
template <> struct Store<__half> {
    __device__ static inline void put(__half* p, float v) { *p = __float2half_rn(v); }
    __device__ static inline float get(const __half* p) { return __half2float(*p); }
};

}  // namespace dgsm
