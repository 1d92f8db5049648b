// Learned per-light transmittance field on gfx950 BF16 MFMA (FP32 accumulate).
//
// Network (one parameter set per light): phi(u, v, rho) -> 4 x (128, ReLU) ->
// z -> T = sigmoid(-z), i.e. log T = -softplus(z).  phi holds u, v, rho and
// sin/cos of f_i u, f_i v, f_i rho for 16 geometric frequencies
// f_i = pi (W/4)^(i/15) (W = atlas width), zero padded to 128.
// (u, v) is the octahedral code of the direction from the light and rho the
// radius coordinate of the atlas (Sec. 3.2), rescaled to [-1, 1].
//
// Kernels (rows = samples or query points):
//   sample_kernel   training / held-out samples from one light's atlas
//   grid_sample_kernel check samples at every texel centre x shell and
//                   uniformly inside every fallback region
//   fwd_kernel      features + 4 MFMA layers (weights in LDS) + output;
//                   modes: train (stashes activations for the backward) and
//                   check (flags regions where |T - T_atlas| > thr)
//   infer_kernel    inference at world points with the weights in registers
//   fallback_kernel trilinear atlas value for points in flagged regions
//   bwd_kernel      data-gradient chain through layers 3..1 (MFMA)
//   wgrad_kernel    per-chunk weight gradients dW_l = dZ_l^T X_l (MFMA)
//   reduce_kernel   fixed-order reduction of the partial gradients, optional
//                   Adam step, BF16 weight copies
// MFMA: v_mfma_f32_16x16x32_bf16.  A (16x32): lane l holds row l%16,
// k = 8(l/16)..+7; B (32x16): lane l holds column l%16, k = 8(l/16)..+7;
// D (16x16): lane l holds column l%16, rows 4(l/16)..+3.

#include <algorithm>

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"
#include "mlp.hpp"

namespace dgsm {
namespace mlp {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int kRows = 16;          // rows per wave
constexpr int kWaves = 4;
constexpr int kTileRows = kRows * kWaves;

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 16-byte chunk c (8 BF16) of a 256-byte row r, XOR-swizzled so that the 16
// lanes reading chunk c of 16 consecutive rows hit 16 different bank groups.
__device__ inline int swz(int r, int c) { return r * 16 + (c ^ (r & 15)); }

__device__ inline __bf16 to_bf16(float x) { return (__bf16)x; }   // round to nearest even

// Fourier features.  sin(f_i x) and cos(f_i x) with f_i = pi (W/4)^(i/15) are
// taken from the phase in turns, ph = c_i x with c_i = (W/4)^(i/15) / 2, formed
// in FP64 and reduced exactly to [-1/2, 1/2] (ph - rint(ph)), so the sine
// argument never carries the rounding of a large FP32 product (at W = 512 the
// phase reaches 64 turns).  Training, gradients and checks evaluate the sine of
// the reduced phase in FP64 (rounded once to FP32, then to BF16 where it enters
// the matrix units); inference evaluates it in FP32 (error about 1e-7).
__device__ inline double turns_per_unit(int i, int W) { return 0.5 * pow(0.25 * (double)W, (double)i / 15.0); }

// sin and cos of 2 pi ph for a phase ph in turns, in FP64: quarter turns
// y = 4 ph = q + f with q = rint(y) (both steps exact), th = f pi/2 in
// [-pi/4, pi/4], the Taylor series of sin to th^15 and of cos to th^16
// (truncation below 5e-17 on that interval), then the quadrant q mod 4.
__device__ inline void sincos_turns(double ph, double& s, double& c) {
    const double y = 4.0 * ph;
    const double q = rint(y);
    const double th = (y - q) * 1.5707963267948966;
    const double t2 = th * th;
    double ps = -1.0 / 1307674368000.0;              // -1/15!
    ps = fma(ps, t2, 1.0 / 6227020800.0);            // 1/13!
    ps = fma(ps, t2, -1.0 / 39916800.0);             // -1/11!
    ps = fma(ps, t2, 1.0 / 362880.0);                // 1/9!
    ps = fma(ps, t2, -1.0 / 5040.0);                 // -1/7!
    ps = fma(ps, t2, 1.0 / 120.0);                   // 1/5!
    ps = fma(ps, t2, -1.0 / 6.0);                    // -1/3!
    const double sn = fma(th * t2, ps, th);
    double pc = 1.0 / 20922789888000.0;              // 1/16!
    pc = fma(pc, t2, -1.0 / 87178291200.0);          // -1/14!
    pc = fma(pc, t2, 1.0 / 479001600.0);             // 1/12!
    pc = fma(pc, t2, -1.0 / 3628800.0);              // -1/10!
    pc = fma(pc, t2, 1.0 / 40320.0);                 // 1/8!
    pc = fma(pc, t2, -1.0 / 720.0);                  // -1/6!
    pc = fma(pc, t2, 1.0 / 24.0);                    // 1/4!
    pc = fma(pc, t2, -0.5);
    const double cs = fma(t2, pc, 1.0);
    const int quad = (int)(long long)q & 3;          // angle = quad pi/2 + th
    s = (quad & 1) ? cs : sn;
    c = (quad & 1) ? sn : cs;
    if (quad == 2 || quad == 3) s = -s;
    if (quad == 1 || quad == 2) c = -c;
}

__device__ inline float fourier_exact(double c, float x, bool cosine) {
    double s, co;
    sincos_turns(c * (double)x, s, co);
    return (float)(cosine ? co : s);
}

__device__ inline void fourier_pair(double c, double x, float& s, float& co) {
    double sd, cd;
    sincos_turns(c * x, sd, cd);
    s = (float)sd;
    co = (float)cd;
}

// Feature f (0..127) of a row; ct[i] = turns_per_unit(i, W).
__device__ inline float feature(int f, float u, float v, float rho, const double* ct) {
    if (f == 0) return u;
    if (f == 1) return v;
    if (f == 2) return rho;
    if (f >= kDin) return 0.f;
    const int q = f - 3, i = q / 6, rem = q - 6 * i;
    const float x = rem < 2 ? u : rem < 4 ? v : rho;
    return fourier_exact(ct[i], x, rem & 1);
}

// Octahedral code and radius coordinate of a point seen from a light.
__device__ inline void encode_point(float x, float y, float z, const float* o, const Geom& g, float& u,
                                    float& v, float& rho, float& r) {
    const float dx = x - o[0], dy = y - o[1], dz = z - o[2];
    const float l1 = fabsf(dx) + fabsf(dy) + fabsf(dz);
    float qx = 0.f, qy = 0.f, qz = 1.f;
    if (l1 > 0.f) {
        const float il = 1.f / l1;
        qx = dx * il; qy = dy * il; qz = dz * il;
    }
    u = qx; v = qy;
    if (qz < 0.f) {
        u = copysignf(1.f - fabsf(qy), qx >= 0.f ? 1.f : -1.f);
        v = copysignf(1.f - fabsf(qx), qy >= 0.f ? 1.f : -1.f);
    }
    r = sqrtf(dx * dx + dy * dy + dz * dz);
    if (g.spacing == DGSM_SHELLS_GEOMETRIC)
        rho = 2.f * (__log2f(r) - __log2f(g.r0)) / __log2f(g.r1 / g.r0) - 1.f;
    else
        rho = 2.f * r / g.r1 - 1.f;
    rho = fminf(fmaxf(rho, -1.f), 1.f);   // log2(0) = -inf clamps to -1
}

// The same code in FP64, for the inference features: the offset of the FP32
// point from the FP32 light is exact in FP64, and (u, v, rho) reach the phase
// of the Fourier features without an FP32 rounding.
__device__ inline void encode_point_f64(float x, float y, float z, const float* o, const Geom& g, double& u,
                                        double& v, double& rho) {
    const double dx = (double)x - (double)o[0], dy = (double)y - (double)o[1], dz = (double)z - (double)o[2];
    const double l1 = fabs(dx) + fabs(dy) + fabs(dz);
    double qx = 0.0, qy = 0.0, qz = 1.0;
    if (l1 > 0.0) {
        qx = dx / l1; qy = dy / l1; qz = dz / l1;
    }
    u = qx; v = qy;
    if (qz < 0.0) {
        u = copysign(1.0 - fabs(qy), qx >= 0.0 ? 1.0 : -1.0);
        v = copysign(1.0 - fabs(qx), qy >= 0.0 ? 1.0 : -1.0);
    }
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (g.spacing == DGSM_SHELLS_GEOMETRIC)
        rho = r > 0.0 ? 2.0 * log(r / (double)g.r0) / log((double)g.r1 / (double)g.r0) - 1.0 : -1.0;
    else
        rho = 2.0 * r / (double)g.r1 - 1.0;
    rho = fmin(fmax(rho, -1.0), 1.0);
}

__device__ inline int wrap_off(int i, int j, int H, int W) {
    if (j < 0) { j = 0; i = H - 1 - i; }
    else if (j >= W) { j = W - 1; i = H - 1 - i; }
    if (i < 0) { i = 0; j = W - 1 - j; }
    else if (i >= H) { i = H - 1; j = W - 1 - j; }
    return i * W + j;
}

// Trilinear atlas lookup at (u, v, rho), the same sampling rule as the query.
// Also returns the fallback region of the floor texel.
template <typename InT>
__device__ inline float atlas_at(const InT* tab, const Geom& g, float u, float v, float rho, int& region) {
    const float jf = fminf(fmaxf((u + 1.f) * (0.5f * (float)g.W) - 0.5f, -0.5f), (float)g.W - 0.5f);
    const float if_ = fminf(fmaxf((v + 1.f) * (0.5f * (float)g.H) - 0.5f, -0.5f), (float)g.H - 0.5f);
    float kf = g.spacing == DGSM_SHELLS_GEOMETRIC ? 0.5f * (rho + 1.f) * (float)(g.K - 1)
                                                  : 0.5f * (rho + 1.f) * (float)g.K - 0.5f;
    kf = fminf(fmaxf(kf, 0.f), (float)(g.K - 1));
    const float j0f = floorf(jf), i0f = floorf(if_);
    const int j0 = (int)j0f, i0 = (int)i0f;
    const float fj = jf - j0f, fi = if_ - i0f;
    const int k0 = min((int)kf, g.K - 2);
    const float fk = kf - (float)k0;
    const size_t plane = (size_t)g.H * g.W;
    const int o00 = wrap_off(i0, j0, g.H, g.W), o01 = wrap_off(i0, j0 + 1, g.H, g.W);
    const int o10 = wrap_off(i0 + 1, j0, g.H, g.W), o11 = wrap_off(i0 + 1, j0 + 1, g.H, g.W);
    const InT* s0 = tab + (size_t)k0 * plane;
    const InT* s1 = s0 + plane;
    const float a0 = (1.f - fj) * Store<InT>::get(s0 + o00) + fj * Store<InT>::get(s0 + o01);
    const float b0 = (1.f - fj) * Store<InT>::get(s0 + o10) + fj * Store<InT>::get(s0 + o11);
    const float a1 = (1.f - fj) * Store<InT>::get(s1 + o00) + fj * Store<InT>::get(s1 + o01);
    const float b1 = (1.f - fj) * Store<InT>::get(s1 + o10) + fj * Store<InT>::get(s1 + o11);
    const int ic = min(max(i0, 0), g.H - 1), jc = min(max(j0, 0), g.W - 1);
    region = (k0 / 8) * g.ntiles + (ic / kTile) * g.TW + jc / kTile;
    return (1.f - fk) * ((1.f - fi) * a0 + fi * b0) + fk * ((1.f - fi) * a1 + fi * b1);
}

// Fallback region of (u, v, rho) (the floor texel's 8x8 tile and 8-shell
// group, as atlas_at returns it), without reading the atlas.
__device__ inline int atlas_region(const Geom& g, float u, float v, float rho) {
    const float jf = fminf(fmaxf((u + 1.f) * (0.5f * (float)g.W) - 0.5f, -0.5f), (float)g.W - 0.5f);
    const float if_ = fminf(fmaxf((v + 1.f) * (0.5f * (float)g.H) - 0.5f, -0.5f), (float)g.H - 0.5f);
    float kf = g.spacing == DGSM_SHELLS_GEOMETRIC ? 0.5f * (rho + 1.f) * (float)(g.K - 1)
                                                  : 0.5f * (rho + 1.f) * (float)g.K - 0.5f;
    kf = fminf(fmaxf(kf, 0.f), (float)(g.K - 1));
    const int j0 = (int)floorf(jf), i0 = (int)floorf(if_);
    const int k0 = min((int)kf, g.K - 2);
    const int ic = min(max(i0, 0), g.H - 1), jc = min(max(j0, 0), g.W - 1);
    return (k0 / 8) * g.ntiles + (ic / kTile) * g.TW + jc / kTile;
}

__device__ inline uint32_t pcg_hash(uint32_t x) {
    // PCG-derived integer hash (Jarzynski and Olano, "Hash Functions for GPU
    // Rendering", JCGT 2020)
    const uint32_t s = x * 747796405u + 2891336453u;
    const uint32_t w = ((s >> ((s >> 28u) + 4u)) ^ s) * 277803737u;
    return (w >> 22u) ^ w;
}

__device__ inline float u01(uint32_t h) { return (float)(h >> 8) * (1.f / 16777216.f); }

// ---------------------------------------------------------------------------
// Samples: even rows at texel centres and shell radii (exact table values),
// odd rows uniform in (u, v, rho) with trilinear targets.
// ---------------------------------------------------------------------------
template <typename InT>
__global__ __launch_bounds__(256) void sample_kernel(const InT* __restrict__ tab, Geom g, int64_t n, uint32_t seed,
                                                     uint32_t step, float4* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const uint32_t base = pcg_hash(seed ^ pcg_hash(step * 0x9E3779B9u + 0x632BE5ABu)) ^ (uint32_t)(i * 3);
    const float r1 = u01(pcg_hash(base)), r2 = u01(pcg_hash(base + 1u)), r3 = u01(pcg_hash(base + 2u));
    float u, v, rho;
    if ((i & 1) == 0) {
        const int col = min((int)(r1 * g.W), g.W - 1), row = min((int)(r2 * g.H), g.H - 1);
        const int k = min((int)(r3 * g.K), g.K - 1);
        u = -1.f + (2.f * col + 1.f) / (float)g.W;
        v = -1.f + (2.f * row + 1.f) / (float)g.H;
        rho = g.spacing == DGSM_SHELLS_GEOMETRIC ? 2.f * (float)k / (float)(g.K - 1) - 1.f
                                                 : (2.f * (float)k + 1.f) / (float)g.K - 1.f;
    } else {
        u = 2.f * r1 - 1.f; v = 2.f * r2 - 1.f; rho = 2.f * r3 - 1.f;
    }
    int region;
    out[i] = make_float4(u, v, rho, atlas_at(tab, g, u, v, rho, region));
}

// Radius coordinate of shell k (its radius on the atlas's radial axis).
__device__ inline float shell_rho(const Geom& g, float kf) {
    return g.spacing == DGSM_SHELLS_GEOMETRIC ? 2.f * kf / (float)(g.K - 1) - 1.f
                                              : (2.f * kf + 1.f) / (float)g.K - 1.f;
}

// Check samples covering the whole atlas domain, rows [row_begin, row_begin + n)
// of a fixed enumeration: rows [0, H W K) are every texel centre at every shell
// radius with the stored value as target (row = (k H + i) W + j); the next
// regions * n_per rows are n_per points drawn uniformly in each fallback
// region's domain -- the continuous (row, column, shell) coordinates whose
// trilinear cell the region holds -- with trilinear targets.
template <typename InT>
__global__ __launch_bounds__(256) void grid_sample_kernel(const InT* __restrict__ tab, Geom g, int64_t row_begin,
                                                          int64_t n, int n_per, uint32_t seed,
                                                          float4* __restrict__ out) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= n) return;
    const int64_t row = row_begin + q;
    const int64_t plane = (int64_t)g.H * g.W, ngrid = plane * g.K;
    if (row < ngrid) {
        const int k = (int)(row / plane);
        const int64_t rem = row - (int64_t)k * plane;
        const int i = (int)(rem / g.W), j = (int)(rem - (int64_t)i * g.W);
        out[q] = make_float4(-1.f + (2.f * j + 1.f) / (float)g.W, -1.f + (2.f * i + 1.f) / (float)g.H,
                             shell_rho(g, (float)k), Store<InT>::get(tab + row));
        return;
    }
    const int64_t s = row - ngrid;
    const int64_t reg = s / n_per;
    const int kk = (int)(reg / g.ntiles), tt = (int)(reg - (int64_t)kk * g.ntiles);
    const int ti = tt / g.TW, tj = tt - ti * g.TW;
    const uint32_t base = pcg_hash(seed ^ pcg_hash((uint32_t)s ^ pcg_hash((uint32_t)(s >> 32) + 0x632BE5ABu)));
    const float r1 = u01(pcg_hash(base)), r2 = u01(pcg_hash(base + 1u)), r3 = u01(pcg_hash(base + 2u));
    // floor cells of the region: rows 8 ti .. 8 ti + 7 (the first tile also holds
    // i_f in [-1/2, 0), the last ends at H - 1/2), likewise columns; shells
    // 8 kk .. 8 kk + 7 with k_f up to K - 1 in the last group
    const float ilo = ti == 0 ? -0.5f : 8.f * ti, ihi = fminf(8.f * ti + 8.f, (float)g.H - 0.5f);
    const float jlo = tj == 0 ? -0.5f : 8.f * tj, jhi = fminf(8.f * tj + 8.f, (float)g.W - 0.5f);
    const float klo = 8.f * kk, khi = fminf(8.f * kk + 8.f, (float)(g.K - 1));
    const float fi = ilo + r1 * (ihi - ilo), fj = jlo + r2 * (jhi - jlo), fk = klo + r3 * fmaxf(khi - klo, 0.f);
    const float u = 2.f * (fj + 0.5f) / (float)g.W - 1.f, v = 2.f * (fi + 0.5f) / (float)g.H - 1.f;
    const float rho = shell_rho(g, fk);
    int region;
    out[q] = make_float4(u, v, rho, atlas_at(tab, g, u, v, rho, region));
}

// ---------------------------------------------------------------------------
// Forward
// ---------------------------------------------------------------------------
enum Mode { kTrain = 0, kCheck = 2 };   // forward of training samples / of check samples

struct FwdArgs {
    Geom g;
    const float* params;       // [L][kNParams]
    const __bf16* wb;          // [L][4][128][128]
    int64_t n;                 // rows
    const float4* uvrt;        // train / check: [n] (u, v, rho, target)
    const float* points;       // infer: [n][3]
    const float* lights;       // infer: [L][3]
    const void* atlas;         // infer fallback / check: [L][K][H][W]
    const unsigned char* mask; // infer: [L][regions] or null
    unsigned char* mask_out;   // check: [regions]
    float thresh;
    unsigned int* check_stats; // check: [0] flagged rows, [1] max |dT| (float bits)
    float* T;                  // infer: [L][n]
    // train stash
    __bf16* xt;                // [4][128][n]
    float* h4;                 // [n][128]
    float* gz;                 // [n]
    float* dw4p;               // [n/16][128]
    float* db4p;               // [n/16]
    float* lossp;              // [n/16]
    float inv_n;               // 1 / batch
    int atlas_f16;
    // check: global index of row 0, and rows below n_grid are texel-centre nodes
    int64_t row_offset;
    int64_t n_grid;
};

// Lanes 0..15 hold the inputs of the wave's 16 rows; any lane reads row r's
// input by a cross-lane shuffle.
__device__ inline float4 input_of(const float4& mine, int r) {
    return make_float4(__shfl(mine.x, r, kWave), __shfl(mine.y, r, kWave), __shfl(mine.z, r, kWave),
                       __shfl(mine.w, r, kWave));
}

// NWV waves per block share the weights in LDS (inference runs 8 waves, two
// per SIMD, so that one wave's LDS and MFMA latencies hide behind the
// other's; training keeps 4 because its stash stores need more registers).
template <int MODE, int NWV>
__global__ __launch_bounds__(kWave * NWV) void fwd_kernel(FwdArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    constexpr int kTile = kRows * NWV;
    bf16x8* wl = reinterpret_cast<bf16x8*>(smem);                        // [4][128 rows][16 chunks]
    bf16x8* act = wl + 4 * kH * 16;                                     // [NWV waves][16 rows][16 chunks]
    __shared__ double cturn[kNF];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    if (tid < kNF) cturn[tid] = turns_per_unit(tid, a.g.W);
    const int light = blockIdx.y;
    const float* P = a.params + (size_t)light * kNParams;
    const __bf16* Wg = a.wb + (size_t)light * 4 * kH * kH;
    // all four weight matrices into LDS, swizzled rows
    for (int q = tid; q < 4 * kH * 16; q += kWave * NWV) {
        const int row = q / 16, c = q % 16;                              // row = 128 l + j
        wl[(row / kH) * kH * 16 + swz(row % kH, c)] = *reinterpret_cast<const bf16x8*>(Wg + (size_t)row * kH + 8 * c);
    }
    __syncthreads();
    bf16x8* my = act + wave * kRows * 16;
    const int ntile = (int)((a.n + kTile - 1) / kTile);
    const int lr = lane % 16, lg = lane / 16;
    for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
        const int64_t row0 = (int64_t)t * kTile + wave * kRows;
        // inputs of the wave's 16 rows (u, v, rho, target) in lanes 0..15
        float4 in_mine = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lane < kRows) {
            const int64_t rr = row0 + lane;
            if (rr < a.n) {
                in_mine = a.uvrt[rr];
            }
        }
        __builtin_amdgcn_wave_barrier();
        {   // features: lane handles row lr, chunks lg + 4q
            const float4 in = input_of(in_mine, lr);
            for (int q = 0; q < 4; ++q) {
                const int c = lg + 4 * q;
                bf16x8 ch;
                for (int e = 0; e < 8; ++e) ch[e] = to_bf16(feature(8 * c + e, in.x, in.y, in.z, cturn));
                my[swz(lr, c)] = ch;
                if (MODE == kTrain && row0 + lr < a.n)
                    for (int e = 0; e < 8; ++e) a.xt[(size_t)(8 * c + e) * a.n + row0 + lr] = ch[e];
            }
        }
        __builtin_amdgcn_s_waitcnt(0xc07f);
        __builtin_amdgcn_wave_barrier();
        f32x4 acc[8];
        for (int l = 0; l < 4; ++l) {
            const float* bias = P + l * kLayer + kH * kH;
            for (int n = 0; n < 8; ++n) {
                const float b = bias[16 * n + lr];
                acc[n] = f32x4{b, b, b, b};
            }
            const bf16x8* W = wl + l * kH * 16;
            for (int kk = 0; kk < 4; ++kk) {
                const bf16x8 av = my[swz(lr, lg + 4 * kk)];
                for (int n = 0; n < 8; ++n) acc[n] = mfma(av, W[swz(16 * n + lr, lg + 4 * kk)], acc[n]);
            }
            for (int n = 0; n < 8; ++n)
                for (int r = 0; r < 4; ++r) acc[n][r] = fmaxf(acc[n][r], 0.f);
            if (l < 3) {
                __builtin_amdgcn_wave_barrier();
                __bf16* myh = reinterpret_cast<__bf16*>(my);
                for (int n = 0; n < 8; ++n) {
                    const int col = 16 * n + lr;
                    __bf16 hb[4];
                    for (int r = 0; r < 4; ++r) {
                        const int row = 4 * lg + r;
                        hb[r] = to_bf16(acc[n][r]);
                        myh[swz(row, col / 8) * 8 + (col % 8)] = hb[r];
                    }
                    if (MODE == kTrain && row0 + 4 * lg + 3 < a.n) {
                        __bf16* dst = a.xt + (size_t)(l + 1) * kH * a.n + (size_t)col * a.n + row0 + 4 * lg;
                        for (int r = 0; r < 4; ++r) dst[r] = hb[r];
                    }
                }
                __builtin_amdgcn_s_waitcnt(0xc07f);
                __builtin_amdgcn_wave_barrier();
            }
        }
        // output layer: z = w4 . h4 + b4 over the 128 columns of each row
        const float* w4 = P + kOffW4;
        float zp[4] = {0.f, 0.f, 0.f, 0.f};
        for (int n = 0; n < 8; ++n) {
            const float w = w4[16 * n + lr];
            for (int r = 0; r < 4; ++r) zp[r] += w * acc[n][r];
        }
        for (int r = 0; r < 4; ++r)
            for (int o = 1; o < 16; o <<= 1) zp[r] += __shfl_xor(zp[r], o, kWave);
        const float b4 = P[kOffB4];
        float T[4];
        for (int r = 0; r < 4; ++r) T[r] = 1.f / (1.f + __expf(zp[r] + b4));
        if (MODE == kTrain) {
            float gzr[4], lsum = 0.f;
            for (int r = 0; r < 4; ++r) {
                const int64_t row = row0 + 4 * lg + r;
                const float tgt = __shfl(in_mine.w, 4 * lg + r, kWave);
                const float d = T[r] - tgt;
                gzr[r] = row < a.n ? 2.f * d * a.inv_n * (-T[r] * (1.f - T[r])) : 0.f;
                lsum += row < a.n ? d * d * a.inv_n : 0.f;
                if (lr == 0 && row < a.n) a.gz[row] = gzr[r];
            }
            // h4 stash (FP32) and per-wave partials of dw4, db4, loss
            const int64_t wid = row0 / kRows;
            for (int n = 0; n < 8; ++n) {
                const int col = 16 * n + lr;
                float s = 0.f;
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = row0 + 4 * lg + r;
                    if (row < a.n) a.h4[(size_t)row * kH + col] = acc[n][r];
                    s += gzr[r] * acc[n][r];
                }
                s += __shfl_xor(s, 16, kWave);
                s += __shfl_xor(s, 32, kWave);
                if (lg == 0) a.dw4p[(size_t)wid * kH + col] = s;
            }
            float gs = gzr[0] + gzr[1] + gzr[2] + gzr[3];
            gs += __shfl_xor(gs, 16, kWave);
            gs += __shfl_xor(gs, 32, kWave);
            lsum += __shfl_xor(lsum, 16, kWave);
            lsum += __shfl_xor(lsum, 32, kWave);
            if (lane == 0) {
                a.db4p[wid] = gs;
                a.lossp[wid] = lsum;
            }
        } else {
            // check: lane (lg, lr < 4) compares row 4 lg + lr with the atlas
            // (the shuffle runs in every lane)
            const int rr = 4 * lg + (lr & 3);
            const float4 in = input_of(in_mine, rr);
            const int64_t row = row0 + rr;
            const float t = (lr & 3) == 0 ? T[0] : (lr & 3) == 1 ? T[1] : (lr & 3) == 2 ? T[2] : T[3];
            if (lr < 4 && row < a.n) {
                const float err = fabsf(t - in.w);
                if (err > a.thresh) {
                    const int64_t grow = a.row_offset + row;
                    if (grow < a.n_grid) {
                        // a texel-centre node (row = (k H + i) W + j) is a corner of the
                        // cells (i - 1 or i, j - 1 or j, k - 1 or k): flag all their regions
                        const int64_t plane = (int64_t)a.g.H * a.g.W;
                        const int k = (int)(grow / plane);
                        const int64_t rem = grow - (int64_t)k * plane;
                        const int i = (int)(rem / a.g.W), j = (int)(rem - (int64_t)i * a.g.W);
                        for (int dk = -1; dk <= 0; ++dk)
                            for (int di = -1; di <= 0; ++di)
                                for (int dj = -1; dj <= 0; ++dj) {
                                    const int kc = min(max(k + dk, 0), a.g.K - 2);
                                    const int ic = max(i + di, 0), jc = max(j + dj, 0);
                                    a.mask_out[(kc / 8) * a.g.ntiles + (ic / ::dgsm::kTile) * a.g.TW +
                                               jc / ::dgsm::kTile] = 1;
                                }
                    } else {
                        a.mask_out[atlas_region(a.g, in.x, in.y, in.z)] = 1;
                    }
                    atomicAdd(a.check_stats, 1u);
                }
                atomicMax(a.check_stats + 1, __float_as_uint(err));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Inference with the weights held in registers.  Wave w of kIW owns output
// features [16 kIJ w, 16 kIJ (w + 1)) of every layer: its weight rows stay in VGPRs as
// the A operand of the MFMA for the whole kernel, and the activations of kIRB
// 16-sample blocks are the B operand, so each product H^T = W X^T leaves four
// consecutive features of one sample per lane (one 8-byte LDS store) and each
// activation fragment read from LDS feeds two MFMAs.  Features: one thread per
// (sample, frequency) writes its six sines and cosines; the zero padding of the
// feature rows is written once.
// ---------------------------------------------------------------------------
constexpr int kIW = 4;      // waves per inference block
constexpr int kIJ = kH / 16 / kIW;   // 16-feature output tiles per wave
constexpr int kIRB = 2;     // 16-sample blocks per iteration
constexpr int kIRows = kIRB * kRows;

typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;

__global__ __launch_bounds__(kWave * kIW, 2) void infer_kernel(FwdArgs a) {
    __shared__ bf16x8 feat[kIRB][kRows * 16];      // [sample block][sample, chunk] (swizzled)
    __shared__ bf16x8 hid[2][kIRB][kRows * 16];
    __shared__ float4 btab[4][kH / 4];            // biases of the four layers
    __shared__ float w4t[kH];
    __shared__ float zpart[kIRows][kIW];
    __shared__ double3 rin[kIRows];
    __shared__ double cturn[kNF];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int light = blockIdx.y;
    const float* P = a.params + (size_t)light * kNParams;
    const __bf16* Wg = a.wb + (size_t)light * 4 * kH * kH;
    const int lr = lane % 16, lg = lane / 16;
    // this wave's weight rows: layer l, feature tile j (features 16 (2 wave + j) ..), k-step kk
    bf16x8 Wf[4][kIJ][4];
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int j = 0; j < kIJ; ++j) {
            const int row = 16 * (kIJ * wave + j) + lr;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
                Wf[l][j][kk] = *reinterpret_cast<const bf16x8*>(Wg + (size_t)l * kH * kH + (size_t)row * kH + 32 * kk +
                                                                8 * lg);
        }
    for (int q = tid; q < 4 * kH; q += kWave * kIW)
        reinterpret_cast<float*>(btab)[q] = P[(q / kH) * kLayer + kH * kH + q % kH];
    for (int q = tid; q < kH; q += kWave * kIW) w4t[q] = P[kOffW4 + q];
    for (int q = tid; q < kIRB * kRows * 16; q += kWave * kIW) {   // zero padding of the feature rows
        bf16x8 z;
#pragma unroll
        for (int e = 0; e < 8; ++e) z[e] = to_bf16(0.f);
        (&feat[0][0])[q] = z;
    }
    const float b4 = P[kOffB4];
    if (tid < kNF) cturn[tid] = turns_per_unit(tid, a.g.W);
    const int64_t ntile = (a.n + kIRows - 1) / kIRows;
    // the next tile's points are loaded one iteration ahead (threads tid < kIRows)
    float px = 0.f, py = 0.f, pz = 0.f;
    auto load_pt = [&](int64_t tt) {
        const int64_t rr = tt * kIRows + tid;
        if (tid < kIRows && tt < ntile && rr < a.n) {
            px = a.points[3 * rr];
            py = a.points[3 * rr + 1];
            pz = a.points[3 * rr + 2];
        }
    };
    load_pt(blockIdx.x);
    __bf16* fe = reinterpret_cast<__bf16*>(&feat[0][0]);

    for (int64_t t = blockIdx.x; t < ntile; t += gridDim.x) {
        const int64_t row0 = t * kIRows;
        if (tid < kIRows) {
            double3 in = make_double3(0.0, 0.0, 0.0);
            if (row0 + tid < a.n) encode_point_f64(px, py, pz, a.lights + 3 * light, a.g, in.x, in.y, in.z);
            rin[tid] = in;
        }
        load_pt(t + gridDim.x);
        __syncthreads();
        // features: thread -> (sample, frequency) pairs tid, tid + 256, ... of kIRows x kNF
        static_assert(kIRows * kNF % (kWave * kIW) == 0, "whole (sample, frequency) sweeps");
#pragma unroll
        for (int h = 0; h < kIRows * kNF / (kWave * kIW); ++h) {
            const int pr = tid + h * kWave * kIW;
            const int smp = pr / kNF, i = pr % kNF;
            const double3 in = rin[smp];
            __bf16* rowp = fe + (size_t)(smp / kRows) * kRows * 16 * 8;
            const int r = smp % kRows;
            auto put = [&](int f, float v) { rowp[swz(r, f / 8) * 8 + (f % 8)] = to_bf16(v); };
            if (i == 0) {
                put(0, (float)in.x);
                put(1, (float)in.y);
                put(2, (float)in.z);
            }
            const double c = cturn[i];
            float sn, cs;
            fourier_pair(c, in.x, sn, cs);
            put(3 + 6 * i, sn);
            put(4 + 6 * i, cs);
            fourier_pair(c, in.y, sn, cs);
            put(5 + 6 * i, sn);
            put(6 + 6 * i, cs);
            fourier_pair(c, in.z, sn, cs);
            put(7 + 6 * i, sn);
            put(8 + 6 * i, cs);
        }
        __syncthreads();
        f32x4 acc[kIRB][kIJ];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            const bf16x8(*src)[kRows * 16] = l == 0 ? feat : hid[(l - 1) & 1];
#pragma unroll
            for (int j = 0; j < kIJ; ++j) {
                const float4 bb = btab[l][(16 * (kIJ * wave + j) + 4 * lg) / 4];
#pragma unroll
                for (int rb = 0; rb < kIRB; ++rb) acc[rb][j] = f32x4{bb.x, bb.y, bb.z, bb.w};
            }
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int rb = 0; rb < kIRB; ++rb) {
                    const bf16x8 xv = src[rb][swz(lr, lg + 4 * kk)];
#pragma unroll
                    for (int j = 0; j < kIJ; ++j) acc[rb][j] = mfma(Wf[l][j][kk], xv, acc[rb][j]);
                }
#pragma unroll
            for (int rb = 0; rb < kIRB; ++rb)
#pragma unroll
                for (int j = 0; j < kIJ; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[rb][j][r] = fmaxf(acc[rb][j][r], 0.f);
            if (l < 3) {
                __bf16* dst = reinterpret_cast<__bf16*>(&hid[l & 1][0][0]);
#pragma unroll
                for (int rb = 0; rb < kIRB; ++rb)
#pragma unroll
                    for (int j = 0; j < kIJ; ++j) {
                        const int f0 = 16 * (kIJ * wave + j) + 4 * lg;   // four consecutive features of sample lr
                        bf16x4 v;
#pragma unroll
                        for (int r = 0; r < 4; ++r) v[r] = to_bf16(acc[rb][j][r]);
                        *reinterpret_cast<bf16x4*>(dst + (size_t)rb * kRows * 16 * 8 + swz(lr, f0 / 8) * 8 + (f0 % 8)) =
                            v;
                    }
                __syncthreads();
            }
        }
        // output layer: this wave's share of z = w4 . h4 per sample, summed over waves in LDS
#pragma unroll
        for (int rb = 0; rb < kIRB; ++rb) {
            float zp = 0.f;
#pragma unroll
            for (int j = 0; j < kIJ; ++j) {
                const int f0 = 16 * (kIJ * wave + j) + 4 * lg;
#pragma unroll
                for (int r = 0; r < 4; ++r) zp += w4t[f0 + r] * acc[rb][j][r];
            }
            zp += __shfl_xor(zp, 16, kWave);
            zp += __shfl_xor(zp, 32, kWave);
            if (lg == 0) zpart[rb * kRows + lr][wave] = zp;
        }
        __syncthreads();
        if (tid < kIRows && row0 + tid < a.n) {
            float z = b4;
#pragma unroll
            for (int w = 0; w < kIW; ++w) z += zpart[tid][w];
            a.T[(size_t)light * a.n + row0 + tid] = 1.f / (1.f + __expf(z));
        }
        __syncthreads();
    }
}

// Atlas fallback after inference: points whose region is flagged take the
// trilinear atlas value (one thread per (point, light); the atlas is read
// only for flagged points).
template <typename InT>
__global__ __launch_bounds__(256) void fallback_kernel(FwdArgs a) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n) return;
    const int light = blockIdx.y;
    float u, v, rho, r;
    encode_point(a.points[3 * p], a.points[3 * p + 1], a.points[3 * p + 2], a.lights + 3 * light, a.g, u, v, rho, r);
    const size_t nreg = (size_t)((a.g.K + 7) / 8) * a.g.ntiles;
    if (!a.mask[light * nreg + atlas_region(a.g, u, v, rho)]) return;
    const size_t tsz = (size_t)a.g.K * a.g.H * a.g.W;
    int region;
    a.T[(size_t)light * a.n + p] = atlas_at(reinterpret_cast<const InT*>(a.atlas) + light * tsz, a.g, u, v, rho, region);
}

// ---------------------------------------------------------------------------
// Backward: data gradients through layers 3..1, pre-activation gradients
// stashed transposed (BF16) for the weight gradients, bias partials.
// ---------------------------------------------------------------------------
struct BwdArgs {
    const float* params;
    const __bf16* wb;     // [4][128][128]
    int64_t n;
    const __bf16* xt;     // [4][128][n]
    const float* h4;      // [n][128]
    const float* gz;      // [n]
    __bf16* dzt;          // [4][128][n]
    float* dbp;           // [n/16][4][128]
};

__global__ __launch_bounds__(256) void bwd_kernel(BwdArgs a) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    bf16x8* wt = reinterpret_cast<bf16x8*>(smem);                 // [3][128 cols j][16 chunks of k]: W_l^T, l = 1..3
    bf16x8* act = wt + 3 * kH * 16;                               // [4 waves][16 rows][16 chunks]
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    __bf16* wth = reinterpret_cast<__bf16*>(wt);
    for (int q = tid; q < 3 * kH * kH; q += 256) {
        const int l = q / (kH * kH), rem = q % (kH * kH), k = rem / kH, j = rem % kH;   // W_{l+1}[k][j]
        wth[(l * kH * 16 + swz(j, k / 8)) * 8 + (k % 8)] = a.wb[(size_t)(l + 1) * kH * kH + (size_t)k * kH + j];
    }
    __syncthreads();
    bf16x8* my = act + wave * kRows * 16;
    __bf16* myh = reinterpret_cast<__bf16*>(my);
    const int lr = lane % 16, lg = lane / 16;
    const float* w4 = a.params + kOffW4;
    const int ntile = (int)((a.n + kTileRows - 1) / kTileRows);
    for (int t = blockIdx.x; t < ntile; t += gridDim.x) {
        const int64_t row0 = (int64_t)t * kTileRows + wave * kRows;
        if (row0 >= a.n) continue;            // n is a multiple of 16: a wave's rows are all in or all out
        const int64_t wid = row0 / kRows;
        f32x4 da[8];
        // layer 3: da3 = gz w4 (h4 > 0)
        float g[4];
        for (int r = 0; r < 4; ++r) g[r] = a.gz[row0 + 4 * lg + r];
        for (int n = 0; n < 8; ++n) {
            const int col = 16 * n + lr;
            const float w = w4[col];
            for (int r = 0; r < 4; ++r) {
                const float h = a.h4[(size_t)(row0 + 4 * lg + r) * kH + col];
                da[n][r] = h > 0.f ? g[r] * w : 0.f;
            }
        }
        for (int l = 3; l >= 0; --l) {
            // stash bf16(da_l) transposed, bias partial, and the MFMA A operand
            __builtin_amdgcn_wave_barrier();
            for (int n = 0; n < 8; ++n) {
                const int col = 16 * n + lr;
                float s = 0.f;
                __bf16* dst = a.dzt + (size_t)l * kH * a.n + (size_t)col * a.n + row0 + 4 * lg;
                for (int r = 0; r < 4; ++r) {
                    const __bf16 b = to_bf16(da[n][r]);
                    dst[r] = b;
                    myh[swz(4 * lg + r, col / 8) * 8 + (col % 8)] = b;
                    s += da[n][r];
                }
                s += __shfl_xor(s, 16, kWave);
                s += __shfl_xor(s, 32, kWave);
                if (lg == 0) a.dbp[((size_t)wid * 4 + l) * kH + col] = s;
            }
            if (l == 0) break;
            __builtin_amdgcn_s_waitcnt(0xc07f);
            __builtin_amdgcn_wave_barrier();
            // dx_l = da_l W_l ; da_{l-1} = dx_l (x_l > 0)
            const bf16x8* Wt = wt + (l - 1) * kH * 16;
            f32x4 dx[8];
            for (int n = 0; n < 8; ++n) dx[n] = f32x4{0.f, 0.f, 0.f, 0.f};
            for (int kk = 0; kk < 4; ++kk) {
                const bf16x8 av = my[swz(lr, lg + 4 * kk)];
                for (int n = 0; n < 8; ++n) dx[n] = mfma(av, Wt[swz(16 * n + lr, lg + 4 * kk)], dx[n]);
            }
            for (int n = 0; n < 8; ++n) {
                const int col = 16 * n + lr;
                const __bf16* xs = a.xt + (size_t)l * kH * a.n + (size_t)col * a.n + row0 + 4 * lg;
                for (int r = 0; r < 4; ++r) da[n][r] = (float)xs[r] > 0.f ? dx[n][r] : 0.f;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradients: partial dW_l over one chunk of rows, MFMA over the rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void wgrad_kernel(const __bf16* __restrict__ dzt, const __bf16* __restrict__ xt,
                                                    int64_t n, int chunk, float* __restrict__ dwp) {
    const int c = blockIdx.x, l = blockIdx.y;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int lr = lane % 16, lg = lane / 16;
    const int64_t k0 = (int64_t)c * chunk, k1 = min((int64_t)(c + 1) * chunk, n);
    const __bf16* Z = dzt + (size_t)l * kH * n;
    const __bf16* X = xt + (size_t)l * kH * n;
    f32x4 acc[2][8];
    for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 8; ++q) acc[m][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t k = k0; k < k1; k += 32) {
        const int64_t kl = k + 8 * lg;
        bf16x8 am[2], bq[8];
        for (int m = 0; m < 2; ++m)
            am[m] = *reinterpret_cast<const bf16x8*>(Z + (size_t)(32 * wave + 16 * m + lr) * n + kl);
        for (int q = 0; q < 8; ++q) bq[q] = *reinterpret_cast<const bf16x8*>(X + (size_t)(16 * q + lr) * n + kl);
        for (int m = 0; m < 2; ++m)
            for (int q = 0; q < 8; ++q) acc[m][q] = mfma(am[m], bq[q], acc[m][q]);
    }
    float* out = dwp + ((size_t)c * 4 + l) * kH * kH;
    for (int m = 0; m < 2; ++m)
        for (int q = 0; q < 8; ++q)
            for (int r = 0; r < 4; ++r)
                out[(size_t)(32 * wave + 16 * m + 4 * lg + r) * kH + 16 * q + lr] = acc[m][q][r];
}

// ---------------------------------------------------------------------------
// Fixed-order gradient reduction, optional Adam, BF16 weight copies.
// ---------------------------------------------------------------------------
struct ReduceArgs {
    float* params;          // updated in place when adam
    float* m;               // [kNParams] (adam)
    float* v;
    __bf16* wb;             // [4][128][128] refreshed BF16 weights
    const float* dwp;       // [nchunk][4][128][128]
    int nchunk;
    const float* dbp;       // [nw][4][128]
    const float* dw4p;      // [nw][128]
    const float* db4p;      // [nw]
    const float* lossp;     // [nw]
    int nw;
    float* gvec;            // [kVecOut] reduced small vectors (vec_reduce_kernel)
    float* grad_out;        // optional [kNParams]
    float* loss_out;        // optional [1]
    int adam;
    float lr, beta1, beta2, eps, bc1, bc2;   // bc = 1 - beta^t
};

// Per-wave partials of the small vectors (biases, w4, b4, loss) summed over
// the waves: one block per output entry, a strided pass then a fixed tree, so
// the order (and the result) is the same on every run.
constexpr int kVecOut = 4 * kH + kH + 2;     // b0..b3, w4, b4, loss

__global__ __launch_bounds__(256) void vec_reduce_kernel(ReduceArgs a) {
    __shared__ float red[256];
    const int o = blockIdx.x, tid = threadIdx.x;
    const float* src;
    int stride;
    if (o < 4 * kH) { src = a.dbp + o; stride = 4 * kH; }
    else if (o < 5 * kH) { src = a.dw4p + (o - 4 * kH); stride = kH; }
    else if (o == 5 * kH) { src = a.db4p; stride = 1; }
    else { src = a.lossp; stride = 1; }
    float s = 0.f;
    for (int w = tid; w < a.nw; w += 256) s += src[(size_t)w * stride];
    red[tid] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) red[tid] += red[tid + h];
        __syncthreads();
    }
    if (tid == 0) a.gvec[o] = red[0];
}

__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs a) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p == 0 && a.loss_out) *a.loss_out = a.gvec[5 * kH + 1];
    if (p >= kNParams) return;
    float g = 0.f;
    int wl = -1, wi = 0;
    if (p < kOffW4) {
        const int l = p / kLayer, q = p % kLayer;
        if (q < kH * kH) {
            for (int c = 0; c < a.nchunk; ++c) g += a.dwp[((size_t)c * 4 + l) * kH * kH + q];
            wl = l;
            wi = q;
        } else {
            g = a.gvec[l * kH + (q - kH * kH)];
        }
    } else if (p < kOffB4) {
        g = a.gvec[4 * kH + (p - kOffW4)];
    } else {
        g = a.gvec[5 * kH];
    }
    if (a.grad_out) a.grad_out[p] = g;
    float val = a.params[p];
    if (a.adam) {
        const float m = a.beta1 * a.m[p] + (1.f - a.beta1) * g;
        const float v = a.beta2 * a.v[p] + (1.f - a.beta2) * g * g;
        a.m[p] = m;
        a.v[p] = v;
        val -= a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
        if (wl == 0 && (wi % kH) >= kDin) val = 0.f;   // padded feature columns stay zero
        a.params[p] = val;
    }
    if (wl >= 0 && a.wb) a.wb[(size_t)wl * kH * kH + wi] = to_bf16(val);
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* __restrict__ params, int L,
                                                      __bf16* __restrict__ wb) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= (int64_t)L * 4 * kH * kH) return;
    const int64_t light = q / (4 * kH * kH), r = q % (4 * kH * kH);
    const int l = (int)(r / (kH * kH)), e = (int)(r % (kH * kH));
    wb[q] = to_bf16(params[light * kNParams + l * kLayer + e]);
}

}  // namespace mlp
}  // namespace dgsm

using namespace dgsm;
using namespace dgsm::mlp;

namespace {

constexpr int kChunk = 512;   // rows per weight-gradient partial

struct TrainWs {
    float4* uvrt;
    __bf16 *xt, *dzt, *wb;
    float *h4, *gz, *dwp, *dbp, *dw4p, *db4p, *lossp, *gvec;
    int nchunk, nw;
    size_t total;
};

TrainWs train_ws(unsigned char* base, int64_t B) {
    TrainWs w{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base ? base + off : nullptr;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    w.nchunk = (int)((B + kChunk - 1) / kChunk);
    w.nw = (int)(B / kRows);
    w.uvrt = reinterpret_cast<float4*>(take(sizeof(float4) * B));
    w.xt = reinterpret_cast<__bf16*>(take(2 * 4 * kH * (size_t)B));
    w.dzt = reinterpret_cast<__bf16*>(take(2 * 4 * kH * (size_t)B));
    w.wb = reinterpret_cast<__bf16*>(take(2 * 4 * kH * kH));
    w.h4 = reinterpret_cast<float*>(take(4 * kH * (size_t)B));
    w.gz = reinterpret_cast<float*>(take(4 * (size_t)B));
    w.dwp = reinterpret_cast<float*>(take(4 * (size_t)w.nchunk * 4 * kH * kH));
    w.dbp = reinterpret_cast<float*>(take(4 * (size_t)w.nw * 4 * kH));
    w.dw4p = reinterpret_cast<float*>(take(4 * (size_t)w.nw * kH));
    w.db4p = reinterpret_cast<float*>(take(4 * (size_t)w.nw));
    w.lossp = reinterpret_cast<float*>(take(4 * (size_t)w.nw));
    w.gvec = reinterpret_cast<float*>(take(4 * (size_t)kVecOut));
    w.total = off;
    return w;
}

constexpr size_t fwd_smem(int nwv) { return (size_t)(4 * kH * 16 + nwv * kRows * 16) * 16; }
constexpr size_t kFwdSmem = fwd_smem(kWaves);
constexpr size_t kBwdSmem = (size_t)(3 * kH * 16 + kWaves * kRows * 16) * 16;

int grid_rows(int64_t n, int rows = kTileRows) {
    const int64_t t = (n + rows - 1) / rows;
    return (int)(t < 1024 ? (t < 1 ? 1 : t) : 1024);
}

hipError_t set_smem() {
    static const hipError_t e = [] {
        hipError_t r = hipFuncSetAttribute((const void*)fwd_kernel<kTrain, kWaves>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFwdSmem);
        if (r == hipSuccess)
            r = hipFuncSetAttribute((const void*)fwd_kernel<kCheck, kWaves>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFwdSmem);
        if (r == hipSuccess)
            r = hipFuncSetAttribute((const void*)bwd_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)kBwdSmem);
        return r;
    }();
    return e;
}

// forward (train) + backward + weight gradients on the samples in w.uvrt
dgsm_status enqueue_fwd_bwd(const float* params, const Geom& g, int64_t B, const TrainWs& w, hipStream_t st) {
    FwdArgs f{};
    f.g = g;
    f.params = params;
    f.wb = w.wb;
    f.n = B;
    f.uvrt = w.uvrt;
    f.xt = w.xt;
    f.h4 = w.h4;
    f.gz = w.gz;
    f.dw4p = w.dw4p;
    f.db4p = w.db4p;
    f.lossp = w.lossp;
    f.inv_n = 1.f / (float)B;
    fwd_kernel<kTrain, kWaves><<<dim3(grid_rows(B), 1), kWave * kWaves, kFwdSmem, st>>>(f);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    BwdArgs b{params, w.wb, B, w.xt, w.h4, w.gz, w.dzt, w.dbp};
    bwd_kernel<<<grid_rows(B), 256, kBwdSmem, st>>>(b);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    wgrad_kernel<<<dim3(w.nchunk, 4), 256, 0, st>>>(w.dzt, w.xt, B, kChunk, w.dwp);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

Geom geom_of(const dgsm_atlas_desc_t* d) { return make_geom(*d); }

// The learned field is a function of the octahedral code (u, v) of the
// direction: it is defined over the octahedral atlas only.
dgsm_status validate_mlp_desc(const dgsm_atlas_desc_t* d) {
    const dgsm_status st = validate_desc(d);
    if (st != DGSM_OK) return st;
    return d->param == DGSM_PARAM_OCTAHEDRAL ? DGSM_OK : DGSM_EUNSUPPORTED;
}

}  // namespace

extern "C" size_t dgsm_mlp_workspace_size(int64_t batch) {
    if (batch < 32 || batch % 32) return 0;
    return train_ws(nullptr, batch).total;
}

extern "C" dgsm_status dgsm_mlp_grad(const float* params, const float* uvrt, int64_t B,
                                     const dgsm_atlas_desc_t* desc, float* grad, float* loss, void* ws,
                                     size_t ws_bytes, void* stream) {
    dgsm_status st = validate_mlp_desc(desc);
    if (st != DGSM_OK) return st;
    if (!params || !uvrt || !grad || B < 32 || B % 32) return DGSM_EINVAL;
    const TrainWs w = train_ws(reinterpret_cast<unsigned char*>(ws), B);
    if (!ws || ws_bytes < w.total) return DGSM_EWORKSPACE;
    if (set_smem() != hipSuccess) return DGSM_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(w.uvrt, uvrt, sizeof(float4) * B, hipMemcpyDeviceToDevice, s) != hipSuccess) return DGSM_EHIP;
    to_bf16_kernel<<<(4 * kH * kH + 255) / 256, 256, 0, s>>>(params, 1, w.wb);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    if ((st = enqueue_fwd_bwd(params, geom_of(desc), B, w, s)) != DGSM_OK) return st;
    ReduceArgs r{};
    r.params = const_cast<float*>(params);
    r.dwp = w.dwp; r.nchunk = w.nchunk; r.dbp = w.dbp; r.dw4p = w.dw4p; r.db4p = w.db4p; r.lossp = w.lossp;
    r.nw = w.nw; r.gvec = w.gvec; r.grad_out = grad; r.loss_out = loss; r.adam = 0;
    vec_reduce_kernel<<<kVecOut, 256, 0, s>>>(r);
    reduce_kernel<<<(kNParams + 255) / 256, 256, 0, s>>>(r);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

extern "C" dgsm_status dgsm_mlp_train(float* params, float* adam_mv, const dgsm_atlas_desc_t* desc,
                                      const void* atlas_l, const dgsm_mlp_train_t* opt, float* loss_out, void* ws,
                                      size_t ws_bytes, void* stream) {
    dgsm_status st = validate_mlp_desc(desc);
    if (st != DGSM_OK) return st;
    if (!params || !adam_mv || !atlas_l || !opt || opt->steps < 0 || opt->batch < 32 || opt->batch % 32)
        return DGSM_EINVAL;
    const int64_t B = opt->batch;
    const TrainWs w = train_ws(reinterpret_cast<unsigned char*>(ws), B);
    if (!ws || ws_bytes < w.total) return DGSM_EWORKSPACE;
    if (set_smem() != hipSuccess) return DGSM_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Geom g = geom_of(desc);
    to_bf16_kernel<<<(4 * kH * kH + 255) / 256, 256, 0, s>>>(params, 1, w.wb);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    for (int i = 0; i < opt->steps; ++i) {
        const int t = opt->step0 + i + 1;   // Adam step count
        const unsigned blocks = (unsigned)((B + 255) / 256);
        if (desc->dtype == DGSM_F16)
            sample_kernel<__half><<<blocks, 256, 0, s>>>(reinterpret_cast<const __half*>(atlas_l), g, B, opt->seed,
                                                        (uint32_t)t, w.uvrt);
        else
            sample_kernel<float><<<blocks, 256, 0, s>>>(reinterpret_cast<const float*>(atlas_l), g, B, opt->seed,
                                                       (uint32_t)t, w.uvrt);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
        if ((st = enqueue_fwd_bwd(params, g, B, w, s)) != DGSM_OK) return st;
        // cosine decay from lr0 to lr1 over the steps of this call
        const double ph = opt->steps > 1 ? (double)i / (double)(opt->steps - 1) : 0.0;
        const float lr = (float)(opt->lr1 + 0.5 * (opt->lr0 - opt->lr1) * (1.0 + cos(3.141592653589793 * ph)));
        ReduceArgs r{};
        r.params = params; r.m = adam_mv; r.v = adam_mv + kNParams; r.wb = w.wb;
        r.dwp = w.dwp; r.nchunk = w.nchunk; r.dbp = w.dbp; r.dw4p = w.dw4p; r.db4p = w.db4p; r.lossp = w.lossp;
        r.nw = w.nw; r.loss_out = loss_out ? loss_out + i : nullptr; r.adam = 1;
        r.lr = lr; r.beta1 = opt->beta1; r.beta2 = opt->beta2; r.eps = opt->eps;
        r.bc1 = (float)(1.0 - pow((double)opt->beta1, (double)t));
        r.bc2 = (float)(1.0 - pow((double)opt->beta2, (double)t));
        r.gvec = w.gvec;
        vec_reduce_kernel<<<kVecOut, 256, 0, s>>>(r);
        reduce_kernel<<<(kNParams + 255) / 256, 256, 0, s>>>(r);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    }
    return DGSM_OK;
}

extern "C" size_t dgsm_mlp_infer_workspace_size(int32_t n_lights) {
    return n_lights < 1 ? 0 : (size_t)n_lights * 4 * kH * kH * sizeof(__bf16);
}

extern "C" dgsm_status dgsm_mlp_check(const float* params, const dgsm_atlas_desc_t* desc, const void* atlas_l,
                                      int64_t n_check, uint32_t seed, float thresh, unsigned char* mask,
                                      unsigned int* stats, void* ws, size_t ws_bytes, void* stream) {
    dgsm_status st = validate_mlp_desc(desc);
    if (st != DGSM_OK) return st;
    if (!params || !atlas_l || !mask || !stats || n_check < 1) return DGSM_EINVAL;
    const size_t need = dgsm_mlp_infer_workspace_size(1) + ((sizeof(float4) * n_check + 255) & ~(size_t)255);
    if (!ws || ws_bytes < need) return DGSM_EWORKSPACE;
    if (set_smem() != hipSuccess) return DGSM_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Geom g = geom_of(desc);
    __bf16* wb = reinterpret_cast<__bf16*>(ws);
    float4* uvrt = reinterpret_cast<float4*>(reinterpret_cast<unsigned char*>(ws) + dgsm_mlp_infer_workspace_size(1));
    to_bf16_kernel<<<(4 * kH * kH + 255) / 256, 256, 0, s>>>(params, 1, wb);
    const unsigned blocks = (unsigned)((n_check + 255) / 256);
    if (desc->dtype == DGSM_F16)
        sample_kernel<__half><<<blocks, 256, 0, s>>>(reinterpret_cast<const __half*>(atlas_l), g, n_check, seed,
                                                    0xFFFFFFFFu, uvrt);
    else
        sample_kernel<float><<<blocks, 256, 0, s>>>(reinterpret_cast<const float*>(atlas_l), g, n_check, seed,
                                                   0xFFFFFFFFu, uvrt);
    FwdArgs f{};
    f.g = g; f.params = params; f.wb = wb; f.n = n_check; f.uvrt = uvrt; f.atlas = atlas_l;
    f.mask_out = mask; f.thresh = thresh; f.check_stats = stats; f.atlas_f16 = desc->dtype == DGSM_F16;
    fwd_kernel<kCheck, kWaves><<<dim3(grid_rows(n_check), 1), kWave * kWaves, kFwdSmem, s>>>(f);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

namespace {
constexpr int64_t kGridChunk = int64_t(1) << 22;   // check rows staged per pass

int64_t grid_rows_total(const dgsm_atlas_desc_t* d, int32_t n_per) {
    const Geom g = make_geom(*d);
    const int64_t regions = (int64_t)((g.K + 7) / 8) * g.ntiles;
    return (int64_t)g.H * g.W * g.K + regions * n_per;
}
}  // namespace

extern "C" size_t dgsm_mlp_check_grid_workspace_size(const dgsm_atlas_desc_t* desc, int32_t n_per_region) {
    if (validate_mlp_desc(desc) != DGSM_OK || n_per_region < 0) return 0;
    const int64_t rows = std::min(grid_rows_total(desc, n_per_region), kGridChunk);
    return dgsm_mlp_infer_workspace_size(1) + ((sizeof(float4) * (size_t)rows + 255) & ~(size_t)255);
}

extern "C" dgsm_status dgsm_mlp_check_grid(const float* params, const dgsm_atlas_desc_t* desc, const void* atlas_l,
                                           int32_t n_per_region, uint32_t seed, float thresh, unsigned char* mask,
                                           unsigned int* stats, void* ws, size_t ws_bytes, void* stream) {
    dgsm_status st = validate_mlp_desc(desc);
    if (st != DGSM_OK) return st;
    if (!params || !atlas_l || !mask || !stats || n_per_region < 0) return DGSM_EINVAL;
    const size_t need = dgsm_mlp_check_grid_workspace_size(desc, n_per_region);
    if (!ws || ws_bytes < need) return DGSM_EWORKSPACE;
    if (set_smem() != hipSuccess) return DGSM_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Geom g = geom_of(desc);
    __bf16* wb = reinterpret_cast<__bf16*>(ws);
    float4* uvrt = reinterpret_cast<float4*>(reinterpret_cast<unsigned char*>(ws) + dgsm_mlp_infer_workspace_size(1));
    to_bf16_kernel<<<(4 * kH * kH + 255) / 256, 256, 0, s>>>(params, 1, wb);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    const int64_t total = grid_rows_total(desc, n_per_region);
    for (int64_t r0 = 0; r0 < total; r0 += kGridChunk) {
        const int64_t n = std::min(kGridChunk, total - r0);
        const unsigned blocks = (unsigned)((n + 255) / 256);
        if (desc->dtype == DGSM_F16)
            grid_sample_kernel<__half><<<blocks, 256, 0, s>>>(reinterpret_cast<const __half*>(atlas_l), g, r0, n,
                                                             n_per_region > 0 ? n_per_region : 1, seed, uvrt);
        else
            grid_sample_kernel<float><<<blocks, 256, 0, s>>>(reinterpret_cast<const float*>(atlas_l), g, r0, n,
                                                            n_per_region > 0 ? n_per_region : 1, seed, uvrt);
        FwdArgs f{};
        f.g = g; f.params = params; f.wb = wb; f.n = n; f.uvrt = uvrt; f.atlas = atlas_l;
        f.mask_out = mask; f.thresh = thresh; f.check_stats = stats; f.atlas_f16 = desc->dtype == DGSM_F16;
        f.row_offset = r0;
        f.n_grid = (int64_t)g.H * g.W * g.K;
        fwd_kernel<kCheck, kWaves><<<dim3(grid_rows(n), 1), kWave * kWaves, kFwdSmem, s>>>(f);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    }
    return DGSM_OK;
}

extern "C" dgsm_status dgsm_mlp_infer(const float* params, const dgsm_lights_t* lights,
                                      const dgsm_atlas_desc_t* desc, const void* atlas, const unsigned char* mask,
                                      const float* points, int64_t P, float* T, void* ws, size_t ws_bytes,
                                      void* stream) {
    dgsm_status st = validate_mlp_desc(desc);
    if (st != DGSM_OK) return st;
    if ((st = validate_lights(lights)) != DGSM_OK) return st;
    if (!params || P < 0 || (P > 0 && (!points || !T)) || (mask && !atlas)) return DGSM_EINVAL;
    if (!ws || ws_bytes < dgsm_mlp_infer_workspace_size(lights->n)) return DGSM_EWORKSPACE;
    if (P == 0) return DGSM_OK;
    if (set_smem() != hipSuccess) return DGSM_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    __bf16* wb = reinterpret_cast<__bf16*>(ws);
    const int64_t nw = (int64_t)lights->n * 4 * kH * kH;
    to_bf16_kernel<<<(unsigned)((nw + 255) / 256), 256, 0, s>>>(params, lights->n, wb);
    FwdArgs f{};
    f.g = geom_of(desc); f.params = params; f.wb = wb; f.n = P; f.points = points; f.lights = lights->pos;
    f.atlas = mask ? atlas : nullptr; f.mask = mask; f.T = T; f.atlas_f16 = desc->dtype == DGSM_F16;
    infer_kernel<<<dim3(grid_rows(P, kIRows), lights->n), kWave * kIW, 0, s>>>(f);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    if (mask) {
        const dim3 grid((unsigned)((P + 255) / 256), lights->n);
        if (f.atlas_f16)
            fallback_kernel<__half><<<grid, 256, 0, s>>>(f);
        else
            fallback_kernel<float><<<grid, 256, 0, s>>>(f);
    }
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}
