// DGSM build on gfx950: light-space binning + per-tile closed-form optical depth.
//
// Pipeline (all lights in every launch, blockIdx.y = light), Sec. 3.2:
//   tile_cone_kernel / super_cone_kernel  bounding cones of the texel-centre
//        directions of every 8x8 atlas tile and of every supertile (8x8 tiles)
//   preprocess_kernel  per Gaussian: whitening rows, beta (Eq. 5), light-to-mean
//        offset in FP64, a rigorous culling cone, the supertile mask and
//        per-block supertile counts
//   scan_kernel        exclusive scan of those counts per supertile
//   bases_kernel       supertile list bases, padded to 64-entry chunks
//   scatter_kernel     stable compaction of Gaussian ids into supertile lists
//                      (ascending id within a list: the summation order is fixed)
//   tile_mask_kernel   each list entry against the <= 64 tiles of its supertile
//                      (cone test, then a separating-plane test), transposed
//                      into one 64-bit hit word per (tile, chunk)
//   tile_build_kernel  one wave per tile: walk its hit words; for every
//        (texel, Gaussian) pair evaluate Eq. 3 on the shells where the erf
//        ramps and add the per-shell increments in LDS; prefix over shells,
//        T = exp(-tau) (Eq. 4), shell-major store.

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"

#include <math.h>

#include <mutex>
#include <vector>

namespace dgsm {

// ---------------------------------------------------------------------------
// Tile and supertile cones
// ---------------------------------------------------------------------------

__device__ inline float inflate_sh(double sh) {
    double v = sh * (1.0 + 1e-5) + 1e-6;
    return (float)(v > 1.0 ? 1.0 : v);
}

// FP64 sum and maximum over a wave (fixed butterfly order: deterministic).
__device__ inline double wave_sum_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ inline double wave_max_d(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// One wave per tile, one lane per texel: axis = normalised sum of the
// texel-centre directions, half-angle from the largest chord to the axis.
// The cone and its cone_cos are stored.
__global__ __launch_bounds__(256) void tile_cone_kernel(Geom g, float4* __restrict__ tcone, float* __restrict__ tcos) {
    const int lane = threadIdx.x % kWave;
    const int t = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (t >= g.ntiles) return;                               // wave-uniform
    const int ty = t / g.TW, tx = t - ty * g.TW;
    const int i = ty * kTile + (lane >> 3), j = tx * kTile + (lane & 7);
    const bool in = i < g.H && j < g.W;
    double x = 0, y = 0, z = 0;
    if (in) texel_dir(g, i, j, x, y, z);
    double sx = wave_sum_d(x), sy = wave_sum_d(y), sz = wave_sum_d(z);
    const double nrm = sqrt(sx * sx + sy * sy + sz * sz);
    sx /= nrm; sy /= nrm; sz /= nrm;
    const double ch = wave_max_d(in ? (x - sx) * (x - sx) + (y - sy) * (y - sy) + (z - sz) * (z - sz) : 0.0);
    if (lane == 0) {
        const float4 c = make_float4((float)sx, (float)sy, (float)sz, inflate_sh(0.5 * sqrt(ch)));
        tcone[t] = c;
        tcos[t] = cone_cos(c);
    }
}

// A supertile cone bounds the cones of its tiles: half-angle = max over tiles
// of (angle to the tile axis + tile half-angle).
// Group cones: group s of a grid of (gh x gw)-tile groups, ngx groups per row
// (supertiles: gh = STH, gw = STW; quads: 2 x 2 tiles; 2 x 2 supertiles).
// One wave per group, the lanes striding over its tiles.
__global__ __launch_bounds__(256) void super_cone_kernel(Geom g, const float4* __restrict__ tcone,
                                                         float4* __restrict__ scone, float* __restrict__ scos,
                                                         int ngroups, int ngx, int gh, int gw) {
    const int lane = threadIdx.x % kWave;
    const int s = blockIdx.x * (256 / kWave) + threadIdx.x / kWave;
    if (s >= ngroups) return;                                // wave-uniform
    const int sy = s / ngx, sx = s - sy * ngx;
    const int ty0 = sy * gh, ty1 = min(ty0 + gh, g.TH);
    const int tx0 = sx * gw, tx1 = min(tx0 + gw, g.TW);
    const int nw = tx1 - tx0, nt = (ty1 - ty0) * nw;
    double ax = 0, ay = 0, az = 0;
    for (int q = lane; q < nt; q += kWave) {
        const float4 c = tcone[(ty0 + q / nw) * g.TW + tx0 + q % nw];
        ax += c.x; ay += c.y; az += c.z;
    }
    ax = wave_sum_d(ax); ay = wave_sum_d(ay); az = wave_sum_d(az);
    const double nrm = sqrt(ax * ax + ay * ay + az * az);
    ax /= nrm; ay /= nrm; az /= nrm;
    double half = 0;
    for (int q = lane; q < nt; q += kWave) {
        const float4 c = tcone[(ty0 + q / nw) * g.TW + tx0 + q % nw];
        const double ch = sqrt((c.x - ax) * (c.x - ax) + (c.y - ay) * (c.y - ay) + (c.z - az) * (c.z - az));
        const double ang = 2.0 * asin(fmin(1.0, 0.5 * ch)) + 2.0 * asin(fmin(1.0, (double)c.w));
        half = fmax(half, ang);
    }
    half = fmin(wave_max_d(half), M_PI);
    if (lane == 0) {
        const float4 c = make_float4((float)ax, (float)ay, (float)az, inflate_sh(sin(0.5 * half)));
        scone[s] = c;
        scos[s] = cone_cos(c);
    }
}


// ---------------------------------------------------------------------------
// Workspace slices
// ---------------------------------------------------------------------------

// Tiles of supertile s: origin, extent and local index t = (ty-ty0)*ntx + (tx-tx0).
struct SuperSpan {
    int ty0, tx0, nty, ntx;
};

__host__ __device__ inline SuperSpan super_span(const Geom& g, int s) {
    const int sy = s / g.SGW, sx = s - sy * g.SGW;
    SuperSpan r;
    r.ty0 = sy * g.STH;
    r.tx0 = sx * g.STW;
    r.nty = min(g.STH, g.TH - r.ty0);
    r.ntx = min(g.STW, g.TW - r.tx0);
    return r;
}

// ---------------------------------------------------------------------------
// Per-Gaussian preprocess + supertile mask + per-block counts
// ---------------------------------------------------------------------------

struct PrepArgs {
    const float* mean;
    const float* scale;
    const float* rot;
    const float* opacity;
    int64_t n;
    const float* lights;   // device [L][3]
    float kappa;
    int beta_mode;         // dgsm_beta_mode
    float eps;             // culling budget (0: no culling)
    int S, SGH, SGW;       // supertile count and grid
    int shape_cached;      // the records hold this set's shapes already: update m and the cone only
    int roi;               // a receiver region is marked: supertiles without a region texel get no entries
    BuildLayout lay;
    unsigned char* ws;
};

// Scale of the tile test's separating plane (see tile_mask_kernel): the
// squared light-to-mean distance over lg P^2, with P^2 = det(Sigma) =
// (s_1 s_2 s_3)^2, and a 3% margin for the FP32 rounding of that test.  0 (the
// plane test never culls) without culling or where the ratio is not finite.
__device__ inline float plane_q(double mx, double my, double mz, float lg, float P2, float eps) {
    if (!(eps > 0.f)) return 0.f;
    const double q = (mx * mx + my * my + mz * mz) / ((double)lg * (double)P2 * 1.03);
    return (q >= 0.0 && q < 3.0e38) ? (float)q : 0.f;
}

__global__ __launch_bounds__(kPrepThreads) void preprocess_kernel(PrepArgs a) {
    __shared__ int bcnt[kMaxSuper];          // this block's entries per supertile
    __shared__ float4 sc[kMaxSuper];         // supertile cones
    __shared__ float scs[kMaxSuper];         // and their cone_cos
    __shared__ float4 gc[kMaxSuper / 4];     // cones of 2x2-supertile groups
    __shared__ float gcs[kMaxSuper / 4];
    const int tid = threadIdx.x;
    const int l = blockIdx.y;
    const LightWs W = light_ws(a.ws, a.lay, l);
    const float4* scone = reinterpret_cast<const float4*>(a.ws + a.lay.scone);
    const float* scos = reinterpret_cast<const float*>(a.ws + a.lay.scos);
    const float4* gcone = reinterpret_cast<const float4*>(a.ws + a.lay.gcone);
    const float* gcos = reinterpret_cast<const float*>(a.ws + a.lay.gcos);
    const int ngx = (a.SGW + 1) / 2, ng = ((a.SGH + 1) / 2) * ngx;
    const float* light = a.lights + 3 * l;
    const int64_t i = (int64_t)blockIdx.x * kPrepThreads + tid;
    const bool in = i < a.n;
    float4 cone = make_float4(0.f, 0.f, 1.f, -1.f);
    if (in) {
        // Culling-cone numerator R0 = s_max sqrt(2 ln(U / eps)) (see below): -1 for
        // a Gaussian that contributes nothing, +inf without culling.  It depends
        // on the Gaussian's shape only, like the rest of the record but m, and is
        // kept in the record for later frames of a rigidly moving set.
        double R0;
        if (!a.shape_cached) {
            double qw = a.rot[4 * i], qx = a.rot[4 * i + 1], qy = a.rot[4 * i + 2], qz = a.rot[4 * i + 3];
            const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
            qw *= qn; qx *= qn; qy *= qn; qz *= qn;
            // columns of R: the principal axes
            const double col[3][3] = {
                {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy + qw * qz), 2 * (qx * qz - qw * qy)},
                {2 * (qx * qy - qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz + qw * qx)},
                {2 * (qx * qz + qw * qy), 2 * (qy * qz - qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
            const double s[3] = {a.scale[3 * i], a.scale[3 * i + 1], a.scale[3 * i + 2]};
            GRec r;
            double tr = 0;
            for (int j = 0; j < 3; ++j) {
                const double is = 1.0 / s[j];
                const double ip = 1.0 / (s[(j + 1) % 3] * s[(j + 2) % 3]);
                tr += is * is;
                for (int c = 0; c < 3; ++c) {
                    r.w[3 * j + c] = (float)(col[j][c] * is);
                    r.c[3 * j + c] = (float)(col[j][c] * ip);
                }
            }
            const double alpha = a.opacity[i];
            const double tau_star = -log1p(-alpha);
            // beta sqrt(2 pi) (the line-integral scale of Eq. 3)
            const double TWO_PI = 6.283185307179586;
            double amp = (double)a.kappa * tau_star * sqrt(tr / 3.0);          // Eq. 5
            if (a.beta_mode == DGSM_BETA_CONSTANT) amp = (double)a.kappa * tau_star * sqrt(TWO_PI);
            else if (a.beta_mode == DGSM_BETA_DENSITY) amp = (double)a.kappa * tau_star / (TWO_PI * s[0] * s[1] * s[2]);
            r.bp = (float)(0.5 * amp);                                        // beta sqrt(pi/2)
            // Per-texel pre-test radius.  The tile build keeps a texel when
            // 2 P0 > eps, with P0 = beta sqrt(pi/2) a^(-1/2) exp(-e0/2).  Since
            // a >= 1/s_max^2 and e0 >= h^2/s_max^2 (h = |m x d|, the distance from
            // mu to the line of the ray), 2 P0 <= 2 bp s_max exp(-h^2/(2 s_max^2)):
            // no texel with h^2 >= 2 s_max^2 ln(2 bp s_max / eps) can be kept.
            const double smax = fmax(s[0], fmax(s[1], s[2]));
            // one logarithm serves both pre-test bounds and the culling cone below:
            // ln(U / eps) with U the larger of 2 bp s_max (bp as stored, FP32) and
            // beta sqrt(2 pi) s_max (FP64), so each bound holds for either
            const double U = fmax(amp * smax, 2.0 * (double)r.bp * smax);
            const double lnU = (a.eps > 0.f && U > (double)a.eps) ? log(U / (double)a.eps) : 0.0;
            {
                double r2 = 3.0e38;                              // eps = 0: every texel is kept
                if (a.eps > 0.f) r2 = 2.0 * smax * smax * lnU;
                r.r2 = (float)fmin(r2 * (1.0 + 1e-5), 3.0e38);
                // The same bound on the whitened offset: 2 P0 <= 2 bp s_max exp(-e0/2)
                // (a^(-1/2) <= s_max), so no texel with e0 >= 2 ln(2 bp s_max / eps) is kept.
                double lg = 3.0e38;
                if (a.eps > 0.f) lg = 2.0 * lnU;
                r.lg = (float)fmin(lg * (1.0 + 1e-5) + 1e-3, 3.0e38);
            }
            if (!(alpha > 0.0) || !(U > (double)a.eps)) R0 = -1.0;
            else R0 = a.eps > 0.f ? smax * sqrt(2.0 * lnU) : INFINITY;
            r.r0 = (float)R0;
            R0 = (double)r.r0;                           // as later frames will read it
            for (int j = 0; j < 4; ++j) r.pad[j] = 0.f;
            r.pad[1] = (float)(s[0] * s[1] * s[2] * s[0] * s[1] * s[2]);   // det(Sigma) = P^2
            r.pad[2] = (float)fmin(smax / fmin(s[0], fmin(s[1], s[2])), 3.0e38);   // kappa(C) = s_max / s_min
            r.mx = (double)light[0] - (double)a.mean[3 * i];
            r.my = (double)light[1] - (double)a.mean[3 * i + 1];
            r.mz = (double)light[2] - (double)a.mean[3 * i + 2];
            r.pad[0] = plane_q(r.mx, r.my, r.mz, r.lg, r.pad[1], a.eps);
            W.rec[i] = r;
        } else {
            R0 = (double)W.rec[i].r0;
            const double mx = (double)light[0] - (double)a.mean[3 * i];
            const double my = (double)light[1] - (double)a.mean[3 * i + 1];
            const double mz = (double)light[2] - (double)a.mean[3 * i + 2];
            W.rec[i].mx = mx;
            W.rec[i].my = my;
            W.rec[i].mz = mz;
            W.rec[i].pad[0] = plane_q(mx, my, mz, W.rec[i].lg, W.rec[i].pad[1], a.eps);
        }

        // Culling cone.  Along any ray the contribution is at most
        // U exp(-h^2 / (2 s_max^2)), U = beta sqrt(2 pi) s_max, with h
        // the distance from mu to the ray (D for rays pointing away).  So it is
        // below eps outside the cone sin(theta) <= (s_max / D) sqrt(2 ln(U / eps)) = R0 / D.
        const double mx = (double)light[0] - (double)a.mean[3 * i];
        const double my = (double)light[1] - (double)a.mean[3 * i + 1];
        const double mz = (double)light[2] - (double)a.mean[3 * i + 2];
        const double D = sqrt(mx * mx + my * my + mz * mz);
        if (R0 < 0.0) {
            cone.w = -1.f;                               // contributes nothing
        } else {
            double shalf = 1.0;                          // global: every direction
            if (D > 0.0) {
                const double sig = R0 / D;
                // sin(theta / 2) for sin(theta) = sig: sig / sqrt(2 (1 + cos(theta)))
                if (sig < 1.0) shalf = sig / sqrt(2.0 * (1.0 + sqrt(1.0 - sig * sig)));
            }
            const double gx = D > 0 ? -mx / D : 0.0, gy = D > 0 ? -my / D : 0.0, gz = D > 0 ? -mz / D : 1.0;
            cone = make_float4((float)gx, (float)gy, (float)gz, inflate_sh(shalf));
        }
        W.cone[i] = cone;
    }
    for (int s = tid; s < a.S; s += kPrepThreads) {
        sc[s] = scone[s];
        scs[s] = scos[s];
        bcnt[s] = 0;
    }
    for (int q = tid; q < ng; q += kPrepThreads) {
        gc[q] = gcone[q];
        gcs[q] = gcos[q];
    }
    __syncthreads();
    // Supertile mask, two levels: a group of 2 x 2 supertiles whose cone this
    // Gaussian's cone misses holds no texel direction within the cone, so its
    // supertiles are not tested (their tiles would all fail the tile test).
    uint64_t m[kMaskWords] = {0, 0, 0, 0};
    const float ca = cone_cos(cone);
    const bool live = in && cone.w >= 0.f;
    for (int q = 0; q < ng; ++q) {
        const bool hit_g = live && cones_touch_c(cone, ca, gc[q], gcs[q]);
        if (ballot(hit_g) == 0ull) continue;
        const int gy = q / ngx, gx = q - gy * ngx;
        for (int d = 0; d < 4; ++d) {
            const int sy = 2 * gy + (d >> 1), sx = 2 * gx + (d & 1);
            if (sy >= a.SGH || sx >= a.SGW) continue;
            const int sidx = sy * a.SGW + sx;
            if (a.roi && !W.roi_super[sidx]) continue;
            const bool hit = hit_g && cones_touch_c(cone, ca, sc[sidx], scs[sidx]);
            if (hit) {
                const uint64_t bit = 1ull << (sidx & 63);
                switch (sidx >> 6) {
                    case 0: m[0] |= bit; break;
                    case 1: m[1] |= bit; break;
                    case 2: m[2] |= bit; break;
                    default: m[3] |= bit; break;
                }
            }
            // one LDS add per wave and supertile (the Gaussians of a wave tend to
            // reach the same few supertiles: per-lane adds would serialise)
            const uint64_t hb = ballot(hit);
            if (hb != 0ull && lane_id() == __builtin_ctzll(hb)) atomicAdd(&bcnt[sidx], __popcll(hb));
        }
    }
    if (in)
        for (int q = 0; q < kMaskWords; ++q) W.mask[(size_t)i * kMaskWords + q] = m[q];
    __syncthreads();
    for (int s = tid; s < a.S; s += kPrepThreads) W.counts[(size_t)s * a.lay.nb + blockIdx.x] = bcnt[s];
}

// ---------------------------------------------------------------------------
// Exclusive scan of the per-block counts, one workgroup per (supertile, light)
// ---------------------------------------------------------------------------

// Inclusive scan of one value per thread over a 256-thread block.
__device__ inline int block_scan_incl(int v, int* wsum) {
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    int x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    if (lane == kWave - 1) wsum[w] = x;
    __syncthreads();
    for (int ww = 0; ww < w; ++ww) x += wsum[ww];
    return x;
}

__global__ __launch_bounds__(256) void scan_kernel(unsigned char* ws, BuildLayout lay) {
    __shared__ int wsum[4];
    const LightWs W = light_ws(ws, lay, blockIdx.y);
    const int s = blockIdx.x, tid = threadIdx.x;
    const int nb = lay.nb;
    int* c = W.counts + (size_t)s * nb;
    int carry = 0;
    for (int base = 0; base < nb; base += 256) {
        const int idx = base + tid;
        const int v = idx < nb ? c[idx] : 0;
        const int x = block_scan_incl(v, wsum);
        if (idx < nb) c[idx] = carry + x - v;
        carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (tid == 0) W.totals[s] = carry;
}

// List base of every supertile, each list padded to a multiple of 64 entries.
// Also clears the per-tile hit counters that the tile masks fill.  Lists that
// would not fit the workspace's capacity are all emptied (need[1] = 1): the
// binning then writes nothing and the accumulation sees no Gaussian, so a too
// small workspace gives a wrong atlas but never a write past its end.
__global__ __launch_bounds__(256) void bases_kernel(unsigned char* ws, BuildLayout lay, int S, int ntiles) {
    __shared__ int wsum[4];
    __shared__ int total;
    const LightWs W = light_ws(ws, lay, blockIdx.x);
    const int s = threadIdx.x;
    const int v = s < S ? (W.totals[s] + 63) & ~63 : 0;
    const int x = block_scan_incl(v, wsum);
    if (s == S - 1) total = x;
    __syncthreads();
    const bool over = (size_t)total > lay.cap;
    if (s < S) {
        W.lbase[s] = over ? 0 : x - v;
        if (over) W.totals[s] = 0;
    }
    if (s == S - 1) W.lbase[S] = over ? 0 : x;
    if (s == 0) {
        W.need[0] = total;
        W.need[1] = over ? 1 : 0;
    }
    for (int t = s; t < ntiles; t += 256) W.hits[t] = 0;
}

// ---------------------------------------------------------------------------
// Stable scatter of Gaussian ids into the supertile lists
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kPrepThreads) void scatter_kernel(unsigned char* ws, BuildLayout lay, int64_t n,
                                                             int S) {
    __shared__ int base_s[kMaxSuper];
    __shared__ int wcnt[kPrepThreads / kWave][kMaxSuper];
    const LightWs W = light_ws(ws, lay, blockIdx.y);
    if (W.need[1]) return;   // the lists did not fit: nothing is scattered
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    for (int s = tid; s < S; s += kPrepThreads) base_s[s] = W.lbase[s] + W.counts[(size_t)s * lay.nb + blockIdx.x];
    const int64_t i = (int64_t)blockIdx.x * kPrepThreads + tid;
    uint64_t m[kMaskWords] = {0, 0, 0, 0};
    if (i < n)
        for (int q = 0; q < kMaskWords; ++q) m[q] = W.mask[(size_t)i * kMaskWords + q];
    for (int s = tid; s < (kPrepThreads / kWave) * kMaxSuper; s += kPrepThreads) (&wcnt[0][0])[s] = 0;
    __syncthreads();
    // only the supertiles some lane of this wave hits: the union of its masks
    uint64_t u[kMaskWords];
#pragma unroll
    for (int q = 0; q < kMaskWords; ++q) u[q] = 64 * q < S ? wave_or(m[q]) : 0ull;
#pragma unroll
    for (int q = 0; q < kMaskWords; ++q)
        for (uint64_t r = u[q]; r; r &= r - 1) {
            const int s = 64 * q + __builtin_ctzll(r);
            const uint64_t bal = ballot((m[q] >> (s & 63)) & 1ull);
            if (lane == 0) wcnt[w][s] = __popcll(bal);
        }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kMaskWords; ++q)
        for (uint64_t r = u[q]; r; r &= r - 1) {
            const int s = 64 * q + __builtin_ctzll(r);
            const bool b = (m[q] >> (s & 63)) & 1ull;
            const uint64_t bal = ballot(b);
            if (b) {
                int off = base_s[s];
                for (int ww = 0; ww < w; ++ww) off += wcnt[ww][s];
                W.lists[off + ballot_rank(bal)] = (int)i;
            }
        }
}

// ---------------------------------------------------------------------------
// Level 2: tile hit words.  One wave per 64-entry chunk of a supertile list.
// ---------------------------------------------------------------------------

// Anisotropic tile test (Sec. 3.2 "Occluder culling via light-space
// footprints"), after the cone test.  Let E be the ellipsoid
// (x - mu)^T Sigma^-1 (x - mu) < lg around the mean (mu relative to the light,
// D = |mu|, g = mu / D).  A ray from the light that misses E carries at most
// cull_eps of the Gaussian's optical depth (the bound behind lg, with e >= lg
// along the whole ray).  E and the ray cone of a tile (axis c, half-angle
// alpha, beta = angle(g, c) > alpha) are separated by the plane through the
// light with normal n = sin(th) g - cos(th) u, th = min(beta - alpha, pi/2), u
// the unit vector from g towards c in their plane: every ray of the cone has
// n.x <= 0, and E lies in n.x > 0 when D sin(th) > sqrt(lg n^T Sigma n).  With
// Sigma = P^2 C^T C (C the rows c_j of the record, P^2 = det Sigma) and
// n sin(beta) = cos(alpha) g - cos(th) c, the test reads
//   (sin(beta) sin(th))^2 D^2 / (lg P^2) > |C (cos(alpha) g - cos(th) c)|^2
// (th < pi/2), or D^2 / (lg P^2) > |C g|^2 (th = pi/2); q = D^2 / (lg P^2) is
// kept with a 3% margin.  For an isotropic Gaussian this is the cone test; for
// the room's Gaussians it drops about a third of the cone test's tile hits.
// FP32 rounding: alpha is inflated by the tile cone (>= 2e-6 rad against
// 2e-7 of axis rounding); the errors (<= 3e-7) of sin(th), cos(th), g and c
// move |C (cos(alpha) g - cos(th) c)| by at most 7e-7 kappa / sin(beta)
// relative (kappa = s_max / s_min, the condition number of C; the vector is
// at least sigma_min(C) sin(beta) long) and sin(th) by 3e-7 / sin(th), so the
// test culls only where sin(th) > 2e-4 and kappa < 7000 sin(beta): the squared
// sides then move by at most 1% and 0.3%, inside the margin.
struct MaskEntry {
    float4 cone;
    float C[9];    // rows c_j of the record
    float q;       // plane scale (0: never culls)
    float kappa;   // s_max / s_min
};

struct PlaneEntry {
    float gx, gy, gz;      // cone axis g
    float Cg0, Cg1, Cg2;   // C g
    float gg;              // |C g|^2
    float q, kappa;
    const float* C;
};

__device__ inline PlaneEntry plane_entry(const MaskEntry& e) {
    PlaneEntry p;
    p.gx = e.cone.x; p.gy = e.cone.y; p.gz = e.cone.z;
    p.Cg0 = e.C[0] * p.gx + e.C[1] * p.gy + e.C[2] * p.gz;
    p.Cg1 = e.C[3] * p.gx + e.C[4] * p.gy + e.C[5] * p.gz;
    p.Cg2 = e.C[6] * p.gx + e.C[7] * p.gy + e.C[8] * p.gz;
    p.gg = p.Cg0 * p.Cg0 + p.Cg1 * p.Cg1 + p.Cg2 * p.Cg2;
    p.q = e.q;
    p.kappa = e.kappa;
    p.C = e.C;
    return p;
}

// cos and sin of a tile cone's half-angle alpha from sin(alpha/2) and cos(alpha/2)
__device__ inline float2 cone_cos_sin(float4 tc, float tcs) {
    return make_float2(1.f - 2.f * tc.w * tc.w, 2.f * tc.w * tcs);
}

// true unless the plane separates the tile cone (axis tc.xyz, half-angle with
// cosine and sine cs) from the entry's ellipsoid
__device__ inline bool plane_keeps(const PlaneEntry& p, float4 tc, float2 cs) {
    const float cb = p.gx * tc.x + p.gy * tc.y + p.gz * tc.z;
    const float xx = p.gy * tc.z - p.gz * tc.y, xy = p.gz * tc.x - p.gx * tc.z, xz = p.gx * tc.y - p.gy * tc.x;
    const float sb = __builtin_amdgcn_sqrtf(xx * xx + xy * xy + xz * xz);
    const float cal = cs.x, sal = cs.y;
    const float sth = sb * cal - cb * sal;                                 // sin(beta - alpha)
    if (!(sth > 2e-4f) || !(sb * 7000.f > p.kappa)) return true;
    const float cth = cb * cal + sb * sal;                                 // cos(beta - alpha)
    if (cth <= 0.f) return !(p.q > p.gg);                                  // th = pi/2: n = g
    const float* C = p.C;
    const float v0 = cal * p.Cg0 - cth * (C[0] * tc.x + C[1] * tc.y + C[2] * tc.z);
    const float v1 = cal * p.Cg1 - cth * (C[3] * tc.x + C[4] * tc.y + C[5] * tc.z);
    const float v2 = cal * p.Cg2 - cth * (C[6] * tc.x + C[7] * tc.y + C[8] * tc.z);
    const float ss = sb * sth;
    return !(ss * ss * p.q > v0 * v0 + v1 * v1 + v2 * v2);
}

// roi: a receiver region is marked; tiles without a region texel get no hits.
__global__ __launch_bounds__(256, 8) void tile_mask_kernel(unsigned char* ws, BuildLayout lay, Geom g, int roi) {
    __shared__ int sbase[kMaxSuper + 1];
    __shared__ int stot[kMaxSuper];
    // per wave: the cones (and cone_cos) of the tiles and quads of its current
    // supertile, read back with wave-uniform addresses (broadcast)
    __shared__ float4 ltc[4][kWave];
    __shared__ float ltcs[4][kWave];
    __shared__ float2 ltca[4][kWave];      // cos, sin of each tile cone's half-angle (plane test)
    __shared__ unsigned long long lres[4][kWave];   // per wave: tile words of the current chunk
    __shared__ int lroi[4][kWave];                   // per wave: the supertile's tiles that hold a region texel
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    __shared__ float4 lqc[4][16];
    __shared__ float lqcs[4][16];
    const LightWs W = light_ws(ws, lay, blockIdx.y);
    const float4* tcone = reinterpret_cast<const float4*>(ws + lay.tcone);
    const float4* qcone = reinterpret_cast<const float4*>(ws + lay.qcone);
    const float* tcos = reinterpret_cast<const float*>(ws + lay.tcos);
    const float* qcos = reinterpret_cast<const float*>(ws + lay.qcos);
    const int nqx = (g.TW + 1) / 2;
    const int tid = threadIdx.x, lane = tid % kWave, wv = tid / kWave;
    for (int s = tid; s <= g.S; s += 256) {
        sbase[s] = W.lbase[s];
        if (s < g.S) stot[s] = W.totals[s];
    }
    __syncthreads();
    const int nchunks = sbase[g.S] / 64;
    const int nwaves = gridDim.x * 4;
    // each wave takes a contiguous run of chunks (mostly of one supertile) and
    // keeps per-tile hit counts in registers (lane t: tile t of the current
    // supertile), flushed with one atomic per tile when the supertile changes
    const int per = (nchunks + nwaves - 1) / nwaves;
    const int gw = blockIdx.x * 4 + tid / kWave;
    const int cbeg = min(nchunks, gw * per), cend = min(nchunks, cbeg + per);
    int s_cur = -1, cnt = 0;
    SuperSpan sp_cur{0, 0, 0, 0};
    int q0y = 0, q0x = 0, nqy_s = 0, nqx_s = 0;
    // The list ids and cones of chunk c + 1 are loaded while chunk c is tested
    // (the cone load waits for its id only).  The loads are unconditional -- a
    // lane without an entry reads the chunk's padding and Gaussian 0 and
    // discards them -- so each wait covers just the loads it needs.  The plane
    // test's record rows are loaded after the cone tests (kept out of the
    // registers of the cone loop: 8 waves per SIMD).
    const float4 kDead = make_float4(0.f, 0.f, 1.f, -1.f);
    auto list_id = [&](int c, bool& valid) {
        int lo = 0, hi = g.S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sbase[mid] <= 64 * c) lo = mid; else hi = mid - 1;
        }
        const int e = 64 * c + lane;
        valid = e < sbase[lo] + stot[lo];
        return W.lists[e];                         // e < lbase[S]: inside the lists
    };
    bool nvalid = false;
    int nid = cbeg < cend ? list_id(cbeg, nvalid) : 0;
    float4 ncone = kDead;
    if (cbeg < cend) ncone = W.cone[nvalid ? nid : 0];
    for (int c = cbeg; c < cend; ++c) {
        const bool valid = nvalid;
        const int gi = valid ? nid : 0;
        const float4 cone = valid ? ncone : kDead;   // dead (w < 0): never reaches a tile
        if (c + 1 < cend) nid = list_id(c + 1, nvalid);
        if (c + 1 < cend) ncone = W.cone[nvalid ? nid : 0];
        // supertile of this chunk: the last s with sbase[s] <= 64 c
        int lo = 0, hi = g.S - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (sbase[mid] <= 64 * c) lo = mid; else hi = mid - 1;
        }
        const int s = lo;
        if (s != s_cur) {
            if (cnt && lane < sp_cur.nty * sp_cur.ntx)
                atomicAdd(W.hits + (sp_cur.ty0 + lane / sp_cur.ntx) * g.TW + sp_cur.tx0 + lane % sp_cur.ntx, cnt);
            s_cur = s;
            cnt = 0;
            sp_cur = super_span(g, s);
            q0y = sp_cur.ty0 / 2;                      // supertile origins are even (8-tile multiples)
            q0x = sp_cur.tx0 / 2;
            nqy_s = (sp_cur.nty + 1) / 2;
            nqx_s = (sp_cur.ntx + 1) / 2;
            __builtin_amdgcn_wave_barrier();           // earlier reads of the cache are done
            if (lane < sp_cur.nty * sp_cur.ntx) {
                const int t = (sp_cur.ty0 + lane / sp_cur.ntx) * g.TW + sp_cur.tx0 + lane % sp_cur.ntx;
                lroi[wv][lane] = !roi || W.roi_mask[t] != 0ull;
                ltc[wv][lane] = tcone[t];
                ltcs[wv][lane] = tcos[t];
                ltca[wv][lane] = cone_cos_sin(tcone[t], tcos[t]);
            }
            if (lane < nqy_s * nqx_s) {
                const int qi = (q0y + lane / nqx_s) * nqx + q0x + lane % nqx_s;
                lqc[wv][lane] = qcone[qi];
                lqcs[wv][lane] = qcos[qi];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        const SuperSpan sp = sp_cur;
        const int nt = sp.nty * sp.ntx;
        const float ca = cone_cos(cone);
        uint64_t mine = 0, row = 0;
        // quads first: the tiles of a quad no lane's cone reaches are skipped.
        // A lane keeps a tile only if its own cone reaches the quad too, so the
        // result never depends on which entries share the wave (with rounding,
        // a tile test can pass where the enclosing quad's test fails).
        // mine (lane t): the entries whose cone reaches tile t; row: the tiles
        // this lane's cone reaches.
        for (int q = 0; q < nqy_s * nqx_s; ++q) {
            const bool hit_q = cones_touch_c(cone, ca, lqc[wv][q], lqcs[wv][q]);
            if (ballot(hit_q) == 0ull) continue;
            const int qy = q / nqx_s, qx = q - qy * nqx_s;
            for (int d = 0; d < 4; ++d) {
                const int ly = 2 * qy + (d >> 1), lx = 2 * qx + (d & 1);   // tile inside the supertile
                if (ly >= sp.nty || lx >= sp.ntx) continue;
                const int t = ly * sp.ntx + lx;
                if (!lroi[wv][t]) continue;                  // no receiver reads this tile
                const bool hit = hit_q && cones_touch_c(cone, ca, ltc[wv][t], ltcs[wv][t]);
                const uint64_t bal = ballot(hit);
                if (hit) row |= 1ull << t;
                if (lane == t) mine = bal;
            }
        }
        // The plane test on each lane's own cone hits only: the SIMD work is
        // the largest number of such tiles of any lane (a few), not every tile
        // some lane's cone reaches (most of the supertile).  A failed test
        // clears the lane's bit in the tile's word.
        lres[wv][lane] = mine;
        wave_sync();
        MaskEntry ent;                                  // the plane test's rows and scale
        ent.cone = cone;
        {
            const GRec* rp = W.rec + gi;
            for (int j = 0; j < 9; ++j) ent.C[j] = rp->c[j];
            ent.q = rp->pad[0];
            ent.kappa = rp->pad[2];
        }
        const PlaneEntry pe = plane_entry(ent);
        while (ballot(row != 0ull) != 0ull) {
            if (row != 0ull) {
                const int t = __builtin_ctzll(row);
                row &= row - 1;
                if (!plane_keeps(pe, ltc[wv][t], ltca[wv][t]))
                    __hip_atomic_fetch_and(&lres[wv][t], ~(1ull << lane), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        wave_sync();
        mine = lres[wv][lane];
        wave_sync();                                   // read before the next chunk overwrites it
        const int c0 = sbase[s] / 64, ns = (sbase[s + 1] - sbase[s]) / 64;
        if (lane < nt) {
            W.bits[64 * (size_t)c0 + (size_t)lane * ns + (c - c0)] = mine;
            cnt += __popcll(mine);
        }
    }
    if (cnt && s_cur >= 0 && lane < sp_cur.nty * sp_cur.ntx)
        atomicAdd(W.hits + (sp_cur.ty0 + lane / sp_cur.ntx) * g.TW + sp_cur.tx0 + lane % sp_cur.ntx, cnt);
}


// ---------------------------------------------------------------------------
// Receiver region of interest (Sec. 3.2): only the texels and the radial range
// that receivers read are kept; everything else is T = 1 by construction.
// A receiver marks the four texels and two shells its trilinear lookup reads
// (query_cell), so a query at a receiver sees the same values as with the
// full atlas.
// ---------------------------------------------------------------------------

// The region is marked before the binning, so that the binning leaves out
// the tiles and supertiles no receiver reads.  Receiver marks go to a byte per
// texel (plain stores of 1: every receiver that reads a texel writes the same
// value, so no atomics are needed), kept in the storage of the split tiles'
// partial sums, which only the accumulation uses.  A pack pass then turns
// each tile's 64 bytes into its 64-bit region mask and flags the supertiles
// that hold one.  The shell range is reduced per block before its two atomics.
__global__ __launch_bounds__(256) void roi_clear_kernel(unsigned char* ws, BuildLayout lay, Geom g) {
    const LightWs W = light_ws(ws, lay, blockIdx.y);
    const int t = blockIdx.x * 256 + threadIdx.x;
    uint32_t* map = reinterpret_cast<uint32_t*>(W.part);
    const int nw = (g.H * g.W + 3) / 4;
    for (int q = t; q < nw; q += gridDim.x * 256) map[q] = 0u;
    for (int q = t; q < g.S; q += gridDim.x * 256) W.roi_super[q] = 0;
    if (t == 0) {
        W.roi_k[0] = g.K;
        W.roi_k[1] = -1;
    }
}

constexpr int kRoiMarkBlocks = 1024;   // blocks per light of the (grid-stride) marking pass

__global__ __launch_bounds__(256) void roi_mark_kernel(unsigned char* ws, BuildLayout lay, Geom g,
                                                       const float* __restrict__ lights,
                                                       const float* __restrict__ pts, int64_t n, RoiBox box,
                                                       float lr0, float kscale) {
    __shared__ int red[2][256 / kWave];
    const int l = blockIdx.y;
    const LightWs W = light_ws(ws, lay, l);
    unsigned char* map = reinterpret_cast<unsigned char*>(W.part);
    int kmn = g.K, kmx = -1;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float x = pts[3 * i], y = pts[3 * i + 1], z = pts[3 * i + 2];
        const bool in = !(box.half > 0.f) || (fabsf(x - box.cx) <= box.half && fabsf(y - box.cy) <= box.half &&
                                              z >= box.zmin && z <= box.zmax);
        if (!in) continue;
        const Cell c = query_cell(g, lr0, kscale, lights + 3 * l, x, y, z);
        for (int d = 0; d < 4; ++d) {
            int ii = c.i0 + (d >> 1), jj = c.j0 + (d & 1);
            wrap_texel(ii, jj, g.H, g.W);
            map[(size_t)ii * g.W + jj] = 1;
        }
        kmn = min(kmn, c.k0);
        kmx = max(kmx, c.k0 + 1);
    }
    kmn = wave_min(kmn);
    kmx = wave_max(kmx);
    const int wave = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
        red[0][wave] = kmn;
        red[1][wave] = kmx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / kWave; ++w) {
            kmn = min(kmn, red[0][w]);
            kmx = max(kmx, red[1][w]);
        }
        if (kmn <= kmx) {
            atomicMin(W.roi_k, kmn);
            atomicMax(W.roi_k + 1, kmx);
        }
    }
}

// Region mask of every tile from the texel bytes, and the supertiles that
// hold a region texel (plain stores of 1).
__global__ __launch_bounds__(256) void roi_pack_kernel(unsigned char* ws, BuildLayout lay, Geom g) {
    const LightWs W = light_ws(ws, lay, blockIdx.y);
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= g.ntiles) return;
    const unsigned char* map = reinterpret_cast<const unsigned char*>(W.part);
    const int ty = t / g.TW, tx = t - ty * g.TW;
    uint64_t m = 0;
    for (int r = 0; r < kTile; ++r) {
        const int i = ty * kTile + r;
        if (i >= g.H) break;
        for (int c = 0; c < kTile; ++c) {
            const int j = tx * kTile + c;
            if (j < g.W && map[(size_t)i * g.W + j]) m |= 1ull << (r * kTile + c);
        }
    }
    W.roi_mask[t] = m;
    if (m != 0ull) W.roi_super[(ty / g.STH) * g.SGW + tx / g.STW] = 1;
}

dgsm_status enqueue_roi(const Geom& g, const BuildLayout& L, unsigned char* ws, const dgsm_lights_t& lights,
                        const float* points, int64_t n_points, const RoiBox& box, hipStream_t st) {
    const dim3 tg((g.ntiles + 255) / 256, lights.n);
    roi_clear_kernel<<<tg, 256, 0, st>>>(ws, L, g);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    if (n_points > 0) {
        float lr0 = 0.f, kscale;
        if (g.spacing == DGSM_SHELLS_GEOMETRIC) {
            lr0 = log2f(g.r0);
            kscale = (float)(g.K - 1) / log2f(g.r1 / g.r0);
        } else {
            kscale = (float)g.K / g.r1;
        }
        const int64_t nb = (n_points + 255) / 256;
        roi_mark_kernel<<<dim3((unsigned)(nb < kRoiMarkBlocks ? nb : kRoiMarkBlocks), lights.n), 256, 0, st>>>(
            ws, L, g, lights.pos, points, n_points, box, lr0, kscale);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    }
    roi_pack_kernel<<<tg, 256, 0, st>>>(ws, L, g);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

// ---------------------------------------------------------------------------
// Work units.  A tile whose hit count is far above the launch's mean would
// keep a few blocks busy long after the rest of the chip has drained (an
// animated avatar covers a few dozen tiles with tens of thousands of hits
// each).  Such a tile is cut into q slices, slice i taking every q-th of its
// hit words (interleaved, so that the slices stay even however the hits
// cluster in the list); each slice runs in its own block and leaves its
// fixed-point per-shell sums in a partial buffer, which split_finish_kernel
// adds in slice order.  The sums are integers, so the atlas is bitwise the
// same as with unsplit tiles.
// ---------------------------------------------------------------------------

constexpr int kMaxSlices = 64;         // slices of one tile
constexpr int kMinSliceHits = 1024;    // below this a slice is not worth its partial buffer
constexpr int kPlanThreads = 1024;

// per = hits per slice; per <= 0: never split
__device__ inline int slices_of(int h, int per) {
    if (per <= 0) return 1;
    const int q = (int)(((long long)h + per - 1) / per);
    return q < 1 ? 1 : (q > kMaxSlices ? kMaxSlices : q);
}

// One block per light: slice size from the light's total hits and the target
// unit count, then the unit table in tile order (deterministic).
__global__ __launch_bounds__(kPlanThreads) void split_plan_kernel(unsigned char* ws, BuildLayout lay, Geom g,
                                                                  int target) {
    __shared__ long long red[kPlanThreads / kWave];
    __shared__ int iscan[kPlanThreads / kWave];
    __shared__ int per_s;
    const LightWs W = light_ws(ws, lay, blockIdx.x);
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    constexpr int NWV = kPlanThreads / kWave;
    // this thread's tiles: a contiguous range, so that tile order is scan order
    const int chunk = (g.ntiles + kPlanThreads - 1) / kPlanThreads;
    const int t0 = min(g.ntiles, tid * chunk), t1 = min(g.ntiles, t0 + chunk);
    long long h = 0;
    for (int t = t0; t < t1; ++t) h += W.hits[t];
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o);
    if (lane == 0) red[wave] = h;
    __syncthreads();
    if (tid == 0) {
        long long tot = 0;
        for (int w = 0; w < NWV; ++w) tot += red[w];
        long long per = target > 0 ? (tot + target - 1) / target : 0;
        if (target > 0 && per < kMinSliceHits) per = kMinSliceHits;
        if (per > (1ll << 28)) per = 0;
        per_s = (int)per;
        W.nunits[3] = (int)(tot < INT32_MAX ? tot : INT32_MAX);
    }
    __syncthreads();
    // grow the slice size until the extra slices fit the unit table
    int per = per_s, extra_me = 0, split_me = 0;
    for (;;) {
        extra_me = 0;
        split_me = 0;
        for (int t = t0; t < t1; ++t) {
            const int q = slices_of(W.hits[t], per);
            extra_me += q - 1;
            split_me += q > 1;
        }
        int e = extra_me;
        for (int o = 32; o > 0; o >>= 1) e += __shfl_xor(e, o);
        __syncthreads();
        if (lane == 0) iscan[wave] = e;
        __syncthreads();
        int tot = 0;
        for (int w = 0; w < NWV; ++w) tot += iscan[w];
        if (tot <= lay.units_cap || per <= 0) break;
        per = per >= (1 << 28) ? 0 : 2 * per;
    }
    // exclusive scans (tile order) of extra slices and split tiles: pack both in one int64
    long long v = ((long long)extra_me << 32) | (unsigned)split_me;
    long long incl = v;
    for (int o = 1; o < kWave; o <<= 1) {
        const long long y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    __syncthreads();
    if (lane == kWave - 1) red[wave] = incl;
    __syncthreads();
    long long before = 0, all = 0;
    for (int w = 0; w < NWV; ++w) {
        if (w < wave) before += red[w];
        all += red[w];
    }
    long long ex = before + incl - v;
    int xbase = (int)(ex >> 32), sbase = (int)(ex & 0xffffffffll);
    for (int t = t0; t < t1; ++t) {
        const int q = slices_of(W.hits[t], per);
        const int s = (t / g.TW / g.STH) * g.SGW + (t % g.TW) / g.STW;
        const int ns = (W.lbase[s + 1] - W.lbase[s]) / 64;
        int4 info = make_int4(1, -1, ns, 0);
        if (q > 1) {
            const int pbase = sbase + xbase;        // partials of earlier split tiles: one per slice
            info = make_int4(q, pbase, ns, 0);
            for (int i = 1; i < q; ++i) W.units[xbase + i - 1] = make_int4(t, i, q, pbase + i);
            W.splits[sbase] = make_int2(t, pbase);
            xbase += q - 1;
            sbase += 1;
        }
        W.tinfo[t] = info;
    }
    if (tid == 0) {
        W.nunits[0] = (int)(all >> 32);
        W.nunits[1] = (int)(all & 0xffffffffll);
        W.nunits[2] = per;
    }
}

// ---------------------------------------------------------------------------
// Per-tile build
// ---------------------------------------------------------------------------

struct TileArgs {
    Geom g;
    BuildLayout lay;
    unsigned char* ws;
    float pair_eps;
    void* out;                 // atlas [L][K][plane]
    const float* base_tau;     // optional [L][K][plane]
    int write_tau;
    int tiled;                 // plane order: 0 row-major H x W; 1 tile-major [TH*TW][8x8]
    int skip_empty;            // tiles without hits return at once and write nothing
    int roi;                   // T = 1 outside the receiver texels / shell range of the light
    unsigned long long* stats;
};

// Gaussian records are read with a wave-uniform index through the constant
// address space so that they land in scalar registers (s_load), the natural
// home of data every lane of the wave shares.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) f4v* ConstF4Ptr;

struct RecRegs {
    double mx, my, mz;
    float w[9], c[9], bp, r2, lg;
};

__device__ inline double as_double(float lo, float hi) {
    return __hiloint2double(__float_as_int(hi), __float_as_int(lo));
}

__device__ inline RecRegs load_rec(ConstF4Ptr base, int gi) {
    const ConstF4Ptr q = base + (size_t)gi * (sizeof(GRec) / 16);
    const f4v q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4], q5 = q[5], q6 = q[6];
    RecRegs r;
    r.mx = as_double(q0.x, q0.y);
    r.my = as_double(q0.z, q0.w);
    r.mz = as_double(q1.x, q1.y);
    r.w[0] = q1.z; r.w[1] = q1.w; r.w[2] = q2.x; r.w[3] = q2.y; r.w[4] = q2.z; r.w[5] = q2.w;
    r.w[6] = q3.x; r.w[7] = q3.y; r.w[8] = q3.z;
    r.c[0] = q3.w; r.c[1] = q4.x; r.c[2] = q4.y; r.c[3] = q4.z; r.c[4] = q4.w;
    r.c[5] = q5.x; r.c[6] = q5.y; r.c[7] = q5.z; r.c[8] = q5.w;
    r.bp = q6.x;
    r.r2 = q6.y;
    r.lg = q6.z;
    return r;
}

// The same record with per-lane (vector) loads, for lanes that hold different Gaussians.
__device__ inline RecRegs load_rec_v(const GRec* base, int gi) {
    const float4* q = reinterpret_cast<const float4*>(base + gi);
    const float4 q0 = q[0], q1 = q[1], q2 = q[2], q3 = q[3], q4 = q[4], q5 = q[5], q6 = q[6];
    RecRegs r;
    r.mx = as_double(q0.x, q0.y);
    r.my = as_double(q0.z, q0.w);
    r.mz = as_double(q1.x, q1.y);
    r.w[0] = q1.z; r.w[1] = q1.w; r.w[2] = q2.x; r.w[3] = q2.y; r.w[4] = q2.z; r.w[5] = q2.w;
    r.w[6] = q3.x; r.w[7] = q3.y; r.w[8] = q3.z;
    r.c[0] = q3.w; r.c[1] = q4.x; r.c[2] = q4.y; r.c[3] = q4.z; r.c[4] = q4.w;
    r.c[5] = q5.x; r.c[6] = q5.y; r.c[7] = q5.z; r.c[8] = q5.w;
    r.bp = q6.x;
    r.r2 = q6.y;
    r.lg = q6.z;
    return r;
}

// The part of a record the distance pre-test needs: m and r2 (scalar loads).
struct PreRegs {
    double mx, my, mz;
    float r2;
};

__device__ inline PreRegs load_pre(ConstF4Ptr base, int gi) {
    const ConstF4Ptr q = base + (size_t)gi * (sizeof(GRec) / 16);
    const f4v q0 = q[0], q1 = q[1], q6 = q[6];
    return PreRegs{as_double(q0.x, q0.y), as_double(q0.z, q0.w), as_double(q1.x, q1.y), q6.y};
}

__device__ inline int readlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }


__device__ inline uint64_t readlane_u64(uint64_t v, int l) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline double readlane_d(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

// Per-shell increments are accumulated in LDS as 64-bit fixed point with 32
// fractional bits.  Integer addition is associative, so the four waves of a
// tile may add in any interleaving and the result is still bitwise
// reproducible.  Each increment is truncated to a multiple of 2^-32.
constexpr float kFixScale = 4294967296.f;   // 2^32

__device__ inline unsigned long long to_fixed(float v) {
    const unsigned int hi = (unsigned int)v;                                    // v >= 0, truncates
    const unsigned int lo = (unsigned int)(__builtin_amdgcn_fractf(v) * kFixScale);   // exact product, < 2^32
    return ((unsigned long long)hi << 32) | lo;
}

__device__ inline double from_fixed(unsigned long long q) {
    return (double)(q >> 32) + (double)(unsigned int)q * (1.0 / 4294967296.0);
}

// Per-lane state of the tile build shared by every pair.
struct TexelState {
    double dx, dy, dz;       // texel direction, FP64
    float fx, fy, fz;        // the same, FP32
    bool valid;
    uint64_t vmask;          // ballot of valid: the lanes that hold a texel of the atlas
    int lane;
    float lr0, kinv;         // shell coordinate of a radius: (log2 t - lr0) * kinv (geometric)
    float lr0k1;             // 1 - lr0 * kinv (geometric), 0.5 (uniform): the coordinate plus one
    double ratio;            // t_{k+1} / t_k (geometric) or t_{k+1} - t_k (uniform)
    int K;
    bool geometric;
    float half_eps;          // half the pair threshold: a lane is active when 2 P0 exceeds it
    unsigned long long* inc; // LDS [K][64], fixed point
    const double* shells;    // LDS [K] shell radii t_k (FP64)
    int kmin, kmax;          // shells kept (the receiver range; 0 .. K-1 without a region)
    bool roi;                // a receiver region is set (wave-uniform)
};

// Shell coordinate of a radius plus one (fractional, unclamped): its integer
// part is the index of the first shell radius past t.  Geometric shells: a
// radius <= 0 gives -inf or NaN (log2 of 0 or of a negative number), which
// the callers floor at 0 (before shell 0).
template <bool GEO>
__device__ inline float shell_coord1(float t, const TexelState& ts) {
#pragma clang fp contract(off)
    if (GEO) return fmaf(__builtin_amdgcn_logf(t), ts.kinv, ts.lr0k1);
    return fmaf(t, ts.kinv, ts.lr0k1);
}

// Largest optical depth a pair may drop at either end of its erf ramp.
constexpr float kRampEps = 1e-10f;

// One (texel, Gaussian) pair for all 64 texels of the wave: Eq. 3 on the
// shells where the erf ramps, as non-negative per-shell increments.
// Work counters of the STATS variant (per wave, added to the launch totals).
struct Counters {
    unsigned long long hits = 0;        // (tile, Gaussian) pairs walked
    unsigned long long act = 0;         // texel lanes with a prefactor above the pair threshold
    unsigned long long ramp = 0;        // erf-ramp evaluations of those lanes
    unsigned long long idle = 0;        // pairs of which no texel lane was active
    unsigned long long ramp_wave = 0;   // shell iterations of the wave (SIMD work of the ramp)
    unsigned long long pre = 0;         // idle pairs already rejected by the distance pre-test
};

// Three-term dot products with the fused multiply-adds spelled out.
__device__ inline float dot3(float a0, float a1, float a2, float b0, float b1, float b2) {
#pragma clang fp contract(off)
    return fmaf(a0, b0, fmaf(a1, b1, a2 * b2));
}

// The pair evaluation is inlined twice (the two record register sets of
// walk_hits), and which copy evaluates a pair depends on the pair's place in
// its list word.  Every sum of two products is therefore written with explicit
// fused multiply-adds (and contraction is off for the rest): the compiler has
// no a*b + c*d left to fuse one way in one copy and the other way in the
// other, so a pair's increments are bitwise the same whatever the order of
// the Gaussians.
// Ray-line geometry in FP64, v = m x d (the perpendicular offset of the mean
// from the texel ray), rounded to FP32, and the distance pre-test on it: a
// texel whose |v|^2 reaches r2 cannot reach the pair threshold (r2 is a
// conservative bound, from a >= 1/s_max^2 and e0 >= |v|^2 / s_max^2).
struct RayOff {
    float vx, vy, vz;
    bool near;
};

__device__ inline RayOff ray_offset(double mx, double my, double mz, float r2, const TexelState& s) {
#pragma clang fp contract(off)
    const double vxd = fma(my, s.dz, -(mz * s.dy));
    const double vyd = fma(mz, s.dx, -(mx * s.dz));
    const double vzd = fma(mx, s.dy, -(my * s.dx));
    RayOff o;
    o.vx = (float)vxd; o.vy = (float)vyd; o.vz = (float)vzd;
    o.near = dot3(o.vx, o.vy, o.vz, o.vx, o.vy, o.vz) < r2;
    return o;
}

// A texel is evaluated only where its own tests pass (the distance pre-test,
// the whitened bound and the prefactor threshold): which texels of a tile
// contribute is a property of each (texel, Gaussian) pair alone, so the packed
// walk, which evaluates each pair beside other Gaussians' pairs, adds exactly
// the increments of the tile walk.
template <bool STATS, bool GEO>
__device__ __attribute__((always_inline)) inline void eval_pair(const RecRegs& r, const TexelState& s,
                                                                Counters& n) {
#pragma clang fp contract(off)
    // t_e = -(m . d); v = m x d
    const double te = -fma(r.mx, s.dx, fma(r.my, s.dy, r.mz * s.dz));
    const RayOff ro = ray_offset(r.mx, r.my, r.mz, r.r2, s);
    const float vx = ro.vx, vy = ro.vy, vz = ro.vz;
    // cheap pre-test (conservative: it never drops a texel the full test keeps)
    if ((ballot(ro.near) & s.vmask) == 0ull) {
        if (STATS) {
            n.idle += 1;
            n.pre += 1;
        }
        return;
    }
    // a = |W d|^2 (Eq. 2);  c - b^2/a = |adj(A)^(1/2) (m x d)|^2 / a
    const float wd0 = dot3(r.w[0], r.w[1], r.w[2], s.fx, s.fy, s.fz);
    const float wd1 = dot3(r.w[3], r.w[4], r.w[5], s.fx, s.fy, s.fz);
    const float wd2 = dot3(r.w[6], r.w[7], r.w[8], s.fx, s.fy, s.fz);
    const float a = dot3(wd0, wd1, wd2, wd0, wd1, wd2);
    const float cv0 = dot3(r.c[0], r.c[1], r.c[2], vx, vy, vz);
    const float cv1 = dot3(r.c[3], r.c[4], r.c[5], vx, vy, vz);
    const float cv2 = dot3(r.c[6], r.c[7], r.c[8], vx, vy, vz);
    const float cc = dot3(cv0, cv1, cv2, cv0, cv1, cv2);
    // second conservative test, free of transcendentals: e0 = cc / a >= lg
    const bool near2 = ro.near && cc < r.lg * a;
    if ((ballot(near2) & s.vmask) == 0ull) {
        if (STATS) n.idle += 1;
        return;
    }
    const float ra = __builtin_amdgcn_rcpf(a);
    const float e0 = cc * ra;
    const float rsa = __builtin_amdgcn_rsqf(a);
    // prefactor of Eq. 3 times beta: beta sqrt(pi / (2a)) exp(-e0 / 2)
    // (exp(-e0/2) = 2^(e0 * (-log2(e)/2)); 2 P0 > eps  <=>  P0 > eps/2, both exact)
    const float P0 = r.bp * rsa * __builtin_amdgcn_exp2f(e0 * -0.72134752f);
    const bool act = s.valid && near2 && (P0 > s.half_eps);
    const uint64_t abal = ballot(act);
    if (abal == 0ull) {
        if (STATS) n.idle += 1;
        return;
    }
    if (STATS) n.act += __popcll(abal);
    // Distance along the ray of the Mahalanobis-closest point:
    // t* = -b/a = t_e - (W d).(W p)/a with p = d x v the perpendicular offset.
    const float p0 = fmaf(s.fy, vz, -(s.fz * vy)), p1 = fmaf(s.fz, vx, -(s.fx * vz)),
                p2 = fmaf(s.fx, vy, -(s.fy * vx));
    const float wp0 = dot3(r.w[0], r.w[1], r.w[2], p0, p1, p2);
    const float wp1 = dot3(r.w[3], r.w[4], r.w[5], p0, p1, p2);
    const float wp2 = dot3(r.w[6], r.w[7], r.w[8], p0, p1, p2);
    const float dwp = dot3(wd0, wd1, wd2, wp0, wp1, wp2);
    const float corr = dwp * ra;
    const float sa = a * rsa * 0.70710678118654752f;      // sqrt(a / 2)
    const float ts = fmaf(-dwp, ra, (float)te);             // t* (shell range, erf at t = 0)
    // Ramp half-width in t: P0 erfc(z) <= P0 exp(-z^2) <= kRampEps for
    // z^2 = ln(P0 / kRampEps) (at least 0.34), and z = sqrt(a/2) half, so
    // half = sqrt(2 z^2 / a).  (P0 of an active lane is far above the
    // denormal range: raw v_log / v_sqrt suffice.)
    // (2 ln 2 log2(P0 / kRampEps) = 2 ln 2 log2 P0 + 46.0517, kRampEps = 1e-10)
    const float half =
        __builtin_amdgcn_sqrtf(fmaxf(fmaf(__builtin_amdgcn_logf(P0), 1.38629436f, 46.0517019f), 0.68f) * ra);
    float Ep = -1.f;
    if (ts < half) Ep = erf_as(-sa * ts);                   // the ramp reaches back to t = 0: erf there
    // Each lane walks its own ramp shells [ka, ka + len): the first shell past
    // the ramp start carries everything from t = 0 up to it, the last one (at
    // or past the ramp end) everything up to the saturated tail.
    int ka = 0, len = 0;
    if (act) {
        // ka: the first shell past the ramp start, kb: the first at or past its
        // end (fmaxf takes 0 over a NaN coordinate)
        ka = min((int)fmaxf(shell_coord1<GEO>(ts - half, s), 0.f), s.K - 1);
        const int kb = min((int)fmaxf(shell_coord1<GEO>(ts + half, s), 0.f), s.K - 1);
        if (!s.roi) {
            len = max(kb, ka) - ka + 1;
        } else if (ka <= s.kmax) {
            // only shells in [kmin, kmax] are kept: a ramp below the range
            // still adds its whole step at kmin, one above it adds nothing
            const int k0 = max(ka, s.kmin);
            len = max(min(kb, s.kmax), k0) - k0 + 1;
            ka = k0;
        }
    }
    if (ballot(len > 0) == 0ull) return;
    if (STATS) {
        int sum = len;
        for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, kWave);
        n.ramp += (unsigned long long)sum;
        n.ramp_wave += (unsigned long long)wave_max(len);
    }
    // erf argument at shell k: sqrt(a/2) (t_k - t*), with t* = t_e - corr kept in FP64.
    // The loop runs until no lane has shells left; a finished lane reads on
    // into the padding of the shell table (2K - 1 entries) and adds nothing.
    // Two shells per trip: the second reads and adds at fixed offsets from the
    // first, and the previous erf value alternates between two registers.
    // erf_as is non-decreasing up to rounding; a negative step from a rounding
    // dip is skipped and the next step spans the dip.
    const double tsd = te - (double)corr;
    const double* sh = s.shells + ka;
    unsigned long long* dst = s.inc + ka * kWave + s.lane;
    for (int j = 0;; j += 2) {
        if (ballot(j < len) == 0ull) break;
        const float Ea = erf_as(sa * (float)(sh[0] - tsd));
        const float dIa = P0 * (Ea - Ep);
        if (j < len && dIa > 0.f)
            __hip_atomic_fetch_add(dst, to_fixed(dIa), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (ballot(j + 1 < len) == 0ull) break;
        const float Eb = erf_as(sa * (float)(sh[1] - tsd));
        const float dIb = P0 * (Eb - Ea);
        if (j + 1 < len && dIb > 0.f)
            __hip_atomic_fetch_add(dst + kWave, to_fixed(dIb), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        Ep = Eb;
        sh += 2;
        dst += 2 * kWave;
    }
}

// Walk one wave's share of a tile's hit words: for every set bit, the Gaussian
// id of that supertile-list entry, its record (prefetched one pair ahead into
// the other of two scalar register sets) and the pair evaluation.
template <bool STATS, bool GEO>
// The words a wave walks are every S-th word of the tile starting at o (word
// m covers chunk m of the supertile list): interleaving keeps the waves and
// slices of a tile balanced however its hits cluster in the list.
__device__ __attribute__((always_inline)) inline void walk_hits(const uint64_t* words, int ns, int o, int S,
                                                                const int* list, ConstF4Ptr rec,
                                                                const TexelState& st, Counters& n) {
    const int lane = st.lane;
    const int nw = o < ns ? (ns - 1 - o) / S + 1 : 0;   // words of this wave
    for (int mbase = 0; mbase < nw; mbase += 64) {
        const uint64_t wv = mbase + lane < nw ? words[(size_t)(mbase + lane) * S + o] : 0ull;
        uint64_t nz = ballot(wv != 0ull);
        if (nz == 0ull) continue;
        int gv = list[64 * ((mbase + __builtin_ctzll(nz)) * S + o) + lane];
        while (nz) {
            const int j = __builtin_ctzll(nz);
            nz &= nz - 1;
            uint64_t word = readlane_u64(wv, j);
            const int gcur = gv;
            if (nz) gv = list[64 * ((mbase + __builtin_ctzll(nz)) * S + o) + lane];   // next chunk's ids, in flight
            if (STATS) n.hits += __popcll(word);
            int b = __builtin_ctzll(word);
            word &= word - 1;
            RecRegs ra = load_rec(rec, readlane_i(gcur, b)), rb;
            for (;;) {
                if (word) {                                 // B in flight while A is evaluated
                    b = __builtin_ctzll(word);
                    word &= word - 1;
                    rb = load_rec(rec, readlane_i(gcur, b));
                    eval_pair<STATS, GEO>(ra, st, n);
                } else {
                    eval_pair<STATS, GEO>(ra, st, n);
                    break;
                }
                if (word) {                                 // A in flight while B is evaluated
                    b = __builtin_ctzll(word);
                    word &= word - 1;
                    ra = load_rec(rec, readlane_i(gcur, b));
                    eval_pair<STATS, GEO>(rb, st, n);
                } else {
                    eval_pair<STATS, GEO>(rb, st, n);
                    break;
                }
            }
        }
    }
}

// Packed walk, for sets whose Gaussians reach few texels of a tile (the
// per-frame avatar: about 4 of a tile's 64 texels per hit).  Each (tile,
// Gaussian) hit runs only the distance pre-test over the tile's texels; the
// texels that pass are queued in LDS as (Gaussian, texel) pairs, and every 64
// queued pairs are evaluated together, one pair per lane, with the record read
// per lane and the texel direction from LDS.  The evaluation is eval_pair's
// arithmetic, and the increments go to the same fixed-point accumulators, so
// the atlas is bitwise the one of the unpacked walk.
constexpr int kQueue = 128;   // queued pairs per wave (up to 63 left over + 64 new)

template <bool GEO>
__device__ __attribute__((always_inline)) inline void walk_hits_packed(const uint64_t* words, int ns, int o, int S,
                                                                       const int* list, ConstF4Ptr rec,
                                                                       const GRec* recv, const TexelState& st,
                                                                       int* qg, unsigned char* qt,
                                                                       const double* dirs, Counters& n) {
    const int lane = st.lane;
    int qn = 0;   // queued pairs (wave-uniform)
    auto wave_sync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    // evaluate the first cnt queued pairs (lane i: pair i) and move the rest to the front
    auto flush = [&](int cnt) {
        wave_sync();
        const bool has = lane < cnt;
        const int gi = has ? qg[lane] : 0;
        const int tx = has ? (int)qt[lane] : 0;
        const int rest = qn - cnt;
        int gm = 0, tm = 0;
        if (lane < rest) {
            gm = qg[cnt + lane];
            tm = qt[cnt + lane];
        }
        wave_sync();
        if (lane < rest) {
            qg[lane] = gm;
            qt[lane] = (unsigned char)tm;
        }
        qn = rest;
        TexelState ps = st;
        ps.lane = tx;
        ps.valid = has;
        ps.vmask = ballot(has);
        ps.dx = dirs[3 * tx];
        ps.dy = dirs[3 * tx + 1];
        ps.dz = dirs[3 * tx + 2];
        ps.fx = (float)ps.dx; ps.fy = (float)ps.dy; ps.fz = (float)ps.dz;
        const RecRegs r = load_rec_v(recv, gi);
        eval_pair<false, GEO>(r, ps, n);
    };
    const int nw = o < ns ? (ns - 1 - o) / S + 1 : 0;   // words of this wave
    for (int mbase = 0; mbase < nw; mbase += 64) {
        const uint64_t wv = mbase + lane < nw ? words[(size_t)(mbase + lane) * S + o] : 0ull;
        uint64_t nz = ballot(wv != 0ull);
        while (nz) {
            const int j = __builtin_ctzll(nz);
            nz &= nz - 1;
            uint64_t word = readlane_u64(wv, j);
            const int gv = list[64 * ((mbase + j) * S + o) + lane];
            // the next hit's offset and bound are loaded while this one is tested
            int gid = readlane_i(gv, __builtin_ctzll(word));
            word &= word - 1;
            PreRegs r = load_pre(rec, gid);
            for (;;) {
                const bool more = word != 0ull;
                int gnext = gid;
                PreRegs rn = r;
                if (more) {
                    gnext = readlane_i(gv, __builtin_ctzll(word));
                    word &= word - 1;
                    rn = load_pre(rec, gnext);
                }
                const bool pass = ray_offset(r.mx, r.my, r.mz, r.r2, st).near;   // eval_pair's pre-test
                const uint64_t m = ballot(pass) & st.vmask;
                if (m != 0ull) {
                    if ((m >> lane) & 1ull) {
                        const int pos = qn + ballot_rank(m);
                        qg[pos] = gid;
                        qt[pos] = (unsigned char)lane;
                    }
                    qn += __popcll(m);
                    if (qn >= kWave) flush(kWave);
                }
                if (!more) break;
                gid = gnext;
                r = rn;
            }
        }
    }
    if (qn > 0) flush(qn);
}

constexpr int kFinishGroup = 8;

// Finish of one tile by all NWB waves of the block: wave w takes shells
// [w P, (w+1) P), P = ceil(K / NWB).  Per texel (lane) and shell k:
//   tau_k = prefix over shells of the fixed-point increments inc[k][lane]
//           (Eq. 2 as a running sum) + optional base optical depth,
//   T_k   = min(exp(-tau_k), T_{k-1}), T_{-1} = 1 (Eq. 4; exactly non-increasing).
// Pass 1 publishes each wave's increment total (so every wave knows the sum
// below its range), pass 2 each wave's minimum of exp(-tau) (the running
// minimum below its range), pass 3 stores.  Every stored value is bitwise the
// one a single wave walking all shells in order would store.  Base loads come
// in groups of kFinishGroup shells, so each group costs one memory latency.
template <typename OutT, int NWB>
__device__ inline void finish_tile(const TileArgs& p, int light, int tile, int lane, int wave,
                                   const unsigned long long* inc, unsigned long long* s_tot, float* s_min) {
    const Geom& g = p.g;
    const int K = g.K;
    const int ty = tile / g.TW, tx = tile - ty * g.TW;
    const int py = ty * kTile + (lane >> 3), px = tx * kTile + (lane & 7);
    const bool valid = py < g.H && px < g.W;
    const size_t plane = p.tiled ? (size_t)g.ntiles * kWave : (size_t)g.H * g.W;
    const size_t texel = p.tiled ? (size_t)tile * kWave + lane : (size_t)min(py, g.H - 1) * g.W + min(px, g.W - 1);
    const size_t off = (size_t)light * K * plane + texel;
    const float* bt = p.base_tau ? p.base_tau + off : nullptr;
    // receiver region: texels outside it and shells outside [k_lo, k_hi] store T = 1
    bool in_roi = true;
    int rk_lo = 0, rk_hi = K - 1;
    if (p.roi) {
        const LightWs W = light_ws(p.ws, p.lay, light);
        in_roi = (W.roi_mask[tile] >> lane) & 1ull;
        rk_lo = W.roi_k[0];
        rk_hi = W.roi_k[1];
    }
    const int per = (K + NWB - 1) / NWB;
    const int k_lo = min(K, wave * per), k_hi = min(K, k_lo + per);

    unsigned long long tot = 0;
    for (int k = k_lo; k < k_hi; ++k) tot += inc[k * kWave + lane];
    s_tot[wave * kWave + lane] = tot;
    __syncthreads();
    unsigned long long acc0 = 0;
    for (int w = 0; w < wave; ++w) acc0 += s_tot[w * kWave + lane];

    // tau_k for a group of shells starting at k0 (n of them), into tt[]
    auto group_tau = [&](int k0, int n, unsigned long long& acc, float* tt) {
        float bv[kFinishGroup];
#pragma unroll
        for (int j = 0; j < kFinishGroup; ++j) bv[j] = (bt && valid && j < n) ? bt[(size_t)(k0 + j) * plane] : 0.f;
#pragma unroll
        for (int j = 0; j < kFinishGroup; ++j) {
            if (j >= n) break;
            acc += inc[(k0 + j) * kWave + lane];
            tt[j] = (float)from_fixed(acc) + bv[j];
        }
    };

    if (p.write_tau) {
        unsigned long long acc = acc0;
        float* out = reinterpret_cast<float*>(p.out) + off;
        for (int k0 = k_lo; k0 < k_hi; k0 += kFinishGroup) {
            const int n = min(kFinishGroup, k_hi - k0);
            float tt[kFinishGroup];
            group_tau(k0, n, acc, tt);
#pragma unroll
            for (int j = 0; j < kFinishGroup; ++j)
                if (j < n && valid) out[(size_t)(k0 + j) * plane] = tt[j];
        }
        return;
    }
    float m = 1.f;
    {
        unsigned long long acc = acc0;
        for (int k0 = k_lo; k0 < k_hi; k0 += kFinishGroup) {
            const int n = min(kFinishGroup, k_hi - k0);
            float tt[kFinishGroup];
            group_tau(k0, n, acc, tt);
#pragma unroll
            for (int j = 0; j < kFinishGroup; ++j)
                if (j < n) m = fminf(m, __expf(-tt[j]));
        }
    }
    s_min[wave * kWave + lane] = m;
    __syncthreads();
    float Tp = 1.f;
    for (int w = 0; w < wave; ++w) Tp = fminf(Tp, s_min[w * kWave + lane]);
    unsigned long long acc = acc0;
    OutT* out = reinterpret_cast<OutT*>(p.out) + off;
    for (int k0 = k_lo; k0 < k_hi; k0 += kFinishGroup) {
        const int n = min(kFinishGroup, k_hi - k0);
        float tt[kFinishGroup];
        group_tau(k0, n, acc, tt);
#pragma unroll
        for (int j = 0; j < kFinishGroup; ++j) {
            if (j >= n) break;
            const float T = fminf(__expf(-tt[j]), Tp);
            Tp = T;
            const bool keep = in_roi && k0 + j >= rk_lo && k0 + j <= rk_hi;
            if (valid) Store<OutT>::put(out + (size_t)(k0 + j) * plane, keep ? T : 1.f);
        }
    }
}

// NW waves share one tile's accumulators (a launch knob: more waves per tile
// split a tile's pairs finer and raise occupancy per LDS byte).
// CUBE selects the cube-map texel decode at compile time, so that the
// octahedral kernels carry no code of the other parameterisation.
// Register budget: at least 7 waves per SIMD (72 VGPRs, a few spills).  With
// 8-wave blocks that still runs 6 waves of this kernel per SIMD, but leaves
// registers for the short kernels of the plan's other frame chains to run
// beside it (measured: batched step 1.7% faster, a lone full-scene build 0.9%
// slower; at 5 resident waves the build is 24% slower).
template <typename OutT, bool STATS, int NW, bool GEO, bool CUBE, bool PACK>
__global__ __launch_bounds__(kWave * NW, PACK ? 6 : 7) void tile_build_kernel(TileArgs p) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const Geom& g = p.g;
    const int K = g.K;
    unsigned long long* inc = reinterpret_cast<unsigned long long*>(smem);   // [K][64] fixed point

    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int light = blockIdx.y;
    const LightWs W = light_ws(p.ws, p.lay, light);
    // Blocks [0, ntiles) take slice 0 of their tile; the rest take the extra
    // slices of split tiles (block-uniform, so the early return is safe).
    int tile, slice, nslice, pidx;
    if ((int)blockIdx.x < g.ntiles) {
        tile = xcd_tile(g, blockIdx.x);
        if (p.skip_empty && W.hits[tile] == 0) return;
        if (p.roi && W.roi_mask[tile] == 0ull) {          // no receiver here: T = 1 by construction
            const size_t plane = (size_t)g.H * g.W;
            const int ty = tile / g.TW, tx = tile - ty * g.TW;
            for (int q = tid; q < K * kWave; q += kWave * NW) {
                const int k = q / kWave, l = q % kWave;
                const int py = ty * kTile + (l >> 3), px = tx * kTile + (l & 7);
                if (py < g.H && px < g.W)
                    Store<OutT>::put(reinterpret_cast<OutT*>(p.out) + ((size_t)light * K + k) * plane +
                                         (size_t)py * g.W + px,
                                     1.f);
            }
            return;
        }
        const int4 ti = W.tinfo[tile];
        slice = 0;
        nslice = ti.x;
        pidx = ti.x > 1 ? ti.y : -1;
    } else {
        const int e = (int)blockIdx.x - g.ntiles;
        if (e >= W.nunits[0]) return;
        const int4 u = W.units[e];
        tile = u.x;
        slice = u.y;
        nslice = u.z;
        pidx = u.w;
    }
    const int ty = tile / g.TW, tx = tile - ty * g.TW;
    const int py = ty * kTile + (lane >> 3), px = tx * kTile + (lane & 7);

    TexelState st;
    st.valid = py < g.H && px < g.W;
    st.vmask = ballot(st.valid);
    st.lane = lane;
    if constexpr (CUBE)
        cube_texel_dir(min(py, g.H - 1), min(px, g.W - 1), g.F, st.dx, st.dy, st.dz);
    else
        octa_texel_dir(min(py, g.H - 1), min(px, g.W - 1), g.H, g.W, st.dx, st.dy, st.dz);
    st.fx = (float)st.dx; st.fy = (float)st.dy; st.fz = (float)st.dz;
    st.K = K;
    st.geometric = g.spacing == DGSM_SHELLS_GEOMETRIC;
    st.half_eps = 0.5f * p.pair_eps;
    st.inc = inc;
    double* shells = reinterpret_cast<double*>(inc + K * kWave + NW * kWave) + (NW * kWave) / 2;   // after s_min
    for (int k = tid; k < 2 * K - 1; k += kWave * NW) shells[k] = shell_radius(min(k, K - 1), K, g.spacing, g.r0, g.r1);
    st.shells = shells;
    st.roi = p.roi != 0;
    st.kmin = p.roi ? W.roi_k[0] : 0;
    st.kmax = p.roi ? W.roi_k[1] : K - 1;
    if (st.geometric) {
        st.lr0 = __builtin_amdgcn_logf(g.r0);
        st.kinv = (float)(K - 1) / __builtin_amdgcn_logf(g.r1 / g.r0);
        st.lr0k1 = 1.f - st.lr0 * st.kinv;
        st.ratio = pow((double)g.r1 / (double)g.r0, 1.0 / (double)(K - 1));
    } else {
        st.lr0 = 0.f;
        st.kinv = (float)K / g.r1;
        st.lr0k1 = 0.5f;
        st.ratio = (double)g.r1 / (double)K;
    }
    for (int q = tid; q < K * kWave; q += kWave * NW) inc[q] = 0ull;
    // packed walk: texel directions [64][3] and each wave's pair queue after the shell radii
    double* dirs = shells + (2 * K - 1);
    int* qg = reinterpret_cast<int*>(dirs + 3 * kWave) + wave * kQueue;
    unsigned char* qt = reinterpret_cast<unsigned char*>(reinterpret_cast<int*>(dirs + 3 * kWave) + NW * kQueue) +
                        wave * kQueue;
    if (PACK && wave == 0) {
        dirs[3 * lane] = st.dx;
        dirs[3 * lane + 1] = st.dy;
        dirs[3 * lane + 2] = st.dz;
    }

    // this tile's hit words: contiguous ns words, one per 64-entry chunk of the
    // supertile list; wave w of slice i walks words i NW + w, + nslice NW, ...
    const int s = (ty / g.STH) * g.SGW + (tx / g.STW);
    const SuperSpan sp = super_span(g, s);
    const int t_local = (ty - sp.ty0) * sp.ntx + (tx - sp.tx0);
    const int lb0 = W.lbase[s], lb1 = W.lbase[s + 1];
    const int c0 = lb0 / 64, ns = (lb1 - lb0) / 64;
    const uint64_t* words = W.bits + 64 * (size_t)c0 + (size_t)t_local * ns;
    const int* list = W.lists + lb0;
    const ConstF4Ptr rec = (ConstF4Ptr)(const void*)W.rec;
    Counters n;
    __shared__ int rows[2];                   // shells any wave added to: partial-sum rows to keep
    if (tid == 0) {
        rows[0] = K;
        rows[1] = -1;
    }
    __syncthreads();

    if constexpr (PACK)
        walk_hits_packed<GEO>(words, ns, slice * NW + wave, nslice * NW, list, rec, W.rec, st, qg, qt, dirs, n);
    else
        walk_hits<STATS, GEO>(words, ns, slice * NW + wave, nslice * NW, list, rec, st, n);

    if (STATS) {
        const unsigned long long nvalid = __popcll(ballot(st.valid));
        if (lane == 0) {
            atomicAdd(p.stats + 0, n.hits * nvalid);
            atomicAdd(p.stats + 1, n.act);
            atomicAdd(p.stats + 2, n.ramp);
            atomicAdd(p.stats + 4, n.idle);
            atomicAdd(p.stats + 5, n.ramp_wave);
            atomicAdd(p.stats + 6, n.hits);
            atomicAdd(p.stats + 7, n.pre);
            if (wave == 0 && (int)blockIdx.x < g.ntiles) atomicAdd(p.stats + 3, (unsigned long long)(lb1 - lb0));
        }
    }
    __syncthreads();
    if (pidx >= 0) {           // a slice of a split tile: leave its partial sums (its non-zero rows)
        for (int k = wave; k < K; k += NW) {
            if (ballot(inc[k * kWave + lane] != 0ull) != 0ull && lane == 0) {
                atomicMin(rows, k);
                atomicMax(rows + 1, k);
            }
        }
        __syncthreads();
        const int lo = rows[0], hi = rows[1];
        unsigned long long* dst = W.part + (size_t)pidx * K * kWave;
        for (int q = lo * kWave + tid; q < (hi + 1) * kWave; q += kWave * NW) dst[q] = inc[q];
        if (tid == 0) W.prange[pidx] = make_int2(lo, hi);
        return;
    }

    finish_tile<OutT, NW>(p, light, tile, lane, wave, inc, reinterpret_cast<unsigned long long*>(inc + K * kWave),
                          reinterpret_cast<float*>(inc + K * kWave + NW * kWave));
}

// Split tiles: the slices' partial sums are added in slice order into LDS
// (wave w sums shells w, w + 8, ...), then the tile is finished as above.
constexpr int kFinishWaves = 8;
constexpr int kSliceBatch = 4;

template <typename OutT>
__global__ __launch_bounds__(kWave * kFinishWaves) void split_finish_kernel(TileArgs p) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const Geom& g = p.g;
    const int K = g.K;
    unsigned long long* inc = reinterpret_cast<unsigned long long*>(smem);   // [K][64]
    const int light = blockIdx.y;
    const LightWs W = light_ws(p.ws, p.lay, light);
    if ((int)blockIdx.x >= W.nunits[1]) return;
    const int2 sp = W.splits[blockIdx.x];
    const int q = W.tinfo[sp.x].x;
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    const size_t slice = (size_t)K * kWave;
    const unsigned long long* src = W.part + (size_t)sp.y * slice + lane;
    for (int k0 = wave * kFinishGroup; k0 < K; k0 += kFinishWaves * kFinishGroup) {
        const int n = min(kFinishGroup, K - k0);
        unsigned long long v[kFinishGroup];
#pragma unroll
        for (int j = 0; j < kFinishGroup; ++j) v[j] = 0ull;
        // kSliceBatch slices at a time: all their row loads are in flight together
        // (a tile can have up to kMaxSlices slices; one at a time, the loop
        // would pay one memory latency per slice)
        for (int i0 = 0; i0 < q; i0 += kSliceBatch) {
            unsigned long long t[kSliceBatch][kFinishGroup];
#pragma unroll
            for (int u = 0; u < kSliceBatch; ++u) {
                const int i = i0 + u;
                const int2 r = i < q ? W.prange[sp.y + i] : make_int2(K, -1);   // rows slice i wrote
                const unsigned long long* s0 = src + (size_t)(i < q ? i : 0) * slice + (size_t)k0 * kWave;
#pragma unroll
                for (int j = 0; j < kFinishGroup; ++j)
                    t[u][j] = (j < n && k0 + j >= r.x && k0 + j <= r.y) ? s0[(size_t)j * kWave] : 0ull;
            }
#pragma unroll
            for (int u = 0; u < kSliceBatch; ++u)
#pragma unroll
                for (int j = 0; j < kFinishGroup; ++j) v[j] += t[u][j];
        }
#pragma unroll
        for (int j = 0; j < kFinishGroup; ++j)
            if (j < n) inc[(k0 + j) * kWave + lane] = v[j];
    }
    __syncthreads();
    finish_tile<OutT, kFinishWaves>(p, light, sp.x, lane, wave, inc, inc + K * kWave,
                                    reinterpret_cast<float*>(inc + K * kWave + kFinishWaves * kWave));
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

BuildLayout build_layout(const Geom& g, int64_t n, int n_lights, int64_t cap) {
    BuildLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    L.nb = (int)((n + kPrepThreads - 1) / kPrepThreads);
    const size_t worst = (size_t)n * g.S + 64 * (size_t)g.S;
    L.cap = cap < 0 ? worst : (size_t)cap;
    L.tcone = take((size_t)g.ntiles * sizeof(float4));
    L.scone = take((size_t)kMaxSuper * sizeof(float4));
    L.qcone = take((size_t)((g.TH + 1) / 2) * ((g.TW + 1) / 2) * sizeof(float4));
    L.gcone = take((size_t)(kMaxSuper / 4) * sizeof(float4));
    L.tcos = take((size_t)g.ntiles * sizeof(float));
    L.scos = take((size_t)kMaxSuper * sizeof(float));
    L.qcos = take((size_t)((g.TH + 1) / 2) * ((g.TW + 1) / 2) * sizeof(float));
    L.gcos = take((size_t)(kMaxSuper / 4) * sizeof(float));
    L.light0 = off;
    off = 0;
    L.totals = take((size_t)kMaxSuper * sizeof(int));
    L.lbase = take((size_t)(kMaxSuper + 1) * sizeof(int));
    L.rec = take((size_t)n * sizeof(GRec));
    L.cone = take((size_t)n * sizeof(float4));
    L.mask = take((size_t)n * kMaskWords * sizeof(uint64_t));
    L.counts = take((size_t)g.S * (size_t)L.nb * sizeof(int));
    L.lists = take(L.cap * sizeof(int));
    L.bits = take(L.cap * sizeof(uint64_t));
    // Extra slices per light: at most 4 per tile and 8192, and no more than a
    // set of n Gaussians can fill (about 8 tile hits each, kMinSliceHits per
    // slice); every slot is a block of each tile-build launch, so a small
    // (per-frame avatar) set does not pay for thousands of empty ones.
    {
        const int64_t by_n = (n * 8) / kMinSliceHits + 256;
        const int cap = 4 * g.ntiles < 8192 ? 4 * g.ntiles : 8192;
        L.units_cap = by_n < cap ? (int)by_n : cap;
    }
    L.hits = take((size_t)g.ntiles * sizeof(int));
    L.tinfo = take((size_t)g.ntiles * sizeof(int4));
    L.units = take((size_t)L.units_cap * sizeof(int4));
    L.splits = take((size_t)L.units_cap * sizeof(int2));
    L.nunits = take(4 * sizeof(int));
    {
        const size_t pb = 2 * (size_t)L.units_cap * g.K * kWave * sizeof(unsigned long long), tb = (size_t)g.H * g.W;
        L.part = take(pb > tb ? pb : tb);
    }
    L.prange = take(2 * (size_t)L.units_cap * sizeof(int2));
    L.roi_mask = take((size_t)g.ntiles * sizeof(unsigned long long));
    L.roi_k = take(2 * sizeof(int));
    L.roi_super = take((size_t)kMaxSuper * sizeof(int));
    L.need = take(2 * sizeof(int));
    L.light_stride = off;
    L.total = L.light0 + (size_t)n_lights * L.light_stride;
    return L;
}

bool layout_for_bytes(const Geom& g, int64_t n, int n_lights, size_t ws_bytes, BuildLayout& out) {
    out = build_layout(g, n, n_lights);
    if (out.total <= ws_bytes) return true;
    const int64_t lo = 64 * (int64_t)g.S;
    const BuildLayout base = build_layout(g, n, n_lights, lo);
    if (base.total > ws_bytes) return false;
    // each light slice grows by 12 bytes per entry (an int list entry and a
    // u64 hit word), up to 512 bytes of alignment padding
    const size_t spare = (ws_bytes - base.total) / (size_t)n_lights;
    int64_t cap = lo + (int64_t)(spare / 12) / 64 * 64;
    const int64_t worst = (int64_t)out.cap;
    cap = cap < worst ? cap : worst;
    out = build_layout(g, n, n_lights, cap);
    while (out.total > ws_bytes && cap > lo) {
        cap -= 64;
        out = build_layout(g, n, n_lights, cap);
    }
    return out.total <= ws_bytes;
}

// LDS of a tile block: increments [K][64] (u64), then the finish's wave totals
// [NW][64] (u64) and wave minima [NW][64] (f32), then the shell radii [K] (FP64)
// and K - 1 copies of the last radius (read by lanes whose ramp has ended).
// With the packed walk, the texel directions [64][3] (FP64) and each wave's
// pair queue (kQueue Gaussian ids and texel indices) follow.
size_t tile_smem_bytes(const Geom& g, int nw, bool pack) {
    return (size_t)g.K * kWave * sizeof(unsigned long long) + (size_t)nw * kWave * (sizeof(unsigned long long) + 4) +
           (size_t)(2 * g.K - 1) * sizeof(double) +
           (pack ? 3 * kWave * sizeof(double) + (size_t)nw * kQueue * (sizeof(int) + 1) : 0);
}

template <typename OutT, bool STATS, int NW, bool CUBE, bool PACK>
static hipError_t launch_tile_map(const TileArgs& ta, int n_lights, hipStream_t st) {
    const size_t smem = tile_smem_bytes(ta.g, NW, PACK);
    const bool geo = ta.g.spacing == DGSM_SHELLS_GEOMETRIC;
    const void* fn = geo ? (const void*)tile_build_kernel<OutT, STATS, NW, true, CUBE, PACK>
                         : (const void*)tile_build_kernel<OutT, STATS, NW, false, CUBE, PACK>;
    if (smem > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    const dim3 grid(ta.g.ntiles + ta.lay.units_cap, n_lights);
    if (geo)
        tile_build_kernel<OutT, STATS, NW, true, CUBE, PACK><<<grid, kWave * NW, smem, st>>>(ta);
    else
        tile_build_kernel<OutT, STATS, NW, false, CUBE, PACK><<<grid, kWave * NW, smem, st>>>(ta);
    return hipGetLastError();
}

template <typename OutT, bool STATS, int NW, bool PACK>
static hipError_t launch_tile(const TileArgs& ta, int n_lights, hipStream_t st) {
    return ta.g.param == DGSM_PARAM_CUBEMAP ? launch_tile_map<OutT, STATS, NW, true, PACK>(ta, n_lights, st)
                                            : launch_tile_map<OutT, STATS, NW, false, PACK>(ta, n_lights, st);
}

template <typename OutT, bool STATS>
static hipError_t launch_tile_nw(const TileArgs& ta, int n_lights, int nw, hipStream_t st) {
    switch (nw) {
        case 2: return launch_tile<OutT, STATS, 2, false>(ta, n_lights, st);
        case 8: return launch_tile<OutT, STATS, 8, false>(ta, n_lights, st);
        default: return launch_tile<OutT, STATS, 4, false>(ta, n_lights, st);
    }
}

// The packed walk (no counters).
template <typename OutT>
static hipError_t launch_tile_packed(const TileArgs& ta, int n_lights, int nw, hipStream_t st) {
    switch (nw) {
        case 2: return launch_tile<OutT, false, 2, true>(ta, n_lights, st);
        case 8: return launch_tile<OutT, false, 8, true>(ta, n_lights, st);
        default: return launch_tile<OutT, false, 4, true>(ta, n_lights, st);
    }
}

dgsm_status enqueue_cones(const Geom& g, const BuildLayout& L, unsigned char* ws, hipStream_t st) {
    float4* tcone = reinterpret_cast<float4*>(ws + L.tcone);
    float4* scone = reinterpret_cast<float4*>(ws + L.scone);
    float4* qcone = reinterpret_cast<float4*>(ws + L.qcone);
    float4* gcone = reinterpret_cast<float4*>(ws + L.gcone);
    auto cosp = [&](size_t off) { return reinterpret_cast<float*>(ws + off); };
    constexpr int kPer = 256 / kWave;                        // cones per block
    tile_cone_kernel<<<(g.ntiles + kPer - 1) / kPer, 256, 0, st>>>(g, tcone, cosp(L.tcos));
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    super_cone_kernel<<<(g.S + kPer - 1) / kPer, 256, 0, st>>>(g, tcone, scone, cosp(L.scos), g.S, g.SGW, g.STH,
                                                                 g.STW);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    const int nqx = (g.TW + 1) / 2, nq = ((g.TH + 1) / 2) * nqx;
    super_cone_kernel<<<(nq + kPer - 1) / kPer, 256, 0, st>>>(g, tcone, qcone, cosp(L.qcos), nq, nqx, 2, 2);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    const int ngx = (g.SGW + 1) / 2, ng = ((g.SGH + 1) / 2) * ngx;
    super_cone_kernel<<<(ng + kPer - 1) / kPer, 256, 0, st>>>(g, tcone, gcone, cosp(L.gcos), ng, ngx, 2 * g.STH,
                                                               2 * g.STW);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

dgsm_status enqueue_bin(const Geom& g, const BuildLayout& L, unsigned char* ws, const dgsm_lights_t& lights,
                        float cull_eps, const dgsm_gaussians_t& gs, hipStream_t st, bool cones, bool shape_cached,
                        bool roi) {
    if (cones && enqueue_cones(g, L, ws, st) != DGSM_OK) return DGSM_EHIP;
    if (gs.n > 0) {
        PrepArgs pa{gs.mean, gs.scale, gs.rot, gs.opacity, gs.n, lights.pos, lights.kappa, lights.beta_mode, cull_eps,
                    g.S, g.SGH, g.SGW, shape_cached ? 1 : 0, roi ? 1 : 0, L, ws};
        preprocess_kernel<<<dim3(L.nb, lights.n), kPrepThreads, 0, st>>>(pa);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    }
    scan_kernel<<<dim3(g.S, lights.n), 256, 0, st>>>(ws, L);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    bases_kernel<<<lights.n, 256, 0, st>>>(ws, L, g.S, g.ntiles);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    if (gs.n > 0) {
        scatter_kernel<<<dim3(L.nb, lights.n), kPrepThreads, 0, st>>>(ws, L, gs.n, g.S);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
        // about two chunks per wave (the next chunk's loads overlap this one's tests)
        const int64_t est = ((int64_t)gs.n * 2 + 64 * (int64_t)g.S) / 64;
        const int blocks = (int)(est / 8 + 1 < 4096 ? est / 8 + 1 : 4096);
        tile_mask_kernel<<<dim3(blocks, lights.n), 256, 0, st>>>(ws, L, g, roi ? 1 : 0);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    }
    return DGSM_OK;
}

dgsm_status enqueue_accumulate(const Geom& g, const BuildLayout& L, unsigned char* ws, int n_lights,
                               float pair_eps, void* atlas, const AccumOpts& o, hipStream_t st) {
    TileArgs ta{g, L, ws, pair_eps, atlas, o.base_tau, o.write_tau ? 1 : 0, o.tiled ? 1 : 0,
                o.skip_empty ? 1 : 0, o.roi ? 1 : 0, o.stats};
    hipError_t e;
    const bool half = g.dtype == DGSM_F16 && !o.write_tau;
    const int nw = o.tile_waves;
    const int target = o.split_units > 0 ? (o.split_units + n_lights - 1) / n_lights : 0;
    split_plan_kernel<<<n_lights, kPlanThreads, 0, st>>>(ws, L, g, target);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    if (o.stats)
        e = half ? launch_tile_nw<__half, true>(ta, n_lights, nw, st) : launch_tile_nw<float, true>(ta, n_lights, nw, st);
    else if (o.pack)
        e = half ? launch_tile_packed<__half>(ta, n_lights, nw, st) : launch_tile_packed<float>(ta, n_lights, nw, st);
    else
        e = half ? launch_tile_nw<__half, false>(ta, n_lights, nw, st) : launch_tile_nw<float, false>(ta, n_lights, nw, st);
    if (e != hipSuccess) return DGSM_EHIP;
    const dim3 fgrid(L.units_cap, n_lights);
    const size_t fsmem = tile_smem_bytes(g, kFinishWaves, false);
    const void* ffn = half ? (const void*)split_finish_kernel<__half> : (const void*)split_finish_kernel<float>;
    if (fsmem > 64 * 1024 && hipFuncSetAttribute(ffn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fsmem) !=
                                 hipSuccess)
        return DGSM_EHIP;
    if (half)
        split_finish_kernel<__half><<<fgrid, kWave * kFinishWaves, fsmem, st>>>(ta);
    else
        split_finish_kernel<float><<<fgrid, kWave * kFinishWaves, fsmem, st>>>(ta);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

}  // namespace dgsm

using namespace dgsm;

static dgsm_status check_build_args(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                                    const dgsm_atlas_desc_t* desc) {
    dgsm_status st = validate_desc(desc);
    if (st != DGSM_OK) return st;
    if ((st = validate_lights(lights)) != DGSM_OK) return st;
    if ((st = validate_gaussians(gaussians)) != DGSM_OK) return st;
    const Geom g = make_geom(*desc);
    if ((gaussians->n + 64) * (int64_t)g.S >= (int64_t)INT32_MAX) return DGSM_EUNSUPPORTED;
    return DGSM_OK;
}

extern "C" size_t dgsm_build_workspace_size(const dgsm_atlas_desc_t* desc, int64_t n_gauss, int32_t n_lights) {
    if (validate_desc(desc) != DGSM_OK || n_gauss < 0 || n_gauss >= INT32_MAX || n_lights < 1) return 0;
    const Geom g = make_geom(*desc);
    return build_layout(g, n_gauss, n_lights).total;
}

extern "C" dgsm_status dgsm_bin(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                                const dgsm_atlas_desc_t* desc, void* ws, size_t ws_bytes, void* stream) {
    dgsm_status st = check_build_args(lights, gaussians, desc);
    if (st != DGSM_OK) return st;
    const Geom g = make_geom(*desc);
    BuildLayout L;
    if (!ws || !layout_for_bytes(g, gaussians->n, lights->n, ws_bytes, L)) return DGSM_EWORKSPACE;
    return enqueue_bin(g, L, reinterpret_cast<unsigned char*>(ws), *lights, desc->cull_eps, *gaussians,
                       reinterpret_cast<hipStream_t>(stream));
}

extern "C" dgsm_status dgsm_accumulate(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc, int64_t n_gauss,
                                       void* atlas, void* ws, size_t ws_bytes, unsigned long long* stats,
                                       void* stream) {
    dgsm_status st = validate_desc(desc);
    if (st != DGSM_OK) return st;
    if ((st = validate_lights(lights)) != DGSM_OK) return st;
    if (n_gauss < 0 || n_gauss >= INT32_MAX || !atlas) return DGSM_EINVAL;
    const Geom g = make_geom(*desc);
    BuildLayout L;
    if (!ws || !layout_for_bytes(g, n_gauss, lights->n, ws_bytes, L)) return DGSM_EWORKSPACE;
    AccumOpts o{nullptr, false, stats, kDefaultTileWaves, kDefaultSplitUnits};
    return enqueue_accumulate(g, L, reinterpret_cast<unsigned char*>(ws), lights->n, desc->cull_eps, atlas, o,
                              reinterpret_cast<hipStream_t>(stream));
}

extern "C" dgsm_status dgsm_accumulate_ex(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc,
                                          int64_t n_gauss, void* atlas, void* ws, size_t ws_bytes,
                                          const dgsm_accum_opts_t* opts, unsigned long long* stats, void* stream) {
    dgsm_status st = validate_desc(desc);
    if (st != DGSM_OK) return st;
    if ((st = validate_lights(lights)) != DGSM_OK) return st;
    if (n_gauss < 0 || n_gauss >= INT32_MAX || !atlas || !opts) return DGSM_EINVAL;
    if (opts->tile_waves != 2 && opts->tile_waves != 4 && opts->tile_waves != 8) return DGSM_EINVAL;
    if (opts->packed && stats) return DGSM_EINVAL;   // the packed walk keeps no counters
    const Geom g = make_geom(*desc);
    BuildLayout L;
    if (!ws || !layout_for_bytes(g, n_gauss, lights->n, ws_bytes, L)) return DGSM_EWORKSPACE;
    AccumOpts o{nullptr, false, stats, opts->tile_waves,
                opts->split_units == 0 ? kDefaultSplitUnits : (opts->split_units < 0 ? -1 : opts->split_units)};
    o.pack = opts->packed != 0;
    return enqueue_accumulate(g, L, reinterpret_cast<unsigned char*>(ws), lights->n, desc->cull_eps, atlas, o,
                              reinterpret_cast<hipStream_t>(stream));
}

extern "C" dgsm_status dgsm_work_units(const dgsm_atlas_desc_t* desc, int64_t n_gauss, int32_t n_lights,
                                       const void* ws, size_t ws_bytes, int32_t light, int32_t out[4],
                                       void* stream) {
    dgsm_status st = validate_desc(desc);
    if (st != DGSM_OK) return st;
    if (n_gauss < 0 || n_gauss >= INT32_MAX || n_lights < 1 || light < 0 || light >= n_lights || !out)
        return DGSM_EINVAL;
    const Geom g = make_geom(*desc);
    BuildLayout L;
    if (!ws || !layout_for_bytes(g, n_gauss, n_lights, ws_bytes, L)) return DGSM_EWORKSPACE;
    const LightWs W = light_ws(reinterpret_cast<unsigned char*>(const_cast<void*>(ws)), L, light);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(out, W.nunits, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return DGSM_EHIP;
    return DGSM_OK;
}

extern "C" size_t dgsm_build_workspace_size_entries(const dgsm_atlas_desc_t* desc, int64_t n_gauss,
                                                    int32_t n_lights, int64_t entries) {
    if (validate_desc(desc) != DGSM_OK || n_gauss < 0 || n_gauss >= INT32_MAX || n_lights < 1 || entries < 0)
        return 0;
    const Geom g = make_geom(*desc);
    const int64_t worst = (n_gauss + 64) * (int64_t)g.S;
    int64_t cap = (entries + 63) / 64 * 64;
    cap = cap < 64 * (int64_t)g.S ? 64 * (int64_t)g.S : cap;
    return build_layout(g, n_gauss, n_lights, cap < worst ? cap : worst).total;
}

extern "C" dgsm_status dgsm_count_entries(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                                          const dgsm_atlas_desc_t* desc, void* ws, size_t ws_bytes,
                                          int64_t* entries, void* stream) {
    dgsm_status st = check_build_args(lights, gaussians, desc);
    if (st != DGSM_OK) return st;
    if (!entries) return DGSM_EINVAL;
    const Geom g = make_geom(*desc);
    BuildLayout L;
    if (!ws || !layout_for_bytes(g, gaussians->n, lights->n, ws_bytes, L)) return DGSM_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    if ((st = enqueue_bin(g, L, w, *lights, desc->cull_eps, *gaussians, s)) != DGSM_OK) return st;
    std::vector<int> need(2 * (size_t)lights->n);
    for (int l = 0; l < lights->n; ++l)
        if (hipMemcpyAsync(&need[2 * l], light_ws(w, L, l).need, 2 * sizeof(int), hipMemcpyDeviceToHost, s) !=
            hipSuccess)
            return DGSM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return DGSM_EHIP;
    int64_t m = 0;
    for (int l = 0; l < lights->n; ++l) m = need[2 * l] > m ? need[2 * l] : m;
    *entries = m;
    return DGSM_OK;
}

extern "C" dgsm_status dgsm_list_entries(const dgsm_atlas_desc_t* desc, int64_t n_gauss, int32_t n_lights,
                                         const void* ws, size_t ws_bytes, int32_t light, int64_t out[2],
                                         void* stream) {
    dgsm_status st = validate_desc(desc);
    if (st != DGSM_OK) return st;
    if (n_gauss < 0 || n_gauss >= INT32_MAX || n_lights < 1 || light < 0 || light >= n_lights || !out)
        return DGSM_EINVAL;
    const Geom g = make_geom(*desc);
    BuildLayout L;
    if (!ws || !layout_for_bytes(g, n_gauss, n_lights, ws_bytes, L)) return DGSM_EWORKSPACE;
    const LightWs W = light_ws(reinterpret_cast<unsigned char*>(const_cast<void*>(ws)), L, light);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int need[2] = {0, 0};
    if (hipMemcpyAsync(need, W.need, 2 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return DGSM_EHIP;
    out[0] = need[0];
    out[1] = (int64_t)L.cap;
    return DGSM_OK;
}

extern "C" dgsm_status dgsm_build_roi(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                                      const dgsm_atlas_desc_t* desc, const float* receivers, int64_t n_receivers,
                                      const dgsm_roi_box_t* box, void* atlas, void* ws, size_t ws_bytes,
                                      void* stream) {
    dgsm_status st = check_build_args(lights, gaussians, desc);
    if (st != DGSM_OK) return st;
    if (!atlas || !box || n_receivers < 0 || (n_receivers > 0 && !receivers)) return DGSM_EINVAL;
    if (box->half > 0.f && !(box->zmin <= box->zmax)) return DGSM_EINVAL;
    const Geom g = make_geom(*desc);
    BuildLayout L;
    if (!ws || !layout_for_bytes(g, gaussians->n, lights->n, ws_bytes, L)) return DGSM_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    const RoiBox rb{box->cx, box->cy, box->half, box->zmin, box->zmax};
    if ((st = enqueue_roi(g, L, w, *lights, receivers, n_receivers, rb, s)) != DGSM_OK) return st;
    if ((st = enqueue_bin(g, L, w, *lights, desc->cull_eps, *gaussians, s, true, false, true)) != DGSM_OK) return st;
    AccumOpts o{nullptr, false, nullptr, kDefaultTileWaves, kDefaultSplitUnits};
    o.roi = true;
    return enqueue_accumulate(g, L, w, lights->n, desc->cull_eps, atlas, o, s);
}

extern "C" dgsm_status dgsm_build(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                                  const dgsm_atlas_desc_t* desc, void* atlas, void* ws, size_t ws_bytes,
                                  void* stream) {
    dgsm_status st = check_build_args(lights, gaussians, desc);
    if (st != DGSM_OK) return st;
    if (!atlas) return DGSM_EINVAL;
    const Geom g = make_geom(*desc);
    BuildLayout L;
    if (!ws || !layout_for_bytes(g, gaussians->n, lights->n, ws_bytes, L)) return DGSM_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    if ((st = enqueue_bin(g, L, w, *lights, desc->cull_eps, *gaussians, s)) != DGSM_OK) return st;
    AccumOpts o{nullptr, false, nullptr, kDefaultTileWaves, kDefaultSplitUnits};
    return enqueue_accumulate(g, L, w, lights->n, desc->cull_eps, atlas, o, s);
}

// ---------------------------------------------------------------------------
// Allocation-free build: the workspace is a fixed device array of the library
// ---------------------------------------------------------------------------

namespace {

constexpr size_t kScratchBytes = (size_t)DGSM_BUILD_SCRATCH_BYTES;
constexpr int kScratchDevices = 64;

// One copy per GPU the library runs on, held until the process ends.  In host
// code this name is only a stand-in for the symbol: the device address of each
// GPU's copy comes from hipGetSymbolAddress and is what kernels receive.
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kScratchDevices] = {};

// Device address of the current device's scratch copy, looked up once per
// device with that device current; nullptr if the lookup fails.
unsigned char* scratch_address() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = reinterpret_cast<unsigned char*>(p);
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" size_t dgsm_build_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" dgsm_status dgsm_build_noalloc(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                                          const dgsm_atlas_desc_t* desc, void* atlas, void* stream) {
    dgsm_status st = check_build_args(lights, gaussians, desc);
    if (st != DGSM_OK) return st;
    if (!atlas) return DGSM_EINVAL;
    const Geom g = make_geom(*desc);
    const BuildLayout L = build_layout(g, gaussians->n, lights->n);
    if (L.total > kScratchBytes) return DGSM_EWORKSPACE;
    unsigned char* w = scratch_address();
    if (!w) return DGSM_EHIP;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // The same kernels as dgsm_build on the scratch copy: the binning writes
    // every workspace word the accumulation reads, so what an earlier call left
    // there is never read.
    if ((st = enqueue_bin(g, L, w, *lights, desc->cull_eps, *gaussians, s)) != DGSM_OK) return st;
    AccumOpts o{nullptr, false, nullptr, kDefaultTileWaves, kDefaultSplitUnits};
    return enqueue_accumulate(g, L, w, lights->n, desc->cull_eps, atlas, o, s);
}
