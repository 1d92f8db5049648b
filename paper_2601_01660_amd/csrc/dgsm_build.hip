// DGSM build on gfx950: light-space binning + per-tile closed-form optical depth.
//
// Pipeline for one light (Sec. 3.2):
//   tile_cone_kernel / super_cone_kernel  bounding cones of the texel-centre
//        directions of every 8x8 atlas tile and of every supertile
//   preprocess_kernel  per Gaussian: whitening rows, beta (Eq. 5), light-to-mean
//        offset in FP64, a rigorous culling cone, the 64-bit supertile mask,
//        per-block supertile counts
//   scan_kernel        exclusive scan of those counts per supertile
//   scatter_kernel     stable compaction of Gaussian ids into supertile lists
//                      (ascending id within a list: the summation order is fixed)
//   tile_build_kernel  one wave per tile: filter the supertile list against the
//        tile cone, then for every (texel, Gaussian) pair evaluate Eq. 3 on the
//        shells where the erf ramps, add the per-shell increments in LDS,
//        prefix over shells, T = exp(-tau) (Eq. 4), shell-major store.

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"

#include <math.h>

namespace dgsm {

// ---------------------------------------------------------------------------
// Tile and supertile cones
// ---------------------------------------------------------------------------

__device__ inline float inflate_sh(double sh) {
    double v = sh * (1.0 + 1e-5) + 1e-6;
    return (float)(v > 1.0 ? 1.0 : v);
}

__global__ __launch_bounds__(64) void tile_cone_kernel(Geom g, float4* __restrict__ tcone) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= g.ntiles) return;
    const int ty = t / g.TW, tx = t - ty * g.TW;
    const int i1 = min(ty * kTile + kTile, g.H), j1 = min(tx * kTile + kTile, g.W);
    double sx = 0, sy = 0, sz = 0;
    for (int i = ty * kTile; i < i1; ++i)
        for (int j = tx * kTile; j < j1; ++j) {
            double x, y, z;
            texel_dir(i, j, g.H, g.W, x, y, z);
            sx += x; sy += y; sz += z;
        }
    const double nrm = sqrt(sx * sx + sy * sy + sz * sz);
    sx /= nrm; sy /= nrm; sz /= nrm;
    double ch = 0;
    for (int i = ty * kTile; i < i1; ++i)
        for (int j = tx * kTile; j < j1; ++j) {
            double x, y, z;
            texel_dir(i, j, g.H, g.W, x, y, z);
            const double c2 = (x - sx) * (x - sx) + (y - sy) * (y - sy) + (z - sz) * (z - sz);
            ch = fmax(ch, c2);
        }
    tcone[t] = make_float4((float)sx, (float)sy, (float)sz, inflate_sh(0.5 * sqrt(ch)));
}

// A supertile cone bounds the cones of its tiles: half-angle = max over tiles
// of (angle to the tile axis + tile half-angle).
__global__ __launch_bounds__(64) void super_cone_kernel(Geom g, const float4* __restrict__ tcone,
                                                        float4* __restrict__ scone) {
    const int s = threadIdx.x;
    if (s >= g.S) return;
    const int sy = s / g.SGW, sx = s - sy * g.SGW;
    const int ty0 = sy * g.STH, ty1 = min(ty0 + g.STH, g.TH);
    const int tx0 = sx * g.STW, tx1 = min(tx0 + g.STW, g.TW);
    double ax = 0, ay = 0, az = 0;
    for (int ty = ty0; ty < ty1; ++ty)
        for (int tx = tx0; tx < tx1; ++tx) {
            const float4 c = tcone[ty * g.TW + tx];
            ax += c.x; ay += c.y; az += c.z;
        }
    const double nrm = sqrt(ax * ax + ay * ay + az * az);
    ax /= nrm; ay /= nrm; az /= nrm;
    double half = 0;
    for (int ty = ty0; ty < ty1; ++ty)
        for (int tx = tx0; tx < tx1; ++tx) {
            const float4 c = tcone[ty * g.TW + tx];
            const double ch = sqrt((c.x - ax) * (c.x - ax) + (c.y - ay) * (c.y - ay) + (c.z - az) * (c.z - az));
            const double ang = 2.0 * asin(fmin(1.0, 0.5 * ch)) + 2.0 * asin(fmin(1.0, (double)c.w));
            half = fmax(half, ang);
        }
    half = fmin(half, M_PI);
    scone[s] = make_float4((float)ax, (float)ay, (float)az, inflate_sh(sin(0.5 * half)));
}

// ---------------------------------------------------------------------------
// Per-Gaussian preprocess + supertile mask + per-block counts
// ---------------------------------------------------------------------------

// Pointers into one light's slice of the workspace.
struct LightWs {
    int* totals;       // [64] list length per supertile
    GRec* rec;         // [n]
    float4* cone;      // [n]
    uint64_t* mask;    // [n]
    int* counts;       // [S][nb] per-block counts, scanned in place
    int* lists;        // [n * S] supertile lists, concatenated in supertile order
};

__host__ __device__ inline LightWs light_ws(unsigned char* ws, const BuildLayout& L, int l) {
    unsigned char* b = ws + L.light0 + (size_t)l * L.light_stride;
    return LightWs{reinterpret_cast<int*>(b + L.totals), reinterpret_cast<GRec*>(b + L.rec),
                   reinterpret_cast<float4*>(b + L.cone), reinterpret_cast<uint64_t*>(b + L.mask),
                   reinterpret_cast<int*>(b + L.counts), reinterpret_cast<int*>(b + L.lists)};
}

struct PrepArgs {
    const float* mean;
    const float* scale;
    const float* rot;
    const float* opacity;
    int64_t n;
    const float* lights;   // device [L][3]
    float kappa;
    float eps;             // culling budget (0: no culling)
    int S;
    BuildLayout lay;
    unsigned char* ws;
};

__global__ __launch_bounds__(kPrepThreads) void preprocess_kernel(PrepArgs a) {
    __shared__ int wcnt[kPrepThreads / kWave][kMaxSuper];
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int l = blockIdx.y;
    const LightWs W = light_ws(a.ws, a.lay, l);
    const float4* scone = reinterpret_cast<const float4*>(a.ws + a.lay.scone);
    const float* light = a.lights + 3 * l;
    const int64_t i = (int64_t)blockIdx.x * kPrepThreads + tid;
    const bool in = i < a.n;
    float4 cone = make_float4(0.f, 0.f, 1.f, -1.f);
    if (in) {
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
        const double amp = (double)a.kappa * tau_star * sqrt(tr / 3.0);   // beta sqrt(2 pi)
        r.bp = (float)(0.5 * amp);                                        // beta sqrt(pi/2)
        r.mx = (double)light[0] - (double)a.mean[3 * i];
        r.my = (double)light[1] - (double)a.mean[3 * i + 1];
        r.mz = (double)light[2] - (double)a.mean[3 * i + 2];
        r.pad[0] = r.pad[1] = r.pad[2] = 0.f;
        W.rec[i] = r;

        // Culling cone.  Along any ray the contribution is at most
        // U exp(-h^2 / (2 s_max^2)), U = kappa tau* sqrt(tr A / 3) s_max, with h
        // the distance from mu to the ray (D for rays pointing away).  So it is
        // below eps outside the cone sin(theta) <= (s_max / D) sqrt(2 ln(U / eps)).
        const double smax = fmax(s[0], fmax(s[1], s[2]));
        const double D = sqrt(r.mx * r.mx + r.my * r.my + r.mz * r.mz);
        const double U = amp * smax;
        if (!(alpha > 0.0) || !(U > (double)a.eps)) {
            cone.w = -1.f;                               // contributes nothing
        } else {
            double shalf = 1.0;                          // global: every direction
            if (a.eps > 0.f && D > 0.0) {
                const double sig = smax / D * sqrt(2.0 * log(U / (double)a.eps));
                if (sig < 1.0) shalf = sin(0.5 * asin(sig));
            }
            const double gx = D > 0 ? -r.mx / D : 0.0, gy = D > 0 ? -r.my / D : 0.0,
                         gz = D > 0 ? -r.mz / D : 1.0;
            cone = make_float4((float)gx, (float)gy, (float)gz, inflate_sh(shalf));
        }
        W.cone[i] = cone;
    }
    uint64_t m = 0;
    for (int s = 0; s < a.S; ++s) {
        const bool b = in && cones_touch(cone, scone[s]);
        m |= (uint64_t)b << s;
        const uint64_t bal = __ballot(b);
        if (lane == 0) wcnt[w][s] = __popcll(bal);
    }
    if (in) W.mask[i] = m;
    __syncthreads();
    if (tid < a.S) {
        int c = 0;
        for (int ww = 0; ww < kPrepThreads / kWave; ++ww) c += wcnt[ww][tid];
        W.counts[(size_t)tid * a.lay.nb + blockIdx.x] = c;
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of the per-block counts, one workgroup per (supertile, light)
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void scan_kernel(unsigned char* ws, BuildLayout lay) {
    __shared__ int wsum[4];
    const LightWs W = light_ws(ws, lay, blockIdx.y);
    const int s = blockIdx.x, tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const int nb = lay.nb;
    int* c = W.counts + (size_t)s * nb;
    int carry = 0;
    for (int base = 0; base < nb; base += 256) {
        const int idx = base + tid;
        const int v = idx < nb ? c[idx] : 0;
        int x = v;   // inclusive wave scan
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int y = __shfl_up(x, o, kWave);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) wsum[w] = x;
        __syncthreads();
        int pre = carry;
        for (int ww = 0; ww < w; ++ww) pre += wsum[ww];
        if (idx < nb) c[idx] = pre + x - v;
        carry += wsum[0] + wsum[1] + wsum[2] + wsum[3];
        __syncthreads();
    }
    if (tid == 0) W.totals[s] = carry;
}

// ---------------------------------------------------------------------------
// Stable scatter of Gaussian ids into the supertile lists
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kPrepThreads) void scatter_kernel(unsigned char* ws, BuildLayout lay, int64_t n,
                                                             int S) {
    __shared__ int base_s[kMaxSuper];
    __shared__ int wcnt[kPrepThreads / kWave][kMaxSuper];
    const LightWs W = light_ws(ws, lay, blockIdx.y);
    const int tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    if (tid < S) {
        int b = 0;
        for (int q = 0; q < tid; ++q) b += W.totals[q];
        base_s[tid] = b + W.counts[(size_t)tid * lay.nb + blockIdx.x];
    }
    const int64_t i = (int64_t)blockIdx.x * kPrepThreads + tid;
    const uint64_t m = i < n ? W.mask[i] : 0ull;
    for (int s = 0; s < S; ++s) {
        const uint64_t bal = __ballot((m >> s) & 1ull);
        if (lane == 0) wcnt[w][s] = __popcll(bal);
    }
    __syncthreads();
    for (int s = 0; s < S; ++s) {
        const bool b = (m >> s) & 1ull;
        const uint64_t bal = __ballot(b);
        if (b) {
            int off = base_s[s];
            for (int ww = 0; ww < w; ++ww) off += wcnt[ww][s];
            W.lists[off + ballot_rank(bal)] = (int)i;
        }
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
    void* out;                 // atlas [L][K][H][W]
    const float* base_tau;     // optional [L][K][H][W]
    int write_tau;
    unsigned long long* stats;
};

// Gaussian records are read with a wave-uniform index through the constant
// address space so that they land in scalar registers (s_load), the natural
// home of data every lane of the wave shares.
typedef float f4v __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) f4v* ConstF4Ptr;

struct RecRegs {
    double mx, my, mz;
    float w[9], c[9], bp;
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
    return r;
}

// Shell index of a radius (fractional, unclamped); -1 for t <= 0.
__device__ inline float shell_index(float t, const Geom& g, float lr0, float inv) {
    if (g.spacing == DGSM_SHELLS_GEOMETRIC) return t > 0.f ? (__log2f(t) - lr0) * inv : -1.f;
    return t * inv - 0.5f;
}

template <typename OutT, bool STATS>
__global__ __launch_bounds__(kWave) void tile_build_kernel(TileArgs p) {
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    const Geom& g = p.g;
    const int K = g.K;
    float* inc = reinterpret_cast<float*>(smem);                   // [K][64] per-shell increments
    float2* shell = reinterpret_cast<float2*>(inc + (size_t)K * kWave);   // [K] t_k as hi + lo
    int* hits = reinterpret_cast<int*>(shell + K);                  // [64]

    const int lane = threadIdx.x;
    const int tile = blockIdx.x;
    const int light = blockIdx.y;
    const LightWs W = light_ws(p.ws, p.lay, light);
    const float4* tcone = reinterpret_cast<const float4*>(p.ws + p.lay.tcone);
    const int ty = tile / g.TW, tx = tile - ty * g.TW;
    const int py = ty * kTile + (lane >> 3), px = tx * kTile + (lane & 7);
    const bool valid = py < g.H && px < g.W;
    double dx, dy, dz;
    texel_dir(min(py, g.H - 1), min(px, g.W - 1), g.H, g.W, dx, dy, dz);
    const float fx = (float)dx, fy = (float)dy, fz = (float)dz;

    for (int k = lane; k < K; k += kWave) {
        const double t = shell_radius(k, K, g.spacing, g.r0, g.r1);
        const float hi = (float)t;
        shell[k] = make_float2(hi, (float)(t - (double)hi));
    }
    for (int q = lane; q < K * kWave; q += kWave) inc[q] = 0.f;
    float lr0, inv;
    if (g.spacing == DGSM_SHELLS_GEOMETRIC) {
        lr0 = __log2f(g.r0);
        inv = (float)(K - 1) / __log2f(g.r1 / g.r0);
    } else {
        lr0 = 0.f;
        inv = (float)K / g.r1;
    }

    const int s = (ty / g.STH) * g.SGW + (tx / g.STW);
    int base = 0;
    for (int q = 0; q < s; ++q) base += W.totals[q];
    const int cnt = W.totals[s];
    const float4 tc = tcone[tile];
    const ConstF4Ptr rec = (ConstF4Ptr)(const void*)W.rec;
    unsigned long long n_hits = 0, n_act = 0, n_ramp = 0;
    __syncthreads();

    for (int c0 = 0; c0 < cnt; c0 += kWave) {
        const int idx = c0 + lane;
        bool hit = false;
        int gid = 0;
        if (idx < cnt) {
            gid = W.lists[base + idx];
            hit = cones_touch(W.cone[gid], tc);
        }
        const uint64_t bal = __ballot(hit);
        if (hit) hits[ballot_rank(bal)] = gid;
        const int nh = __popcll(bal);
        if (STATS) n_hits += nh;
        __syncthreads();
        for (int h = 0; h < nh; ++h) {
            const int gi = __builtin_amdgcn_readfirstlane(hits[h]);
            const RecRegs r = load_rec(rec, gi);
            // Ray-line geometry in FP64: v = m x d, t_e = -(m . d).
            const double vxd = r.my * dz - r.mz * dy;
            const double vyd = r.mz * dx - r.mx * dz;
            const double vzd = r.mx * dy - r.my * dx;
            const double te = -(r.mx * dx + r.my * dy + r.mz * dz);
            const float vx = (float)vxd, vy = (float)vyd, vz = (float)vzd;
            // a = |W d|^2 (Eq. 2);  c - b^2/a = |adj(A)^(1/2) (m x d)|^2 / a
            const float wd0 = r.w[0] * fx + r.w[1] * fy + r.w[2] * fz;
            const float wd1 = r.w[3] * fx + r.w[4] * fy + r.w[5] * fz;
            const float wd2 = r.w[6] * fx + r.w[7] * fy + r.w[8] * fz;
            const float a = wd0 * wd0 + wd1 * wd1 + wd2 * wd2;
            const float cv0 = r.c[0] * vx + r.c[1] * vy + r.c[2] * vz;
            const float cv1 = r.c[3] * vx + r.c[4] * vy + r.c[5] * vz;
            const float cv2 = r.c[6] * vx + r.c[7] * vy + r.c[8] * vz;
            const float ra = __builtin_amdgcn_rcpf(a);
            const float e0 = (cv0 * cv0 + cv1 * cv1 + cv2 * cv2) * ra;
            const float rsa = __builtin_amdgcn_rsqf(a);
            // prefactor of Eq. 3 times beta: beta sqrt(pi / (2a)) exp(-e0 / 2)
            const float P0 = r.bp * rsa * __expf(-0.5f * e0);
            const bool act = valid && (P0 + P0 > p.pair_eps);
            const uint64_t abal = __ballot(act);
            if (abal == 0ull) continue;
            if (STATS) n_act += __popcll(abal);
            // Distance along the ray of the Mahalanobis-closest point:
            // t* = -b/a = t_e - (W d).(W p)/a with p = d x v the perpendicular offset.
            const float p0 = fy * vz - fz * vy, p1 = fz * vx - fx * vz, p2 = fx * vy - fy * vx;
            const float wp0 = r.w[0] * p0 + r.w[1] * p1 + r.w[2] * p2;
            const float wp1 = r.w[3] * p0 + r.w[4] * p1 + r.w[5] * p2;
            const float wp2 = r.w[6] * p0 + r.w[7] * p1 + r.w[8] * p2;
            const float corr = (wd0 * wp0 + wd1 * wp1 + wd2 * wp2) * ra;
            const float th = (float)te;
            const float tl = (float)(te - (double)th);
            const float sa = a * rsa * 0.70710678118654752f;      // sqrt(a / 2)
            const float ts = (th - corr) + tl;                      // t*
            const float xs = -sa * ts;                              // erf argument at t = 0
            float Ep = -1.f;
            if (xs > -kZc) Ep = erff(xs);
            int ka = K, kb = -1;
            if (act) {
                // shells whose erf argument lies in (-kZc, kZc), widened by one on each side
                const float half = kZc * __builtin_amdgcn_rcpf(sa);
                const float klo = fminf(shell_index(ts - half, g, lr0, inv), (float)K);
                const float khi = fmaxf(shell_index(ts + half, g, lr0, inv), -1.f);
                ka = klo < 1.f ? 0 : (int)klo - 1;
                kb = khi > (float)(K - 3) ? K - 1 : max(0, (int)khi + 2);
            }
            const int kmin = wave_min(ka), kmax = wave_max(kb);
            if (STATS && kmax >= kmin) n_ramp += (unsigned long long)__popcll(abal) * (kmax - kmin + 1);
            for (int k = kmin; k <= kmax; ++k) {
                const float2 tk = shell[k];
                const float x = sa * (((tk.x - th) + (tk.y - tl)) + corr);
                const float E = fmaxf(erff(x), Ep);     // keep the increments non-negative
                const float dI = P0 * (E - Ep);
                Ep = E;
                if (act && dI > 0.f)
                    __hip_atomic_fetch_add(inc + k * kWave + lane, dI, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        __syncthreads();
    }

    if (STATS) {
        const unsigned long long nvalid = __popcll(__ballot(valid));
        if (lane == 0) {
            atomicAdd(p.stats + 0, n_hits * nvalid);
            atomicAdd(p.stats + 1, n_act);
            atomicAdd(p.stats + 2, n_ramp);
            atomicAdd(p.stats + 3, (unsigned long long)cnt);
        }
    }

    if (valid) {
        const size_t plane = (size_t)g.H * g.W;
        const size_t off = (size_t)light * K * plane + (size_t)py * g.W + px;
        const float* bt = p.base_tau ? p.base_tau + off : nullptr;
        float tau = 0.f, Tp = 1.f;
        if (p.write_tau) {
            float* out = reinterpret_cast<float*>(p.out) + off;
            for (int k = 0; k < K; ++k) {
                tau += inc[k * kWave + lane];
                out[(size_t)k * plane] = bt ? tau + bt[(size_t)k * plane] : tau;
            }
        } else {
            OutT* out = reinterpret_cast<OutT*>(p.out) + off;
            for (int k = 0; k < K; ++k) {
                tau += inc[k * kWave + lane];
                const float tt = bt ? tau + bt[(size_t)k * plane] : tau;
                const float T = fminf(__expf(-tt), Tp);   // exactly non-increasing in k
                Tp = T;
                Store<OutT>::put(out + (size_t)k * plane, T);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

BuildLayout build_layout(const Geom& g, int64_t n, int n_lights) {
    BuildLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    L.nb = (int)((n + kPrepThreads - 1) / kPrepThreads);
    L.tcone = take((size_t)g.ntiles * sizeof(float4));
    L.scone = take((size_t)kMaxSuper * sizeof(float4));
    L.light0 = off;
    off = 0;
    L.totals = take((size_t)kMaxSuper * sizeof(int));
    L.rec = take((size_t)n * sizeof(GRec));
    L.cone = take((size_t)n * sizeof(float4));
    L.mask = take((size_t)n * sizeof(uint64_t));
    L.counts = take((size_t)g.S * (size_t)L.nb * sizeof(int));
    L.lists = take((size_t)n * (size_t)g.S * sizeof(int));
    L.light_stride = off;
    L.total = L.light0 + (size_t)n_lights * L.light_stride;
    return L;
}

size_t tile_smem_bytes(const Geom& g) {
    return (size_t)g.K * kWave * sizeof(float) + (size_t)g.K * sizeof(float2) + kWave * sizeof(int);
}

template <typename OutT, bool STATS>
static hipError_t launch_tile(const TileArgs& ta, int n_lights, hipStream_t st) {
    const size_t smem = tile_smem_bytes(ta.g);
    if (smem > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute((const void*)tile_build_kernel<OutT, STATS>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
        if (e != hipSuccess) return e;
    }
    tile_build_kernel<OutT, STATS><<<dim3(ta.g.ntiles, n_lights), kWave, smem, st>>>(ta);
    return hipGetLastError();
}

dgsm_status enqueue_bin(const Geom& g, const BuildLayout& L, unsigned char* ws, const dgsm_lights_t& lights,
                        float cull_eps, const dgsm_gaussians_t& gs, hipStream_t st) {
    float4* tcone = reinterpret_cast<float4*>(ws + L.tcone);
    float4* scone = reinterpret_cast<float4*>(ws + L.scone);
    tile_cone_kernel<<<(g.ntiles + 63) / 64, 64, 0, st>>>(g, tcone);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    super_cone_kernel<<<1, 64, 0, st>>>(g, tcone, scone);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    if (gs.n > 0) {
        PrepArgs pa{gs.mean, gs.scale, gs.rot, gs.opacity, gs.n, lights.pos, lights.kappa, cull_eps,
                    g.S, L, ws};
        preprocess_kernel<<<dim3(L.nb, lights.n), kPrepThreads, 0, st>>>(pa);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    }
    scan_kernel<<<dim3(g.S, lights.n), 256, 0, st>>>(ws, L);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    if (gs.n > 0) {
        scatter_kernel<<<dim3(L.nb, lights.n), kPrepThreads, 0, st>>>(ws, L, gs.n, g.S);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    }
    return DGSM_OK;
}

dgsm_status enqueue_accumulate(const Geom& g, const BuildLayout& L, unsigned char* ws, int n_lights,
                               float pair_eps, void* atlas, const AccumOpts& o, hipStream_t st) {
    TileArgs ta{g, L, ws, pair_eps, atlas, o.base_tau, o.write_tau ? 1 : 0, o.stats};
    hipError_t e;
    const bool half = g.dtype == DGSM_F16 && !o.write_tau;
    if (o.stats)
        e = half ? launch_tile<__half, true>(ta, n_lights, st) : launch_tile<float, true>(ta, n_lights, st);
    else
        e = half ? launch_tile<__half, false>(ta, n_lights, st) : launch_tile<float, false>(ta, n_lights, st);
    return e == hipSuccess ? DGSM_OK : DGSM_EHIP;
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
    if (gaussians->n * (int64_t)g.S >= (int64_t)INT32_MAX) return DGSM_EUNSUPPORTED;
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
    const BuildLayout L = build_layout(g, gaussians->n, lights->n);
    if (!ws || ws_bytes < L.total) return DGSM_EWORKSPACE;
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
    const BuildLayout L = build_layout(g, n_gauss, lights->n);
    if (!ws || ws_bytes < L.total) return DGSM_EWORKSPACE;
    AccumOpts o{nullptr, false, stats};
    return enqueue_accumulate(g, L, reinterpret_cast<unsigned char*>(ws), lights->n, desc->cull_eps, atlas, o,
                              reinterpret_cast<hipStream_t>(stream));
}

extern "C" dgsm_status dgsm_build(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                                  const dgsm_atlas_desc_t* desc, void* atlas, void* ws, size_t ws_bytes,
                                  void* stream) {
    dgsm_status st = check_build_args(lights, gaussians, desc);
    if (st != DGSM_OK) return st;
    if (!atlas) return DGSM_EINVAL;
    const Geom g = make_geom(*desc);
    const BuildLayout L = build_layout(g, gaussians->n, lights->n);
    if (!ws || ws_bytes < L.total) return DGSM_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    unsigned char* w = reinterpret_cast<unsigned char*>(ws);
    if ((st = enqueue_bin(g, L, w, *lights, desc->cull_eps, *gaussians, s)) != DGSM_OK) return st;
    AccumOpts o{nullptr, false, nullptr};
    return enqueue_accumulate(g, L, w, lights->n, desc->cull_eps, atlas, o, s);
}
