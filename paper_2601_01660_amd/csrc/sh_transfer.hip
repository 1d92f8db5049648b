// Per-Gaussian SH radiance transfer on gfx950 (Sec. 3.4 evaluation, Sec. 3.5).
//
// probe_table_kernel evaluates the probe once per call on the lat-long grid
// into the caller's workspace.  sh_transfer_kernel then forms, for every
// Gaussian, the four sums over grid directions w_j of the cosine lobe S_j =
// max(0, n . w_j)^q times (sin theta L_r, sin theta L_g, sin theta L_b,
// sin theta).  Those sums are a product of the [Gaussians x directions] lobe
// matrix with the [directions x 4] table; most of it runs on the matrix cores,
// the rest on the vector units, which also form the lobes: two multiply-adds
// per direction, with the grid's rows and the column groups' first edges
// factored out of n . w.  A workgroup serves 64 Gaussians (one per lane, the
// same 64 in each of its eight waves); wave w sweeps the w-th eighth of the
// direction groups and the eight partial sums are added in wave order at the
// end.  Eight waves rather than four: the 150k-Gaussian avatar then makes 2.3
// rounds of resident waves instead of 1.15, whose second round left most
// SIMDs idle.

#include <algorithm>

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"

namespace dgsm {

constexpr int kShThreads = 512;   // eight waves
constexpr int kShWaves = kShThreads / kWave;   // waves sharing one lane's Gaussians
constexpr int kShMfma = 12;   // directions of each group of 16 summed on the matrix cores
static_assert(kShMfma >= 4 && kShMfma <= 12 && kShMfma % 4 == 0, "whole scalar table entries on both sides");
constexpr int kShColPer = (kWave * 48 + kShThreads - 1) / kShThreads;   // colour floats per thread

struct ShArgs {
    const float* probe;      // [kp][3]
    int kp;
    const float* mean;
    const float* scale;
    const float* rot;
    int64_t n;
    const float* colour_sh;  // [n][16][3] or null
    const float* centroid;   // [3]
    int n_theta, n_phi;
    float q, clip_max, eps, gamma;
    float* scale_out;
    float* colour_sh_out;
    float* rgb_out;
    int n_phi16;             // columns padded to a multiple of 16
    const float* bt;         // [n_theta][n_phi16][4] weighted radiance and weight
    const float2* cs;        // [16] (cos, sin) of the columns of a group from its first edge
    const float2* cg;        // [max(2, n_phi16 / 16)] (cos, sin) of the groups' first edges
    const float2* rt;        // [n_theta] (sin theta, cos theta)
};

// Normal of Gaussian i: rotation column of its smallest scale, facing away
// from the centroid.
__device__ inline float3 gaussian_normal(const ShArgs& a, int64_t i) {
    float qw = a.rot[4 * i], qx = a.rot[4 * i + 1], qy = a.rot[4 * i + 2], qz = a.rot[4 * i + 3];
    const float qn = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    const float s0 = a.scale[3 * i], s1 = a.scale[3 * i + 1], s2 = a.scale[3 * i + 2];
    int ax = 0;
    if (s1 < s0) ax = 1;
    if (s2 < (ax == 0 ? s0 : s1)) ax = 2;
    float nx, ny, nz;
    if (ax == 0) { nx = 1 - 2 * (qy * qy + qz * qz); ny = 2 * (qx * qy + qw * qz); nz = 2 * (qx * qz - qw * qy); }
    else if (ax == 1) { nx = 2 * (qx * qy - qw * qz); ny = 1 - 2 * (qx * qx + qz * qz); nz = 2 * (qy * qz + qw * qx); }
    else { nx = 2 * (qx * qz + qw * qy); ny = 2 * (qy * qz - qw * qx); nz = 1 - 2 * (qx * qx + qy * qy); }
    const float side = nx * (a.mean[3 * i] - a.centroid[0]) + ny * (a.mean[3 * i + 1] - a.centroid[1]) +
                       nz * (a.mean[3 * i + 2] - a.centroid[2]);
    if (side < 0.f) { nx = -nx; ny = -ny; nz = -nz; }
    return make_float3(nx, ny, nz);
}

// Probe table, written once per call into the caller's workspace.  The grid
// has cell centres theta_a = (a + 1/2) pi / n_theta, phi_b = (b + 1/2) dphi
// with dphi = 2 pi / n_phi and solid-angle weight sin theta_a; its columns are
// padded to a multiple of 16 (padded directions carry zero weight):
//   bt[a][b] = (sin theta L_r, sin theta L_g, sin theta L_b, sin theta), L = B(w) A
//   cs[t]    = (cos (t + 1/2) dphi, sin (t + 1/2) dphi), t < 16: the columns
//              of a group of 16 relative to its first edge
//   cg[c]    = (cos 16 c dphi, sin 16 c dphi): the first edge of column group
//              c (at least two entries; cg[1] is the step between groups)
//   rt[a]    = (sin theta_a, cos theta_a)
// One thread per padded direction.
__global__ __launch_bounds__(256) void probe_table_kernel(const float* __restrict__ probe, int kp, int n_theta,
                                                          int n_phi, int n_phi16, float4* __restrict__ bt,
                                                          float2* __restrict__ cs, float2* __restrict__ cg,
                                                          float2* __restrict__ rt) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n_theta * n_phi16) return;
    const int ia = j / n_phi16, ib = j - ia * n_phi16;
    const float dphi = 6.28318530717958648f / (float)n_phi;
    float st, ct, sp, cp;
    sincosf(((float)ia + 0.5f) * (3.14159265358979324f / (float)n_theta), &st, &ct);
    sincosf(((float)ib + 0.5f) * dphi, &sp, &cp);
    if (ib == 0) rt[ia] = make_float2(st, ct);
    if (ia == 0) {
        if (ib < 16) cs[ib] = make_float2(cp, sp);
        if (ib % 16 == 0) {
            float sg, cgc;
            sincosf((float)ib * dphi, &sg, &cgc);
            cg[ib / 16] = make_float2(cgc, sg);
            if (n_phi16 == 16) {   // one group per row: the step entry is never used
                sincosf(16.f * dphi, &sg, &cgc);
                cg[1] = make_float2(cgc, sg);
            }
        }
    }
    if (ib >= n_phi) {
        bt[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        return;
    }
    float Y[16];
    real_sh16(st * cp, st * sp, ct, kp, Y);
    float L0 = 0.f, L1 = 0.f, L2 = 0.f;
    for (int k = 0; k < kp; ++k) {
        L0 += Y[k] * probe[3 * k];
        L1 += Y[k] * probe[3 * k + 1];
        L2 += Y[k] * probe[3 * k + 2];
    }
    bt[j] = make_float4(st * L0, st * L1, st * L2, st);
}

// The sums over directions, split between the matrix cores and the vector
// units.  For the 16 directions of a group, lane l of one VGPR holds entry l
// of the group's 16 x 4 table block (direction l / 4, channel l % 4).  One
// v_mfma_f32_4x4x1_16b_f32 per direction t < kShMfma broadcasts that
// direction's four channels (the A operand of block t) to all 16 blocks
// (CBSZ 4, ABID t) and multiplies them by the lanes' cosine lobes (the B
// operand, lane j + 4b of block b), so the accumulator of lane l collects its
// own Gaussian's four sums in its four registers.  The other 16 - kShMfma
// directions are summed with four vector multiply-adds each, from table
// entries read with scalar loads one group ahead.  One such product keeps the
// matrix pipe busy for 32 cycles (the FP32 4x4 shape runs at a quarter of the
// matrix cores' FP32 rate), about as long as the four multiply-adds it
// replaces take on the vector unit, and the two pipes overlap only in part
// (counters on the 150k avatar: matrix pipe busy 73% and vector unit 67% of
// the kernel); 12 of 16 on the matrix cores ran fastest (0.069 ms per call;
// 16: 0.074, 8: 0.073, 4: 0.073, all on the vector units as before: 0.104).
typedef float shv4 __attribute__((ext_vector_type(4)));
typedef float shv16 __attribute__((ext_vector_type(16)));
typedef const __attribute__((address_space(4))) shv16* ShConst16;
typedef float shv2 __attribute__((ext_vector_type(2)));
typedef const __attribute__((address_space(4))) shv2* ShConst2;

template <int T>
__device__ inline void sh_mfma(float bv, const float (&S)[16], shv4 (&acc)[2]) {
    acc[T % 2] = __builtin_amdgcn_mfma_f32_4x4x1f32(bv, S[T], acc[T % 2], 4, T, 0);
    if constexpr (T + 1 < kShMfma) sh_mfma<T + 1>(bv, S, acc);
}

template <bool LAMBERT>
__global__ __launch_bounds__(kShThreads) void sh_transfer_kernel(ShArgs a) {
    __shared__ float4 part[kShWaves][kWave];
    __shared__ float sc[kWave][3];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int64_t base = (int64_t)blockIdx.x * kWave;
    const int64_t i = base + lane;
    const float3 nrm = i < a.n ? gaussian_normal(a, i) : make_float3(0.f, 0.f, 1.f);
    // the colour coefficients this thread rescales at the end (48 consecutive
    // floats per Gaussian, one per thread and pass), loaded now so that their
    // latency passes during the sums
    const int64_t ng = min((int64_t)kWave, a.n - base);
    float fc[kShColPer];
    if (a.colour_sh_out) {
        const float* f = a.colour_sh + 48 * base;
#pragma unroll
        for (int k = 0; k < kShColPer; ++k) {
            const int e = tid + k * kShThreads;
            fc[k] = e < ng * 48 ? f[e] : 0.f;
        }
    }
    float f0[3] = {0.f, 0.f, 0.f};   // DC colour of the lane's Gaussian (wave 0)
    if (a.rgb_out && wave == 0 && i < a.n) {
        f0[0] = a.colour_sh[48 * i];
        f0[1] = a.colour_sh[48 * i + 1];
        f0[2] = a.colour_sh[48 * i + 2];
    }
    const int gpr = a.n_phi16 / 16;   // 16-direction groups per row
    const int G = a.n_theta * gpr;
    const int per = (G + kShWaves - 1) / kShWaves;
    // wave-uniform group range (readfirstlane: the table reads below become
    // scalar loads)
    const int g0 = __builtin_amdgcn_readfirstlane(min(G, wave * per));
    const int g1 = __builtin_amdgcn_readfirstlane(min(G, g0 + per));
    shv4 acc[2] = {{0.f, 0.f, 0.f, 0.f}, {0.f, 0.f, 0.f, 0.f}};
    float vx = 0.f, vy = 0.f, vz = 0.f, vw = 0.f;
    if (g0 < g1) {
        const ShConst16 csv = (ShConst16)(const void*)a.cs;
        const ShConst16 btv = (ShConst16)(const void*)a.bt;   // four directions per entry
        const ShConst2 cgv = (ShConst2)(const void*)a.cg;
        const ShConst2 rtv = (ShConst2)(const void*)a.rt;
        // (cos, sin) of the 16 columns of a group relative to its first edge:
        // the same 32 values for every group of the sweep
        const shv16 c0s = csv[0], c1s = csv[1];
        float c0[16], c1[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            // vector-register copies (one move each per sweep), so that the
            // scalar registers can hold the next group's table entries while
            // this group is summed
            asm("v_mov_b32 %0, %1" : "=v"(c0[k]) : "s"(c0s[k]));
            asm("v_mov_b32 %0, %1" : "=v"(c1[k]) : "s"(c1s[k]));
        }
        const shv2 step = cgv[1];
        int row = g0 / gpr, c16 = g0 - row * gpr;
        // n . w = (sin theta n_x) cos phi + (sin theta n_y) sin phi + cos theta n_z;
        // with phi = alpha + beta (alpha the group's first edge) the first two
        // terms are Pr cos beta + Qr sin beta, where (Pr, Qr) is
        // (P, Q) = sin theta (n_x, n_y) rotated by alpha
        shv2 r = rtv[row], r_next = rtv[min(row + 1, a.n_theta - 1)];
        float P = r.x * nrm.x, Q = r.x * nrm.y, R = r.y * nrm.z;
        const shv2 a0 = cgv[c16];
        float Pr = fmaf(P, a0.x, Q * a0.y), Qr = fmaf(Q, a0.x, -P * a0.y);
        float bv = a.bt[(size_t)g0 * 64 + lane];
        shv16 e[(16 - kShMfma) / 4];
#pragma unroll
        for (int k = 0; k < (16 - kShMfma) / 4; ++k) e[k] = btv[(size_t)g0 * 4 + kShMfma / 4 + k];
        for (int g = g0; g < g1; ++g) {
            const int gn = min(g + 1, g1 - 1);
            const float bv_next = a.bt[(size_t)gn * 64 + lane];
            float S[16];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const float x0 = fmaf(Pr, c0[2 * t], fmaf(Qr, c0[2 * t + 1], R));
                const float x1 = fmaf(Pr, c1[2 * t], fmaf(Qr, c1[2 * t + 1], R));
                if (LAMBERT) {
                    // max(0, n.w): n.w cannot exceed 1 beyond rounding, so the
                    // clamp to [0, 1] rides on the last multiply-add
                    S[t] = __builtin_amdgcn_fmed3f(x0, 0.f, 1.f);
                    S[t + 8] = __builtin_amdgcn_fmed3f(x1, 0.f, 1.f);
                } else {
                    S[t] = x0 > 0.f ? __powf(x0, a.q) : 0.f;
                    S[t + 8] = x1 > 0.f ? __powf(x1, a.q) : 0.f;
                }
            }
            sh_mfma<0>(bv, S, acc);
#pragma unroll
            for (int t = kShMfma; t < 16; ++t) {
                const int k = (t - kShMfma) / 4, o = 4 * ((t - kShMfma) % 4);
                vx = fmaf(e[k][o], S[t], vx);
                vy = fmaf(e[k][o + 1], S[t], vy);
                vz = fmaf(e[k][o + 2], S[t], vz);
                vw = fmaf(e[k][o + 3], S[t], vw);
            }
            // the next group's scalar entries, in flight during its lobes and
            // matrix products
#pragma unroll
            for (int k = 0; k < (16 - kShMfma) / 4; ++k) e[k] = btv[(size_t)gn * 4 + kShMfma / 4 + k];
            bv = bv_next;
            if (++c16 == gpr) {
                // next row: exact restart at its first column
                c16 = 0;
                ++row;
                r = r_next;
                r_next = rtv[min(row + 1, a.n_theta - 1)];
                P = r.x * nrm.x; Q = r.x * nrm.y; R = r.y * nrm.z;
                Pr = P; Qr = Q;
            } else {
                // next group of the row: rotate by 16 dphi
                const float t = Pr;
                Pr = fmaf(step.x, Pr, step.y * Qr);
                Qr = fmaf(step.x, Qr, -step.y * t);
            }
        }
    }

    // the waves' partial sums, added in wave order; wave 0 forms the scales,
    // then the whole workgroup writes the relit coefficients coalesced
    part[wave][lane] = make_float4(acc[0][0] + acc[1][0] + vx, acc[0][1] + acc[1][1] + vy,
                                   acc[0][2] + acc[1][2] + vz, acc[0][3] + acc[1][3] + vw);
    __syncthreads();
    if (wave == 0) {
        float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int w = 0; w < kShWaves; ++w) {
            const float4 q = part[w][lane];
            sum.x += q.x; sum.y += q.y; sum.z += q.z; sum.w += q.w;
        }
        const float inv = 1.f / (sum.w + a.eps);
        const float s0 = fminf(fmaxf(sum.x * inv, 0.f), a.clip_max), s1 = fminf(fmaxf(sum.y * inv, 0.f), a.clip_max),
                    s2 = fminf(fmaxf(sum.z * inv, 0.f), a.clip_max);
        sc[lane][0] = s0; sc[lane][1] = s1; sc[lane][2] = s2;
        if (i < a.n) {
            a.scale_out[3 * i] = s0; a.scale_out[3 * i + 1] = s1; a.scale_out[3 * i + 2] = s2;
            if (a.rgb_out) {
                a.rgb_out[3 * i] = fmaxf(0.f, a.gamma * (0.5f + 0.28209479177387814f * f0[0]) * s0);
                a.rgb_out[3 * i + 1] = fmaxf(0.f, a.gamma * (0.5f + 0.28209479177387814f * f0[1]) * s1);
                a.rgb_out[3 * i + 2] = fmaxf(0.f, a.gamma * (0.5f + 0.28209479177387814f * f0[2]) * s2);
            }
        }
    }
    if (!a.colour_sh_out) return;
    __syncthreads();
    // relit coefficients gamma s_c f_kc of the workgroup's Gaussians
    float* fo = a.colour_sh_out + 48 * base;
#pragma unroll
    for (int k = 0; k < kShColPer; ++k) {
        const int e = tid + k * kShThreads;
        if (e < ng * 48) {
            const int gi = e / 48, c = (e - gi * 48) % 3;
            fo[e] = a.gamma * sc[gi][c] * fc[k];
        }
    }
}

// Alpha-weighted centroid, one workgroup, FP64 partial sums in a fixed order.
__global__ __launch_bounds__(1024) void centroid_kernel(const float* __restrict__ mean,
                                                       const float* __restrict__ opacity, int64_t n,
                                                       float* __restrict__ out) {
    __shared__ double red[4][1024];
    const int tid = threadIdx.x;
    double sx = 0, sy = 0, sz = 0, sa = 0;
    for (int64_t i = tid; i < n; i += 1024) {
        const double al = opacity[i];
        sx += al * mean[3 * i]; sy += al * mean[3 * i + 1]; sz += al * mean[3 * i + 2]; sa += al;
    }
    red[0][tid] = sx; red[1][tid] = sy; red[2][tid] = sz; red[3][tid] = sa;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (tid < o)
            for (int c = 0; c < 4; ++c) red[c][tid] += red[c][tid + o];
        __syncthreads();
    }
    if (tid < 3) out[tid] = (float)(red[tid][0] / red[3][0]);
}

}  // namespace dgsm

using namespace dgsm;

namespace {
// Workspace layout of the probe table: bt, cs, cg and rt, each 256-byte aligned.
struct ShTableLayout {
    int n_phi16;
    size_t cs, cg, rt, bytes;
};
ShTableLayout sh_table_layout(int32_t n_theta, int32_t n_phi) {
    ShTableLayout t;
    t.n_phi16 = (n_phi + 15) / 16 * 16;
    auto up = [](size_t b) { return (b + 255) / 256 * 256; };
    t.cs = up((size_t)n_theta * t.n_phi16 * sizeof(float4));
    t.cg = t.cs + up(16 * sizeof(float2));
    t.rt = t.cg + up((size_t)std::max(2, t.n_phi16 / 16) * sizeof(float2));
    t.bytes = t.rt + up((size_t)n_theta * sizeof(float2));
    return t;
}
}  // namespace

extern "C" size_t sh_transfer_workspace_size(int32_t n_theta, int32_t n_phi) {
    if (n_theta < 1 || n_phi < 1 || (int64_t)n_theta * n_phi > (1 << 24)) return 0;
    return sh_table_layout(n_theta, n_phi).bytes;
}

extern "C" dgsm_status sh_transfer(const float* probe_sh, int32_t Kp, const dgsm_gaussians_t* gaussians,
                                   const float* colour_sh, const dgsm_sh_params_t* params, float* scale_out,
                                   float* colour_sh_out, float* rgb_out, void* ws, size_t ws_bytes,
                                   void* stream) {
    if (!probe_sh || !(Kp == 1 || Kp == 4 || Kp == 9 || Kp == 16)) return DGSM_EINVAL;
    dgsm_status st = validate_gaussians(gaussians);
    if (st != DGSM_OK) return st;
    if (!params || params->n_theta < 1 || params->n_phi < 1 || !(params->q > 0.f) ||
        !(params->clip_max > 0.f) || !(params->eps >= 0.f) || !params->centroid)
        return DGSM_EINVAL;
    if ((int64_t)params->n_theta * params->n_phi > (1 << 24)) return DGSM_EINVAL;
    if ((colour_sh_out || rgb_out) && !colour_sh) return DGSM_EINVAL;
    if (gaussians->n > 0 && !scale_out) return DGSM_EINVAL;
    if (!ws || ws_bytes < sh_transfer_workspace_size(params->n_theta, params->n_phi)) return DGSM_EWORKSPACE;
    if (reinterpret_cast<uintptr_t>(ws) % 16) return DGSM_EINVAL;
    if (gaussians->n == 0) return DGSM_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const ShTableLayout t = sh_table_layout(params->n_theta, params->n_phi);
    const int M16 = params->n_theta * t.n_phi16;
    char* w = reinterpret_cast<char*>(ws);
    float4* bt = reinterpret_cast<float4*>(w);
    float2* cs = reinterpret_cast<float2*>(w + t.cs);
    float2* cg = reinterpret_cast<float2*>(w + t.cg);
    float2* rt = reinterpret_cast<float2*>(w + t.rt);
    probe_table_kernel<<<(M16 + 255) / 256, 256, 0, s>>>(probe_sh, Kp, params->n_theta, params->n_phi, t.n_phi16,
                                                          bt, cs, cg, rt);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    ShArgs a{probe_sh, Kp, gaussians->mean, gaussians->scale, gaussians->rot, gaussians->n, colour_sh,
             params->centroid, params->n_theta, params->n_phi, params->q, params->clip_max, params->eps,
             params->gamma, scale_out, colour_sh_out, rgb_out, t.n_phi16,
             reinterpret_cast<const float*>(bt), cs, cg, rt};
    const unsigned blocks = (unsigned)((gaussians->n + kWave - 1) / kWave);
    if (params->q == 1.f)
        sh_transfer_kernel<true><<<blocks, kShThreads, 0, s>>>(a);
    else
        sh_transfer_kernel<false><<<blocks, kShThreads, 0, s>>>(a);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

extern "C" dgsm_status dgsm_alpha_centroid(const dgsm_gaussians_t* gaussians, float* centroid, void* stream) {
    dgsm_status st = validate_gaussians(gaussians);
    if (st != DGSM_OK) return st;
    if (gaussians->n < 1 || !centroid) return DGSM_EINVAL;
    centroid_kernel<<<1, 1024, 0, reinterpret_cast<hipStream_t>(stream)>>>(gaussians->mean, gaussians->opacity,
                                                                          gaussians->n, centroid);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}
