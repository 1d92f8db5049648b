// Per-Gaussian SH radiance transfer on gfx950 (Sec. 3.4 evaluation, Sec. 3.5).
//
// Each workgroup stages chunks of the lat-long grid in LDS as
// (w_x, w_y, w_z, weight) and (weight * L_r, weight * L_g, weight * L_b)
// with L = B(w) A evaluated from the probe.  A workgroup serves 64 Gaussians
// (one per lane, the same 64 in each of its four waves); the four waves sweep
// every fourth staged direction, and their partial sums are added in wave
// order at the end (four times the waves of one Gaussian per thread sweeping
// every direction, for latency).

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"

namespace dgsm {

constexpr int kShThreads = 256;
constexpr int kShWaves = kShThreads / kWave;   // waves sharing one lane's Gaussian
constexpr int kShChunk = 512;
constexpr int kShG = 1;                        // Gaussians per lane

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

// Clipped per-channel scale from the sums (n_r, n_g, n_b, den), then the relit
// SH coefficients and RGB of Gaussian i.
__device__ inline void finish_gaussian(const ShArgs& a, int64_t i, float4 acc) {
    const float inv = 1.f / (acc.w + a.eps);
    const float s[3] = {fminf(fmaxf(acc.x * inv, 0.f), a.clip_max), fminf(fmaxf(acc.y * inv, 0.f), a.clip_max),
                        fminf(fmaxf(acc.z * inv, 0.f), a.clip_max)};
    for (int c = 0; c < 3; ++c) a.scale_out[3 * i + c] = s[c];
    if (a.colour_sh) {
        const float* f = a.colour_sh + 48 * i;
        if (a.colour_sh_out) {
            float* fo = a.colour_sh_out + 48 * i;
            for (int k = 0; k < 16; ++k)
                for (int c = 0; c < 3; ++c) fo[3 * k + c] = a.gamma * s[c] * f[3 * k + c];
        }
        if (a.rgb_out)
            for (int c = 0; c < 3; ++c)
                a.rgb_out[3 * i + c] = fmaxf(0.f, a.gamma * (0.5f + 0.28209479177387814f * f[c]) * s[c]);
    }
}

__global__ __launch_bounds__(kShThreads) void sh_transfer_kernel(ShArgs a) {
    __shared__ float4 dirw[kShChunk];
    __shared__ float4 lw[kShChunk];
    __shared__ float4 part[kShWaves][kShG * kWave];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    // lane's Gaussians: i0 + 64 g, g < kShG
    const int64_t i0 = (int64_t)blockIdx.x * (kShG * kWave) + lane;
    float3 nrm[kShG];
#pragma unroll
    for (int g = 0; g < kShG; ++g)
        nrm[g] = i0 + kWave * g < a.n ? gaussian_normal(a, i0 + kWave * g) : make_float3(0.f, 0.f, 1.f);

    float4 acc[kShG];
#pragma unroll
    for (int g = 0; g < kShG; ++g) acc[g] = make_float4(0.f, 0.f, 0.f, 0.f);
    const int M = a.n_theta * a.n_phi;
    const float dth = 3.14159265358979324f / (float)a.n_theta;
    const float dph = 6.28318530717958648f / (float)a.n_phi;
    for (int c0 = 0; c0 < M; c0 += kShChunk) {
        const int cnt = min(kShChunk, M - c0);
        __syncthreads();
        for (int j = tid; j < cnt; j += kShThreads) {
            const int gj = c0 + j;
            const int ia = gj / a.n_phi, ib = gj - ia * a.n_phi;
            float st, ct, sp, cp;
            sincosf(((float)ia + 0.5f) * dth, &st, &ct);
            sincosf(((float)ib + 0.5f) * dph, &sp, &cp);
            const float wx = st * cp, wy = st * sp, wz = ct;
            float Y[16];
            real_sh16(wx, wy, wz, a.kp, Y);
            float L0 = 0.f, L1 = 0.f, L2 = 0.f;
            for (int k = 0; k < a.kp; ++k) {
                L0 += Y[k] * a.probe[3 * k];
                L1 += Y[k] * a.probe[3 * k + 1];
                L2 += Y[k] * a.probe[3 * k + 2];
            }
            dirw[j] = make_float4(wx, wy, wz, st);
            lw[j] = make_float4(st * L0, st * L1, st * L2, 0.f);
        }
        __syncthreads();
        // the cosine lobe max(0, n.w)^q; q = 1 (the default) without the power
        if (a.q == 1.f) {
            for (int j = wave; j < cnt; j += kShWaves) {
                const float4 d = dirw[j];
                const float4 l = lw[j];
#pragma unroll
                for (int g = 0; g < kShG; ++g) {
                    const float S = fmaxf(0.f, nrm[g].x * d.x + nrm[g].y * d.y + nrm[g].z * d.z);
                    acc[g].x += l.x * S; acc[g].y += l.y * S; acc[g].z += l.z * S; acc[g].w += d.w * S;
                }
            }
        } else {
            for (int j = wave; j < cnt; j += kShWaves) {
                const float4 d = dirw[j];
                const float4 l = lw[j];
#pragma unroll
                for (int g = 0; g < kShG; ++g) {
                    const float c = nrm[g].x * d.x + nrm[g].y * d.y + nrm[g].z * d.z;
                    const float S = c > 0.f ? __powf(c, a.q) : 0.f;
                    acc[g].x += l.x * S; acc[g].y += l.y * S; acc[g].z += l.z * S; acc[g].w += d.w * S;
                }
            }
        }
    }
    // the waves' partial sums, added in wave order; wave g finishes Gaussian i0 + 64 g
#pragma unroll
    for (int g = 0; g < kShG; ++g) part[wave][g * kWave + lane] = acc[g];
    __syncthreads();
    if (wave >= kShG) return;
    const int64_t i = i0 + kWave * wave;
    if (i >= a.n) return;
    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int w = 0; w < kShWaves; ++w) {
        const float4 q = part[w][wave * kWave + lane];
        sum.x += q.x; sum.y += q.y; sum.z += q.z; sum.w += q.w;
    }
    finish_gaussian(a, i, sum);
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

extern "C" dgsm_status sh_transfer(const float* probe_sh, int32_t Kp, const dgsm_gaussians_t* gaussians,
                                   const float* colour_sh, const dgsm_sh_params_t* params, float* scale_out,
                                   float* colour_sh_out, float* rgb_out, void* stream) {
    if (!probe_sh || !(Kp == 1 || Kp == 4 || Kp == 9 || Kp == 16)) return DGSM_EINVAL;
    dgsm_status st = validate_gaussians(gaussians);
    if (st != DGSM_OK) return st;
    if (!params || params->n_theta < 1 || params->n_phi < 1 || !(params->q > 0.f) ||
        !(params->clip_max > 0.f) || !(params->eps >= 0.f) || !params->centroid)
        return DGSM_EINVAL;
    if ((int64_t)params->n_theta * params->n_phi > (1 << 24)) return DGSM_EINVAL;
    if ((colour_sh_out || rgb_out) && !colour_sh) return DGSM_EINVAL;
    if (gaussians->n > 0 && !scale_out) return DGSM_EINVAL;
    if (gaussians->n == 0) return DGSM_OK;
    ShArgs a{probe_sh, Kp, gaussians->mean, gaussians->scale, gaussians->rot, gaussians->n, colour_sh,
             params->centroid, params->n_theta, params->n_phi, params->q, params->clip_max, params->eps,
             params->gamma, scale_out, colour_sh_out, rgb_out};
    const unsigned blocks = (unsigned)((gaussians->n + kShG * kWave - 1) / (kShG * kWave));
    sh_transfer_kernel<<<blocks, kShThreads, 0, reinterpret_cast<hipStream_t>(stream)>>>(a);
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
