// Per-Gaussian SH radiance transfer on gfx950 (Sec. 3.4 evaluation, Sec. 3.5).
//
// probe_table_kernel evaluates the probe once per call on the lat-long grid
// into the caller's workspace: per direction j, (w_x, w_y, w_z, weight) and
// (weight * L_r, weight * L_g, weight * L_b, 0) with L = B(w) A.
// sh_transfer_kernel streams that table: a workgroup serves 64 Gaussians (one
// per lane, the same 64 in each of its eight waves); wave w sweeps the w-th
// eighth of the directions, reading each direction with wave-uniform scalar
// loads (the table entry lands in scalar registers and feeds the vector
// arithmetic directly, with no LDS traffic), and the eight partial sums are
// added in wave order at the end.  Eight waves per workgroup rather than four:
// the 150k-Gaussian avatar then makes 2.3 rounds of resident waves instead of
// 1.15, whose second round left most SIMDs idle (0.126 -> 0.102 ms).

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"

namespace dgsm {

constexpr int kShThreads = 512;   // eight waves
constexpr int kShWaves = kShThreads / kWave;   // waves sharing one lane's Gaussian

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
    const float4* table;     // [M][2] probe table
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

// Probe radiance and solid-angle weight of every grid direction (cell centres
// theta_a = (a + 1/2) pi / n_theta, phi_b = (b + 1/2) 2 pi / n_phi, weight
// sin theta), one thread per direction.
__global__ __launch_bounds__(256) void probe_table_kernel(const float* __restrict__ probe, int kp, int n_theta,
                                                          int n_phi, float4* __restrict__ table) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n_theta * n_phi) return;
    const int ia = j / n_phi, ib = j - ia * n_phi;
    float st, ct, sp, cp;
    sincosf(((float)ia + 0.5f) * (3.14159265358979324f / (float)n_theta), &st, &ct);
    sincosf(((float)ib + 0.5f) * (6.28318530717958648f / (float)n_phi), &sp, &cp);
    const float wx = st * cp, wy = st * sp, wz = ct;
    float Y[16];
    real_sh16(wx, wy, wz, kp, Y);
    float L0 = 0.f, L1 = 0.f, L2 = 0.f;
    for (int k = 0; k < kp; ++k) {
        L0 += Y[k] * probe[3 * k];
        L1 += Y[k] * probe[3 * k + 1];
        L2 += Y[k] * probe[3 * k + 2];
    }
    table[2 * j] = make_float4(wx, wy, wz, st);
    table[2 * j + 1] = make_float4(st * L0, st * L1, st * L2, 0.f);
}

// Table entries are read with a wave-uniform index through the constant
// address space, so that they land in scalar registers.
typedef float shf4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) shf4* ShConstPtr;

// One direction's contribution to a lane's four sums.
template <bool LAMBERT>
__device__ inline void sh_accum(const float3& nrm, float q, float dx, float dy, float dz, float dw, float lx,
                                float ly, float lz, float& ax, float& ay, float& az, float& aw) {
    const float c = fmaf(nrm.x, dx, fmaf(nrm.y, dy, nrm.z * dz));
    float S;
    if (LAMBERT)
        S = fmaxf(0.f, c);     // the cosine lobe max(0, n.w)^q at q = 1
    else
        S = c > 0.f ? __powf(c, q) : 0.f;
    ax = fmaf(lx, S, ax);
    ay = fmaf(ly, S, ay);
    az = fmaf(lz, S, az);
    aw = fmaf(dw, S, aw);
}

constexpr int kShUnroll = 8;   // directions per scalar-load batch

template <bool LAMBERT>
__global__ __launch_bounds__(kShThreads) void sh_transfer_kernel(ShArgs a) {
    __shared__ float4 part[kShWaves][kWave];
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    const int64_t i = (int64_t)blockIdx.x * kWave + lane;
    const float3 nrm = i < a.n ? gaussian_normal(a, i) : make_float3(0.f, 0.f, 1.f);
    const int M = a.n_theta * a.n_phi;
    const int per = (M + kShWaves - 1) / kShWaves;
    // wave-uniform range (readfirstlane: the compiler then knows it, and the
    // table reads below become scalar loads)
    const int j0 = __builtin_amdgcn_readfirstlane(min(M, wave * per));
    const int j1 = __builtin_amdgcn_readfirstlane(min(M, j0 + per));
    float ax = 0.f, ay = 0.f, az = 0.f, aw = 0.f;
    const ShConstPtr tab = (ShConstPtr)(const void*)a.table;
    int j = j0;
    // batches of kShUnroll directions: all their scalar loads are issued before
    // the arithmetic that uses them
    for (; j + kShUnroll <= j1; j += kShUnroll) {
        shf4 d[kShUnroll], l[kShUnroll];
#pragma unroll
        for (int u = 0; u < kShUnroll; ++u) {
            d[u] = tab[2 * (j + u)];
            l[u] = tab[2 * (j + u) + 1];
        }
#pragma unroll
        for (int u = 0; u < kShUnroll; ++u)
            sh_accum<LAMBERT>(nrm, a.q, d[u].x, d[u].y, d[u].z, d[u].w, l[u].x, l[u].y, l[u].z, ax, ay, az, aw);
    }
    for (; j < j1; ++j) {
        const shf4 d = tab[2 * j], l = tab[2 * j + 1];
        sh_accum<LAMBERT>(nrm, a.q, d.x, d.y, d.z, d.w, l.x, l.y, l.z, ax, ay, az, aw);
    }

    // the waves' partial sums, added in wave order; wave 0 finishes the Gaussians
    part[wave][lane] = make_float4(ax, ay, az, aw);
    __syncthreads();
    if (wave != 0 || i >= a.n) return;
    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int w = 0; w < kShWaves; ++w) {
        const float4 q = part[w][lane];
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

extern "C" size_t sh_transfer_workspace_size(int32_t n_theta, int32_t n_phi) {
    if (n_theta < 1 || n_phi < 1 || (int64_t)n_theta * n_phi > (1 << 24)) return 0;
    return (size_t)n_theta * n_phi * 2 * sizeof(float4);
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
    if (gaussians->n == 0) return DGSM_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int M = params->n_theta * params->n_phi;
    float4* table = reinterpret_cast<float4*>(ws);
    probe_table_kernel<<<(M + 255) / 256, 256, 0, s>>>(probe_sh, Kp, params->n_theta, params->n_phi, table);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    ShArgs a{probe_sh, Kp, gaussians->mean, gaussians->scale, gaussians->rot, gaussians->n, colour_sh,
             params->centroid, params->n_theta, params->n_phi, params->q, params->clip_max, params->eps,
             params->gamma, scale_out, colour_sh_out, rgb_out, table};
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
