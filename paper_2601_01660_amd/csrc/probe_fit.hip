// Approximate HDRI probe (Sec. 3.4): SH coefficients of the environment by
// weighted ridge least squares, (B^T W B + lambda I) A = B^T W Y, from radiance
// samples Y at unit directions D with weights w (a cube-map render's pixels
// and their solid angles).  The normal equations are accumulated in FP64 in a
// fixed order (partial sums per block, then one block in block order) and
// solved by Cholesky in FP64.

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"

#include <math.h>

namespace dgsm {

constexpr int kFitThreads = 256;
constexpr int kFitBlocks = 256;
constexpr int kFitMaxK = 16;

// Entries of the normal equations: the upper triangle of B^T W B (K (K+1) / 2,
// row by row), then B^T W Y (K x 3).
__host__ __device__ constexpr int fit_entries(int K) { return K * (K + 1) / 2 + 3 * K; }

__device__ inline void fit_entry(int e, int K, int& i, int& j, bool& gram) {
    const int ng = K * (K + 1) / 2;
    gram = e < ng;
    if (gram) {
        i = 0;
        while (e >= K - i) {
            e -= K - i;
            ++i;
        }
        j = i + e;
    } else {
        i = (e - ng) / 3;
        j = (e - ng) % 3;
    }
}

__global__ __launch_bounds__(kFitThreads) void fit_partial_kernel(const float* __restrict__ Y,
                                                                  const float* __restrict__ D,
                                                                  const float* __restrict__ w, int64_t n, int K,
                                                                  double* __restrict__ part) {
    __shared__ float sB[kFitThreads][kFitMaxK + 1];
    __shared__ float sY[kFitThreads][4];   // w, Y_r, Y_g, Y_b
    const int tid = threadIdx.x;
    const int ne = fit_entries(K);
    int ei = 0, ej = 0;
    bool gram = false;
    if (tid < ne) fit_entry(tid, K, ei, ej, gram);
    double acc = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * kFitThreads; base < n; base += (int64_t)gridDim.x * kFitThreads) {
        const int64_t s = base + tid;
        float Bv[kFitMaxK];
        for (int k = 0; k < kFitMaxK; ++k) Bv[k] = 0.f;
        float ws = 0.f, y0 = 0.f, y1 = 0.f, y2 = 0.f;
        if (s < n) {
            real_sh16(D[3 * s], D[3 * s + 1], D[3 * s + 2], K, Bv);
            ws = w[s];
            y0 = Y[3 * s];
            y1 = Y[3 * s + 1];
            y2 = Y[3 * s + 2];
        }
        for (int k = 0; k < K; ++k) sB[tid][k] = Bv[k];
        sY[tid][0] = ws;
        sY[tid][1] = y0;
        sY[tid][2] = y1;
        sY[tid][3] = y2;
        __syncthreads();
        if (tid < ne)
            for (int t = 0; t < kFitThreads; ++t) {
                const double other = gram ? (double)sB[t][ej] : (double)sY[t][1 + ej];
                acc += (double)sY[t][0] * (double)sB[t][ei] * other;
            }
        __syncthreads();
    }
    if (tid < ne) part[(size_t)blockIdx.x * ne + tid] = acc;
}

__global__ __launch_bounds__(kFitThreads) void fit_solve_kernel(const double* __restrict__ part, int nb, int K,
                                                                float lambda, float* __restrict__ A) {
    __shared__ double G[kFitMaxK][kFitMaxK];
    __shared__ double R[kFitMaxK][3];
    const int tid = threadIdx.x;
    const int ne = fit_entries(K);
    if (tid < ne) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[(size_t)b * ne + tid];
        int i, j;
        bool gram;
        fit_entry(tid, K, i, j, gram);
        if (gram) {
            G[i][j] = s + (i == j ? (double)lambda : 0.0);
            G[j][i] = G[i][j];
        } else {
            R[i][j] = s;
        }
    }
    __syncthreads();
    if (tid != 0) return;
    // Cholesky G = L L^T (L in the lower triangle of G), then L Z = R, L^T A = Z
    for (int c = 0; c < K; ++c) {
        double d = G[c][c];
        for (int k = 0; k < c; ++k) d -= G[c][k] * G[c][k];
        d = sqrt(d);
        G[c][c] = d;
        for (int r = c + 1; r < K; ++r) {
            double v = G[r][c];
            for (int k = 0; k < c; ++k) v -= G[r][k] * G[c][k];
            G[r][c] = v / d;
        }
    }
    for (int ch = 0; ch < 3; ++ch) {
        double z[kFitMaxK];
        for (int r = 0; r < K; ++r) {
            double v = R[r][ch];
            for (int k = 0; k < r; ++k) v -= G[r][k] * z[k];
            z[r] = v / G[r][r];
        }
        for (int r = K - 1; r >= 0; --r) {
            double v = z[r];
            for (int k = r + 1; k < K; ++k) v -= G[k][r] * z[k];
            z[r] = v / G[r][r];
        }
        for (int r = 0; r < K; ++r) A[3 * r + ch] = (float)z[r];
    }
}

}  // namespace dgsm

using namespace dgsm;

extern "C" size_t dgsm_probe_fit_workspace_size(int32_t Kp) {
    if (Kp != 1 && Kp != 4 && Kp != 9 && Kp != 16) return 0;
    return (size_t)kFitBlocks * fit_entries(Kp) * sizeof(double);
}

extern "C" dgsm_status dgsm_probe_fit(const float* Y, const float* D, const float* w, int64_t n, int32_t Kp,
                                      float lambda, float* A, void* ws, size_t ws_bytes, void* stream) {
    if (Kp != 1 && Kp != 4 && Kp != 9 && Kp != 16) return DGSM_EINVAL;
    if (n < 1 || !Y || !D || !w || !A || !(lambda >= 0.f)) return DGSM_EINVAL;
    if (!ws || ws_bytes < dgsm_probe_fit_workspace_size(Kp)) return DGSM_EWORKSPACE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    double* part = reinterpret_cast<double*>(ws);
    fit_partial_kernel<<<kFitBlocks, kFitThreads, 0, s>>>(Y, D, w, n, Kp, part);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    fit_solve_kernel<<<1, kFitThreads, 0, s>>>(part, kFitBlocks, Kp, lambda, A);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}
