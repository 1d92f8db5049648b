// Domain check of a Gaussian set (Eqs. 1-5 need finite parameters, positive
// scales, opacities in [0, 1) and a non-zero rotation quaternion).

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"

#include <math.h>

namespace dgsm {

__global__ __launch_bounds__(256) void zero_counter_kernel(long long* c) {
    if (threadIdx.x == 0) *c = 0;
}

__global__ __launch_bounds__(256) void check_kernel(dgsm_gaussians_t gs, long long* counter) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool bad = false;
    if (i < gs.n) {
        float q2 = 0.f;
        for (int c = 0; c < 3; ++c) {
            const float m = gs.mean[3 * i + c], s = gs.scale[3 * i + c];
            bad |= !isfinite(m) || !isfinite(s) || !(s > 0.f);
        }
        for (int c = 0; c < 4; ++c) {
            const float q = gs.rot[4 * i + c];
            bad |= !isfinite(q);
            q2 += q * q;
        }
        const float a = gs.opacity[i];
        bad |= !(q2 > 0.f) || !(a >= 0.f && a < 1.f);
    }
    const uint64_t b = __ballot(bad);
    if (b && (threadIdx.x % kWave) == 0) atomicAdd(reinterpret_cast<unsigned long long*>(counter), __popcll(b));
}

}  // namespace dgsm

using namespace dgsm;

extern "C" dgsm_status dgsm_check_gaussians(const dgsm_gaussians_t* gaussians, long long* counter, long long* n_bad,
                                            void* stream) {
    dgsm_status st = validate_gaussians(gaussians);
    if (st != DGSM_OK) return st;
    if (!counter || !n_bad) return DGSM_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    zero_counter_kernel<<<1, 64, 0, s>>>(counter);
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    if (gaussians->n > 0) {
        check_kernel<<<(unsigned)((gaussians->n + 255) / 256), 256, 0, s>>>(*gaussians, counter);
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    }
    if (hipMemcpyAsync(n_bad, counter, sizeof(long long), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return DGSM_EHIP;
    return DGSM_OK;
}
