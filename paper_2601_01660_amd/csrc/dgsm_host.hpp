// Host-side helpers of the DGSM C ABI: argument validation and workspace layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dgsm.h"
#include "dgsm_device.hpp"

namespace dgsm {

constexpr int kMaxShells = 512;

inline dgsm_status validate_desc(const dgsm_atlas_desc_t* d) {
    if (!d) return DGSM_EINVAL;
    if (d->H < 2 || d->W < 2 || (d->H & 1) || (d->W & 1)) return DGSM_EINVAL;
    if (d->H > 16384 || d->W > 16384) return DGSM_EINVAL;
    if (d->K < 2 || d->K > kMaxShells) return DGSM_EINVAL;
    if (d->spacing != DGSM_SHELLS_UNIFORM && d->spacing != DGSM_SHELLS_GEOMETRIC) return DGSM_EINVAL;
    if (!(d->r1 > 0.f)) return DGSM_EINVAL;
    if (d->spacing == DGSM_SHELLS_GEOMETRIC && !(d->r0 > 0.f && d->r0 < d->r1)) return DGSM_EINVAL;
    if (d->dtype != DGSM_F32 && d->dtype != DGSM_F16) return DGSM_EINVAL;
    if (!(d->cull_eps >= 0.f)) return DGSM_EINVAL;
    return DGSM_OK;
}

inline dgsm_status validate_lights(const dgsm_lights_t* l) {
    if (!l || !l->pos || l->n < 1) return DGSM_EINVAL;
    if (!(l->kappa >= 0.f)) return DGSM_EINVAL;
    return DGSM_OK;
}

inline dgsm_status validate_gaussians(const dgsm_gaussians_t* g) {
    if (!g || g->n < 0) return DGSM_EINVAL;
    if (g->n > 0 && (!g->mean || !g->scale || !g->rot || !g->opacity)) return DGSM_EINVAL;
    if (g->n >= (int64_t)INT32_MAX) return DGSM_EUNSUPPORTED;
    return DGSM_OK;
}

struct BuildLayout {
    int nb;            // preprocess blocks
    size_t tcone, scone, totals, rec, cone, mask, counts, lists;
    size_t total;
};

BuildLayout build_layout(const Geom& g, int64_t n);
size_t tile_smem_bytes(const Geom& g);
dgsm_status build_geometry(const Geom& g, const BuildLayout& L, unsigned char* ws, hipStream_t st);
dgsm_status build_light(const Geom& g, const BuildLayout& L, unsigned char* ws, const float* light_pos,
                        float kappa, float cull_eps, const dgsm_gaussians_t& gs, void* atlas_l,
                        hipStream_t st);
hipError_t launch_query(const Geom& g, const float* lights, int L, const void* atlas, const float* points,
                        int64_t P, float* T, hipStream_t st);

}  // namespace dgsm
