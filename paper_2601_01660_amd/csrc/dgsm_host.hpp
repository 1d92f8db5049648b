// Host-side helpers of the DGSM C ABI: argument validation and workspace layout.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dgsm.h"
#include "dgsm_device.hpp"

namespace dgsm {

constexpr int kMaxShells = 256;      // 4 shells per lane of a wave

inline dgsm_status validate_desc(const dgsm_atlas_desc_t* d) {
    if (!d) return DGSM_EINVAL;
    if (d->param == DGSM_PARAM_OCTAHEDRAL) {
        if (d->H < 2 || d->W < 2 || (d->H & 1) || (d->W & 1)) return DGSM_EINVAL;
    } else if (d->param == DGSM_PARAM_CUBEMAP) {
        if (d->H < 4 || (d->H & 1) || 2 * d->W != 3 * d->H) return DGSM_EINVAL;
    } else {
        return DGSM_EINVAL;
    }
    if (d->H > kMaxAtlasSide || d->W > kMaxAtlasSide) return DGSM_EINVAL;
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
    if (l->beta_mode < DGSM_BETA_TRACE || l->beta_mode > DGSM_BETA_DENSITY) return DGSM_EINVAL;
    return DGSM_OK;
}

inline dgsm_status validate_gaussians(const dgsm_gaussians_t* g) {
    if (!g || g->n < 0) return DGSM_EINVAL;
    if (g->n > 0 && (!g->mean || !g->scale || !g->rot || !g->opacity)) return DGSM_EINVAL;
    if (g->n >= (int64_t)INT32_MAX) return DGSM_EUNSUPPORTED;
    return DGSM_OK;
}

// Workspace of the build: shared atlas geometry, then one slice per light.
struct BuildLayout {
    int nb;                  // preprocess blocks (256 Gaussians each)
    size_t cap;              // list / bitmap capacity per light (entries)
    size_t tcone, scone;     // absolute offsets: tile cones [ntiles], supertile cones [kMaxSuper]
    size_t qcone;            // absolute offset: cones of 2x2-tile quads [ceil(TH/2) * ceil(TW/2)]
    size_t gcone;            // absolute offset: cones of 2x2-supertile groups [kMaxSuper / 4]
    size_t tcos, scos, qcos, gcos;   // absolute offsets: cone_cos of each cone above
    size_t light0;           // absolute offset of light 0's slice
    size_t light_stride;     // bytes per light slice
    int units_cap;           // extra work units per light (tiles split over several blocks)
    // offsets inside a light slice
    size_t totals, lbase, rec, cone, mask, counts, lists, bits;
    size_t hits, tinfo, units, splits, nunits, part, prange, roi_mask, roi_k, roi_super, need;
    size_t total;            // bytes for all lights
};

// Pointers into one light's slice of the workspace.
struct LightWs {
    int* totals;       // [kMaxSuper] list length per supertile
    int* lbase;        // [kMaxSuper + 1] list base per supertile, multiples of 64
    GRec* rec;         // [n]
    float4* cone;      // [n]
    uint64_t* mask;    // [n][kMaskWords] supertile masks
    int* counts;       // [S][nb] per-block counts, scanned in place
    int* lists;        // [cap] supertile lists, 64-entry chunks
    uint64_t* bits;    // [cap] per supertile: [tile][chunk] hit words
    int* hits;         // [ntiles] set bits over a tile's hit words
    int4* tinfo;       // [ntiles] {slices, first partial (-1: not split), words, 0}
    int4* units;       // [units_cap] extra slices: {tile, slice index, slices, partial}
    int2* splits;      // [units_cap] split tiles: {tile, first partial}
    int* nunits;       // [4] {extra slices, split tiles, hits per slice, total hits}
    unsigned long long* part;   // [2 units_cap][K][64] fixed-point partial optical depths (at least H W
                                // bytes: before the binning of a receiver-region build, the texel marks)
    int2* prange;               // [2 units_cap] shell rows [lo, hi] each partial holds (lo > hi: none)
    unsigned long long* roi_mask;   // [ntiles] receiver texels of each tile (bit = texel in the tile)
    int* roi_k;                     // [2] receiver shell range {k_min, k_max}
    int* roi_super;                 // [kMaxSuper] 1 where a supertile holds a receiver texel
    int* need;                      // [2] {list entries the last binning needed, 1 if they exceeded cap}
};

__host__ __device__ inline LightWs light_ws(unsigned char* ws, const BuildLayout& L, int l) {
    unsigned char* b = ws + L.light0 + (size_t)l * L.light_stride;
    return LightWs{reinterpret_cast<int*>(b + L.totals), reinterpret_cast<int*>(b + L.lbase),
                   reinterpret_cast<GRec*>(b + L.rec), reinterpret_cast<float4*>(b + L.cone),
                   reinterpret_cast<uint64_t*>(b + L.mask), reinterpret_cast<int*>(b + L.counts),
                   reinterpret_cast<int*>(b + L.lists), reinterpret_cast<uint64_t*>(b + L.bits),
                   reinterpret_cast<int*>(b + L.hits), reinterpret_cast<int4*>(b + L.tinfo),
                   reinterpret_cast<int4*>(b + L.units), reinterpret_cast<int2*>(b + L.splits),
                   reinterpret_cast<int*>(b + L.nunits), reinterpret_cast<unsigned long long*>(b + L.part),
                   reinterpret_cast<int2*>(b + L.prange),
                   reinterpret_cast<unsigned long long*>(b + L.roi_mask), reinterpret_cast<int*>(b + L.roi_k),
                   reinterpret_cast<int*>(b + L.roi_super), reinterpret_cast<int*>(b + L.need)};
}

// Workspace layout for n Gaussians and n_lights lights.  cap: list entries
// per light (supertile lists and hit words); negative = the worst case
// n S + 64 S, which every set of n Gaussians fits.
BuildLayout build_layout(const Geom& g, int64_t n, int n_lights, int64_t cap = -1);
// The layout a workspace of ws_bytes holds: the worst case if it fits,
// otherwise the largest list capacity (a multiple of 64, at least 64 S) that
// does; false if not even that fits.
bool layout_for_bytes(const Geom& g, int64_t n, int n_lights, size_t ws_bytes, BuildLayout& out);
size_t tile_smem_bytes(const Geom& g, int nw, bool pack);

// Tile and supertile cones of the atlas geometry (depend on the atlas only).
dgsm_status enqueue_cones(const Geom& g, const BuildLayout& L, unsigned char* ws, hipStream_t st);

// Enqueue the binning of all lights (preprocess, scan, scatter, tile masks);
// cones = false reuses cones already in the workspace; roi = true bins only
// the tiles of a receiver region already marked (enqueue_roi).
dgsm_status enqueue_bin(const Geom& g, const BuildLayout& L, unsigned char* ws, const dgsm_lights_t& lights,
                        float cull_eps, const dgsm_gaussians_t& gs, hipStream_t st, bool cones = true,
                        bool shape_cached = false, bool roi = false);

// Options of the per-tile accumulation.
struct AccumOpts {
    const float* base_tau;   // optional [L][K][H][W] FP32 optical depth added before exp (may be null)
    bool write_tau;          // store tau (FP32) instead of T
    unsigned long long* stats;   // optional device counters [4]
    int tile_waves;              // waves sharing one tile: 2, 4 or 8
    int split_units;             // target work units per launch (all lights); <= 0: never split a tile
    bool tiled = false;          // atlas / base_tau planes in tile-major order (see kTile)
    bool skip_empty = false;     // leave tiles without hits untouched (their atlas values stay as they are)
    bool roi = false;            // receiver region: T = 1 outside the marked texels and shell range
    bool pack = false;           // packed walk: only pairs past the distance pre-test, 64 per wave (no stats)
};

// Receiver box of the region of interest (Sec. 3.2): |x - cx|, |y - cy| <= half,
// zmin <= z <= zmax; half <= 0 takes every receiver point.
struct RoiBox {
    float cx, cy, half, zmin, zmax;
};

// Mark the receiver region of every light: the texels and shells the
// trilinear lookup of each receiver point inside the box reads.
dgsm_status enqueue_roi(const Geom& g, const BuildLayout& L, unsigned char* ws, const dgsm_lights_t& lights,
                        const float* points, int64_t n_points, const RoiBox& box, hipStream_t st);

// Elements of one shell plane: H*W row-major, or ntiles*64 tile-major (each
// 8x8 tile's texels contiguous, row-major inside the tile).
__host__ __device__ inline size_t plane_elems(const Geom& g, bool tiled) {
    return tiled ? (size_t)g.ntiles * kWave : (size_t)g.H * g.W;
}

constexpr int kDefaultTileWaves = 8;
constexpr int kDefaultSplitUnits = 32768;

// Enqueue the per-tile accumulation of all lights into atlas [L][K][H][W].
dgsm_status enqueue_accumulate(const Geom& g, const BuildLayout& L, unsigned char* ws, int n_lights,
                               float pair_eps, void* atlas, const AccumOpts& o, hipStream_t st);
// T [L][P] (light-major, row stride ld or P), or [P][L] (point-major) with point_major.
hipError_t launch_query(const Geom& g, const float* lights, int L, const void* atlas, const float* points,
                        int64_t P, float* T, hipStream_t st, bool tiled = false,
                        const int* out_index = nullptr, bool point_major = false, int64_t ld = 0);
// Points that never move indexed by the tiles their lookups read (tiled
// atlas).  With offs == nullptr: counts[l][tile] += entries; else idx[offs[b]
// + counts[b]++] = point for every (light, tile) bucket b of every point
// (counts zeroed before each pass).
hipError_t launch_point_buckets(const Geom& g, const float* lights, int L, const float* points, int64_t P,
                                int* counts, const int* offs, int* idx, hipStream_t st);
// For every tile with a nonzero count in hits (light l's int array at hits0 +
// l * hits_stride bytes): the lookups of its bucket's points in the tiled
// atlas into T[l][out_col[p]] (row stride ld), each point once.  chunks:
// {bucket, first entry} of every 256-entry piece of every bucket.
hipError_t launch_patch(const Geom& g, const float* lights, int L, const void* atlas, const float* points,
                        const unsigned char* hits0, size_t hits_stride, const int* offs, const int2* chunks,
                        int64_t nchunks, const int* idx, const int* out_col, float* T, int64_t ld, hipStream_t st);
// dst[r][i] = src[r][i] for r < rows, i < n (dst row stride ld)
hipError_t launch_copy_rows(const float* src, int64_t n, int rows, float* dst, int64_t ld, hipStream_t st);

}  // namespace dgsm
