// Batched DGSM: many lights x animation frames in one captured HIP graph.
//
// A plan owns every buffer it needs (allocated once, at creation).  One run
// processes F frames of a scene made of a static Gaussian set and a dynamic
// set that either moves rigidly, one translation per group of Gaussians per
// frame (several avatars on their own trajectories), or takes new means,
// scales, rotations and opacities every frame (free motion):
//   per frame f: the dynamic Gaussians of frame f; build the atlas of every
//   light from all Gaussians; query T at all Gaussian centres into T_out[f].
// With the static cache on, the optical depth of the static set is built once
// per run (it does not change between frames) and each frame only bins and
// accumulates the dynamic Gaussians on top of it: tau = tau_static +
// tau_dynamic is exact because Eq. 2 is a sum over Gaussians.
// The plan's own atlas and static optical depth store each shell plane in
// tile-major order (the texels of an 8x8 tile contiguous): a tile's store is
// one 128/256-byte run per shell, and most trilinear lookups stay inside one
// tile, so a shell's two texel rows come from one cache line.
// In cache mode the frames alternate between independent chains of buffers
// on their own streams (see kMaxChains), so that the short launches of one
// frame overlap the tile build of the next.
// The whole run (static build + all frames) is captured once into a hipGraph
// and replayed; the knobs of the tile accumulation (waves per tile, work
// units per launch) are chosen on the first run by timing each candidate pair
// on frame 0 of the real workload.

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

namespace dgsm {

// dst = base + t of the Gaussian's group (one FP32 addition per coordinate);
// group: [n] group index of each Gaussian, or null for a single group.
__global__ __launch_bounds__(256) void translate_kernel(const float* __restrict__ base, int64_t n,
                                                        const float* __restrict__ t,
                                                        const unsigned short* __restrict__ group,
                                                        float* __restrict__ dst) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= 3 * n) return;
    const int c = (int)(i % 3);
    const int gi = group ? (int)group[i / 3] : 0;
    dst[i] = base[i] + t[3 * gi + c];
}

__global__ __launch_bounds__(256) void group_index_kernel(unsigned short* __restrict__ group, int64_t from,
                                                          int64_t to, int gi) {
    const int64_t i = from + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < to) group[i] = (unsigned short)gi;
}

// Frames of a cached run are spread over up to kMaxChains independent chains
// (frame f on chain f mod chains), each on its own stream with its own atlas,
// query staging, means and dynamic workspace: one frame's short binning,
// finish, query and restore launches overlap another frame's tile build.
constexpr int kMaxChains = 3;

// T of the static set alone, T = exp(-tau_static) with the running minimum
// over shells (the same arithmetic as the tile build's finish of a tile that
// no dynamic Gaussian reaches), into its baseline copy and into the atlas of
// every chain (atlas[c] null past the plan's chains).
template <typename OutT>
struct ChainAtlases {
    OutT* a[kMaxChains];
};

template <typename OutT>
__global__ __launch_bounds__(kWave) void static_finish_kernel(Geom g, const float* __restrict__ tau,
                                                              ChainAtlases<OutT> atlas, OutT* __restrict__ base) {
    const int tile = blockIdx.x, light = blockIdx.y, lane = threadIdx.x;
    const int ty = tile / g.TW, tx = tile - ty * g.TW;
    if (ty * kTile + (lane >> 3) >= g.H || tx * kTile + (lane & 7) >= g.W) return;
    const size_t plane = plane_elems(g, true);
    const size_t off = (size_t)light * g.K * plane + (size_t)tile * kWave + lane;
    float Tp = 1.f;
    for (int k = 0; k < g.K; ++k) {
        const float T = fminf(__expf(-tau[off + (size_t)k * plane]), Tp);
        Tp = T;
        Store<OutT>::put(base + off + (size_t)k * plane, T);
#pragma unroll
        for (int c = 0; c < kMaxChains; ++c)
            if (atlas.a[c]) Store<OutT>::put(atlas.a[c] + off + (size_t)k * plane, T);
    }
}

// After a frame's query: tiles the dynamic set reached get their static-only
// values back, so that the next frame starts from the baseline again.
template <typename OutT>
__global__ __launch_bounds__(kWave) void restore_kernel(Geom g, BuildLayout lay, unsigned char* ws,
                                                        const OutT* __restrict__ base, OutT* __restrict__ atlas) {
    const int tile = blockIdx.x, light = blockIdx.y, lane = threadIdx.x;
    const LightWs W = light_ws(ws, lay, light);
    if (W.hits[tile] == 0) return;
    const size_t plane = plane_elems(g, true);
    const size_t off = (size_t)light * g.K * plane + (size_t)tile * kWave + lane;
    for (int k = 0; k < g.K; ++k) atlas[off + (size_t)k * plane] = base[off + (size_t)k * plane];
}

// ---------------------------------------------------------------------------
// Spatial order of the static set (once, at plan creation).  Gaussians that
// are close in space are close in every light's supertile lists, so a tile's
// hits gather into few hit words and its records share cache lines, and
// queries of neighbouring points read neighbouring texels.  Keys: 30-bit
// Morton code of the mean in the set's bounding box, then the index (unique,
// so the order is deterministic); bitonic sort over the next power of two.
// The atlas does not depend on the order (the per-shell sums are integers).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void bbox_partial_kernel(const float* __restrict__ mean, int64_t n,
                                                           float* __restrict__ part) {
    __shared__ float red[6][256];
    const int tid = threadIdx.x;
    float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
    for (int64_t i = (int64_t)blockIdx.x * 256 + tid; i < n; i += (int64_t)gridDim.x * 256)
        for (int c = 0; c < 3; ++c) {
            lo[c] = fminf(lo[c], mean[3 * i + c]);
            hi[c] = fmaxf(hi[c], mean[3 * i + c]);
        }
    for (int c = 0; c < 3; ++c) {
        red[c][tid] = lo[c];
        red[3 + c][tid] = hi[c];
    }
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h)
            for (int c = 0; c < 3; ++c) {
                red[c][tid] = fminf(red[c][tid], red[c][tid + h]);
                red[3 + c][tid] = fmaxf(red[3 + c][tid], red[3 + c][tid + h]);
            }
        __syncthreads();
    }
    if (tid < 6) part[blockIdx.x * 6 + tid] = red[tid][0];
}

__device__ inline uint32_t spread_bits10(uint32_t v) {      // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ __launch_bounds__(256) void morton_kernel(const float* __restrict__ mean, int64_t n,
                                                     const float* __restrict__ part, int nparts,
                                                     uint64_t* __restrict__ keys, int64_t npad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npad) return;
    if (i >= n) {
        keys[i] = ~0ull;
        return;
    }
    uint32_t code = 0;
    for (int c = 0; c < 3; ++c) {
        float lo = 3e38f, hi = -3e38f;
        for (int b = 0; b < nparts; ++b) {
            lo = fminf(lo, part[6 * b + c]);
            hi = fmaxf(hi, part[6 * b + 3 + c]);
        }
        const float ext = hi - lo;
        const float f = ext > 0.f ? (mean[3 * i + c] - lo) / ext : 0.f;
        const uint32_t q = (uint32_t)fminf(fmaxf(f * 1024.f, 0.f), 1023.f);
        code |= spread_bits10(q) << c;
    }
    keys[i] = ((uint64_t)code << 32) | (uint64_t)i;
}

__global__ __launch_bounds__(256) void bitonic_kernel(uint64_t* __restrict__ keys, int64_t npad, int64_t j,
                                                      int64_t k) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npad) return;
    const int64_t l = i ^ j;
    if (l <= i) return;
    const uint64_t a = keys[i], b = keys[l];
    const bool up = (i & k) == 0;
    if ((a > b) == up) {
        keys[i] = b;
        keys[l] = a;
    }
}

// Sorted static set into the plan's arrays; out_index maps sorted position to
// the caller's index (the query writes each result to the caller's column).
__global__ __launch_bounds__(256) void gather_static_kernel(dgsm_gaussians_t src, const uint64_t* __restrict__ keys,
                                                            float* mean, float* scale, float* rot, float* opacity,
                                                            int* out_index) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= src.n) return;
    const int64_t s = (int64_t)(keys[p] & 0xffffffffull);
    for (int c = 0; c < 3; ++c) {
        mean[3 * p + c] = src.mean[3 * s + c];
        scale[3 * p + c] = src.scale[3 * s + c];
    }
    for (int c = 0; c < 4; ++c) rot[4 * p + c] = src.rot[4 * s + c];
    opacity[p] = src.opacity[s];
    out_index[p] = (int)s;
}

// Inverse of the point order: in_pos[caller column] = plan position.
__global__ __launch_bounds__(256) void invert_kernel(const int* __restrict__ out_index, int64_t n,
                                                     int* __restrict__ in_pos) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < n) in_pos[out_index[p]] = (int)p;
}

// Frame results from the point-major staging [np][L] (plan order) into the
// caller's [L][np]: thread i gathers caller point i's L values (one contiguous
// read) and writes them coalesced, one light after another.
__global__ __launch_bounds__(256) void unstage_kernel(const float* __restrict__ tq, const int* __restrict__ in_pos,
                                                      int64_t n, int L, float* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float* src = tq + (size_t)in_pos[i] * L;
    if (L == 4) {
        const float4 v = *reinterpret_cast<const float4*>(src);
        out[i] = v.x;
        out[n + i] = v.y;
        out[2 * n + i] = v.z;
        out[3 * n + i] = v.w;
    } else {
        for (int l = 0; l < L; ++l) out[(size_t)l * n + i] = src[l];
    }
}

__global__ __launch_bounds__(256) void iota_kernel(int* __restrict__ v, int64_t from, int64_t to) {
    const int64_t i = from + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < to) v[i] = (int)i;
}

}  // namespace dgsm

using namespace dgsm;

struct dgsm_plan_s {
    Geom g;
    dgsm_atlas_desc_t desc;
    int L;
    float kappa;
    int beta_mode;
    int64_t ns, nd, np;
    int frames;
    bool cache;
    int autotune;
    int tile_waves;
    int split_units;
    bool tuned;
    bool tuned_cached;    // the knobs came from the tuning cache
    int pack;             // packed walk for the dynamic accumulation (cache mode)
    int static_waves;     // knobs of the once-per-run static build (cache mode)
    int static_units;
    int motion;           // DGSM_MOTION_RIGID or DGSM_MOTION_FREE
    int groups;           // rigid groups of the dynamic set
    unsigned short* group;   // [nd] group of each dynamic Gaussian (null: one group)
    BuildLayout lay_a;    // workspace of the static set (cache mode) or of the whole set
    BuildLayout lay_b;    // workspace of the dynamic set (cache mode)
    // device buffers owned by the plan
    float* lights;        // [L][3]
    float* mean;          // [ns + nd][3]: static means, then this frame's dynamic means
    float* scale;         // [ns + nd][3]
    float* rot;           // [ns + nd][4]
    float* opacity;       // [ns + nd]
    int* out_index;       // [ns + nd] caller column of each plan point (static part in spatial order)
    int* in_pos;          // [ns + nd] plan position of each caller column (without the cache)
    float* tq;            // [ns + nd][L] one frame's query results in plan order (point-major; without the cache)
    float* tau_static;    // [L][K][H][W] (cache mode)
    float* ts;            // [L][ns] cache mode: T of the static points in the static-only atlas (caller order)
    int* boffs;           // [L ntiles + 1] cache mode: static points per (light, tile) bucket, offsets
    int* bidx;            // cache mode: static points (plan order) of each bucket
    int2* bchunk;         // cache mode: {bucket, first entry} of every 256-entry piece of a bucket
    int64_t nchunks;
    void* atlas;          // [L][K][plane] of desc.dtype (tile-major planes)
    void* atlas_static;   // cache mode: T of the static set alone (the per-frame baseline)
    unsigned char* ws_a;  // workspace for the static (cache) or full (no cache) set
    size_t ws_a_bytes;
    unsigned char* ws_b;  // workspace for the dynamic set (cache mode)
    size_t ws_b_bytes;
    // frame chains (cache mode): chain 0 uses mean, tq, atlas, ws_b and the
    // caller's stream; chain c > 0 its own copies and stream, forked from and
    // joined back into the caller's stream around the frames
    int chains;
    float* cmean[kMaxChains];
    float* ctq[kMaxChains];
    void* catlas[kMaxChains];
    unsigned char* cws[kMaxChains];
    hipStream_t cstream[kMaxChains];
    hipEvent_t ev_fork, ev_join[kMaxChains];
    // captured graph and the arguments it was captured for
    hipGraphExec_t exec;
    const void* cap_key[6];
};

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t bytes) {
    return hipMalloc(reinterpret_cast<void**>(p), bytes ? bytes : 256);
}

void plan_free(dgsm_plan p) {
    if (!p) return;
    // a run may still be in flight on the caller's stream or the chain streams
    (void)hipDeviceSynchronize();
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    void* bufs[] = {p->lights,     p->mean,  p->scale,        p->rot,  p->opacity, p->out_index,
                    p->tau_static, p->atlas, p->atlas_static, p->ws_a, p->ws_b,    p->in_pos,
                    p->tq,         p->group, p->ts,           p->boffs, p->bidx,    p->bchunk};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    for (int c = 1; c < kMaxChains; ++c) {
        void* cb[] = {p->cmean[c], p->ctq[c], p->catlas[c], p->cws[c]};
        for (void* b : cb)
            if (b) (void)hipFree(b);
        if (p->cstream[c]) (void)hipStreamDestroy(p->cstream[c]);
        if (p->ev_join[c]) (void)hipEventDestroy(p->ev_join[c]);
    }
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    delete p;
}

dgsm_gaussians_t set_of(const dgsm_plan p, const float* mean, int64_t off, int64_t n) {
    return dgsm_gaussians_t{mean + 3 * off, p->scale + 3 * off, p->rot + 4 * off, p->opacity + off, n};
}

// Static part of a run: tau of the static set for every light.
dgsm_status enqueue_static(dgsm_plan p, int tile_waves, int split_units, hipStream_t st, hipEvent_t* ev = nullptr) {
    const dgsm_lights_t lt{p->lights, p->L, p->kappa, p->beta_mode};
    const BuildLayout& La = p->lay_a;
    dgsm_status s = enqueue_bin(p->g, La, p->ws_a, lt, p->desc.cull_eps, set_of(p, p->mean, 0, p->ns), st, false);
    if (s != DGSM_OK) return s;
    if (ev) (void)hipEventRecord(ev[0], st);
    AccumOpts o{nullptr, true, nullptr, tile_waves, split_units, true};
    s = enqueue_accumulate(p->g, La, p->ws_a, p->L, p->desc.cull_eps, p->tau_static, o, st);
    if (s != DGSM_OK) return s;
    if (ev) (void)hipEventRecord(ev[1], st);
    const dim3 grid(p->g.ntiles, p->L);
    if (p->desc.dtype == DGSM_F16) {
        ChainAtlases<__half> a{};
        for (int c = 0; c < p->chains; ++c) a.a[c] = static_cast<__half*>(p->catlas[c]);
        static_finish_kernel<__half><<<grid, kWave, 0, st>>>(p->g, p->tau_static, a, static_cast<__half*>(p->atlas_static));
    } else {
        ChainAtlases<float> a{};
        for (int c = 0; c < p->chains; ++c) a.a[c] = static_cast<float*>(p->catlas[c]);
        static_finish_kernel<float><<<grid, kWave, 0, st>>>(p->g, p->tau_static, a, static_cast<float*>(p->atlas_static));
    }
    if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    // T of the static points (they never move) in the static-only atlas, in
    // the caller's columns: every frame starts from these
    return launch_query(p->g, p->lights, p->L, p->atlas_static, p->mean, p->ns, p->ts, st, true, p->out_index,
                        false) == hipSuccess
               ? DGSM_OK
               : DGSM_EHIP;
}

// One frame on chain c (its stream st): dynamic means, build (on top of the
// static tau in cache mode), query, and in cache mode the restore of the
// chain's atlas to the static baseline.
dgsm_status enqueue_frame(dgsm_plan p, int f, int c, const dgsm_gaussians_t* dyn_base, const float* translations,
                          float* T_out, int tile_waves, int split_units, int pack, hipStream_t st,
                          hipEvent_t* ev = nullptr) {
    // ev (optional, 5 events): recorded before the dynamic binning, before the
    // accumulation, before the query, before the restore and at the end
    auto mark = [&](int i) { if (ev) (void)hipEventRecord(ev[i], st); };
    mark(0);
    const dgsm_lights_t lt{p->lights, p->L, p->kappa, p->beta_mode};
    float* mean = p->cmean[c];
    void* atlas = p->catlas[c];
    unsigned char* ws_b = p->cws[c];
    const bool rigid = p->motion == DGSM_MOTION_RIGID;
    // the dynamic Gaussians of this frame: rigid motion moves the base means
    // (shape in the plan's arrays); free motion takes frame f of the caller's arrays
    dgsm_gaussians_t dyn{mean + 3 * p->ns, p->scale + 3 * p->ns, p->rot + 4 * p->ns, p->opacity + p->ns, p->nd};
    if (p->nd > 0) {
        const int64_t n3 = 3 * p->nd;
        if (rigid) {
            translate_kernel<<<(unsigned)((n3 + 255) / 256), 256, 0, st>>>(
                dyn_base->mean, p->nd, translations + (size_t)3 * p->groups * f, p->group, mean + 3 * p->ns);
            if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
        } else {
            const size_t fo = (size_t)f * p->nd;
            if (hipMemcpyAsync(mean + 3 * p->ns, dyn_base->mean + 3 * fo, 12 * p->nd, hipMemcpyDeviceToDevice, st) !=
                hipSuccess)
                return DGSM_EHIP;
            dyn.scale = dyn_base->scale + 3 * fo;
            dyn.rot = dyn_base->rot + 4 * fo;
            dyn.opacity = dyn_base->opacity + fo;
            if (!p->cache &&   // the whole set is binned from the plan's arrays: this frame's shapes into them
                (hipMemcpyAsync(p->scale + 3 * p->ns, dyn.scale, 12 * p->nd, hipMemcpyDeviceToDevice, st) !=
                     hipSuccess ||
                 hipMemcpyAsync(p->rot + 4 * p->ns, dyn.rot, 16 * p->nd, hipMemcpyDeviceToDevice, st) != hipSuccess ||
                 hipMemcpyAsync(p->opacity + p->ns, dyn.opacity, 4 * p->nd, hipMemcpyDeviceToDevice, st) !=
                     hipSuccess))
                return DGSM_EHIP;
        }
    }
    dgsm_status s;
    if (p->cache) {
        const BuildLayout& Lb = p->lay_b;
        // rigid motion: from the chain's second frame of the run on, the
        // dynamic records keep their shape part and only the light-to-mean
        // offsets change
        s = enqueue_bin(p->g, Lb, ws_b, lt, p->desc.cull_eps, dyn, st, false, rigid && f >= p->chains);
        if (s != DGSM_OK) return s;
        mark(1);
        // only tiles the dynamic set reaches are rebuilt; the rest hold the static baseline
        AccumOpts o{p->tau_static, false, nullptr, tile_waves, split_units, true, true};
        o.pack = pack != 0;
        s = enqueue_accumulate(p->g, Lb, ws_b, p->L, p->desc.cull_eps, atlas, o, st);
    } else {
        const BuildLayout& La = p->lay_a;
        s = enqueue_bin(p->g, La, p->ws_a, lt, p->desc.cull_eps, set_of(p, mean, 0, p->np), st, false);
        if (s != DGSM_OK) return s;
        mark(1);
        AccumOpts o{nullptr, false, nullptr, tile_waves, split_units, true};
        s = enqueue_accumulate(p->g, La, p->ws_a, p->L, p->desc.cull_eps, atlas, o, st);
    }
    if (s != DGSM_OK) return s;
    mark(2);
    float* Tf = T_out + (size_t)f * p->L * p->np;
    if (p->cache) {
        // A tile the dynamic set did not reach holds the static baseline, so a
        // static point whose footprint lies in such tiles has its once-per-run
        // static value: the frame starts from those and looks up again only
        // the static points listed under reached tiles, then the dynamic
        // points (whose plan order is the caller's).
        const BuildLayout& Lb = p->lay_b;
        if (launch_copy_rows(p->ts, p->ns, p->L, Tf, p->np, st) != hipSuccess ||
            launch_patch(p->g, p->lights, p->L, atlas, mean, ws_b + Lb.light0 + Lb.hits, Lb.light_stride, p->boffs,
                         p->bchunk, p->nchunks, p->bidx, p->out_index, Tf, p->np, st) != hipSuccess ||
            launch_query(p->g, p->lights, p->L, atlas, mean + 3 * p->ns, p->nd, Tf + p->ns, st, true, nullptr,
                         false, p->np) != hipSuccess)
            return DGSM_EHIP;
    } else {
        // Query in plan (spatial) order with coalesced point-major writes, then
        // one gather into the caller's order: writing straight to the caller's
        // columns scatters 4-byte stores over the whole output.
        if (launch_query(p->g, p->lights, p->L, atlas, mean, p->np, p->ctq[c], st, true, nullptr, true) != hipSuccess)
            return DGSM_EHIP;
        if (p->np > 0) {
            unstage_kernel<<<(unsigned)((p->np + 255) / 256), 256, 0, st>>>(p->ctq[c], p->in_pos, p->np, p->L, Tf);
            if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
        }
    }
    mark(3);
    if (p->cache) {
        const BuildLayout& Lb = p->lay_b;
        const dim3 grid(p->g.ntiles, p->L);
        if (p->desc.dtype == DGSM_F16)
            restore_kernel<__half><<<grid, kWave, 0, st>>>(p->g, Lb, ws_b, static_cast<const __half*>(p->atlas_static),
                                                           static_cast<__half*>(atlas));
        else
            restore_kernel<float><<<grid, kWave, 0, st>>>(p->g, Lb, ws_b, static_cast<const float*>(p->atlas_static),
                                                          static_cast<float*>(atlas));
        if (hipGetLastError() != hipSuccess) return DGSM_EHIP;
    }
    mark(4);
    return DGSM_OK;
}

// Frames 0 .. nf - 1 dealt round-robin to the chains: fork from st, the
// frames, join back into st.
dgsm_status enqueue_frames(dgsm_plan p, int nf, const dgsm_gaussians_t* dyn, const float* translations, float* T_out,
                           int tile_waves, int split_units, int pack, hipStream_t st) {
    // fork: every chain starts after what st holds (the static build and the copies)
    hipStream_t cs[kMaxChains];
    cs[0] = st;
    if (p->chains > 1 && hipEventRecord(p->ev_fork, st) != hipSuccess) return DGSM_EHIP;
    for (int c = 1; c < p->chains; ++c) {
        cs[c] = p->cstream[c];
        if (hipStreamWaitEvent(cs[c], p->ev_fork, 0) != hipSuccess) return DGSM_EHIP;
    }
    dgsm_status s = DGSM_OK;
    for (int f = 0; f < nf && s == DGSM_OK; ++f) {
        const int c = f % p->chains;
        s = enqueue_frame(p, f, c, dyn, translations, T_out, tile_waves, split_units, pack, cs[c]);
    }
    // join: the caller's stream waits for every chain (also after a failed
    // enqueue, so that a capture never ends with a stream left forked)
    for (int c = 1; c < p->chains; ++c)
        if (hipEventRecord(p->ev_join[c], cs[c]) != hipSuccess || hipStreamWaitEvent(st, p->ev_join[c], 0) != hipSuccess)
            return DGSM_EHIP;
    return s;
}

dgsm_status enqueue_run(dgsm_plan p, const dgsm_gaussians_t* dyn, const float* translations, float* T_out,
                        hipStream_t st) {
    if (p->nd > 0 && p->motion == DGSM_MOTION_RIGID) {
        const int64_t o = p->ns;
        if (hipMemcpyAsync(p->scale + 3 * o, dyn->scale, 12 * p->nd, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(p->rot + 4 * o, dyn->rot, 16 * p->nd, hipMemcpyDeviceToDevice, st) != hipSuccess ||
            hipMemcpyAsync(p->opacity + o, dyn->opacity, 4 * p->nd, hipMemcpyDeviceToDevice, st) != hipSuccess)
            return DGSM_EHIP;
    }
    dgsm_status s;
    // the static build is a full-scene accumulation: it keeps the defaults
    // (the tuned knobs fit the per-frame dynamic accumulation)
    if (p->cache && (s = enqueue_static(p, p->static_waves, p->static_units, st)) != DGSM_OK) return s;
    return enqueue_frames(p, p->frames, dyn, translations, T_out, p->tile_waves, p->split_units, p->pack, st);
}

// Knobs found by the autotuner, shared by the plans of the process: a plan
// whose workload matches an earlier one's (atlas H, W, K, spacing, storage and
// parameterisation, light count, cache mode, motion, and the static and
// dynamic Gaussian counts to the nearest power of two) takes its knobs without
// timing.  Guarded by a mutex; dgsm_autotune_cache_clear empties it.
struct TuneKnobs {
    int waves, units, pack, static_waves, static_units;
};
using TuneKey = std::tuple<int, int, int, int, int, int, int, int, int, int, int>;
std::mutex g_tune_mu;
std::map<TuneKey, TuneKnobs> g_tune;

int log2_bucket(int64_t n) {
    int b = 0;
    while (n > 1) {
        n >>= 1;
        ++b;
    }
    return b;
}

TuneKey tune_key(const dgsm_plan p) {
    return TuneKey{p->g.H, p->g.W, p->g.K, p->g.spacing, p->desc.dtype, p->g.param, p->L, p->cache ? 1 : 0,
                   p->motion, log2_bucket(p->ns), log2_bucket(p->nd)};
}

// Time each (waves per tile, work units, packed walk) candidate on the
// frames the run repeats: in cache mode a window of frames dealt to the
// chains as the run deals them (the chains overlap, and the knobs that win a
// lone frame need not win there: measured 1.086 vs 1.053 ms/frame), otherwise
// frame 0 (a full-scene build).
dgsm_status autotune(dgsm_plan p, const dgsm_gaussians_t* dyn, const float* translations, float* T_out,
                     hipStream_t st) {
    // 2 waves per tile and unsplit tiles never won a measurement (alone or
    // with overlapping chains) and are not candidates
    const int waves[2] = {4, 8};
    const int units[3] = {8192, 32768, 131072};
    const int npack = p->cache ? 2 : 1;   // the packed walk is a candidate for the dynamic accumulation
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return DGSM_EHIP;
    dgsm_status s = DGSM_OK;
    float best = 1e30f;
    int best_nw = kDefaultTileWaves, best_units = kDefaultSplitUnits, best_pack = 0;
    if (p->nd > 0 && p->motion == DGSM_MOTION_RIGID) {
        const int64_t o = p->ns;
        (void)hipMemcpyAsync(p->scale + 3 * o, dyn->scale, 12 * p->nd, hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(p->rot + 4 * o, dyn->rot, 16 * p->nd, hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(p->opacity + o, dyn->opacity, 4 * p->nd, hipMemcpyDeviceToDevice, st);
    }
    // the once-per-run static build (cache mode): 4 or 8 waves per tile x
    // 32768 or 131072 work units (a full-scene build; 2 waves and unsplit tiles
    // lose there), each timed once after a warm-up build with the defaults
    int best_sw = kDefaultTileWaves, best_su = kDefaultSplitUnits;
    if (p->cache && p->ns > 0) {
        const int swaves[2] = {4, 8}, sunits[2] = {32768, 131072};
        hipEvent_t ea[2];
        if (hipEventCreate(&ea[0]) != hipSuccess || hipEventCreate(&ea[1]) != hipSuccess) return DGSM_EHIP;
        float sbest = 1e30f;
        for (int c = -1; c < 4 && s == DGSM_OK; ++c) {
            const int nw = c < 0 ? kDefaultTileWaves : swaves[c % 2], nu = c < 0 ? kDefaultSplitUnits : sunits[c / 2];
            s = enqueue_static(p, nw, nu, st, ea);
            if (s == DGSM_OK && hipEventSynchronize(ea[1]) != hipSuccess) s = DGSM_EHIP;
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ea[0], ea[1]);
            if (c >= 0 && ms < sbest) {
                sbest = ms;
                best_sw = nw;
                best_su = nu;
            }
        }
        (void)hipEventDestroy(ea[0]);
        (void)hipEventDestroy(ea[1]);
    }
    p->static_waves = best_sw;
    p->static_units = best_su;
    if (p->cache && s == DGSM_OK) s = enqueue_static(p, best_sw, best_su, st);
    const int window = p->cache ? std::min(p->frames, 3 * p->chains) : 1;
    // c = -1: one warm-up window with the defaults, then each candidate once
    for (int c = -1; c < 6 * npack && s == DGSM_OK; ++c) {
        const int nw = c < 0 ? kDefaultTileWaves : waves[c % 2], nu = c < 0 ? kDefaultSplitUnits : units[(c / 2) % 3],
                  pk = c < 0 ? 0 : c / 6;
        (void)hipEventRecord(e0, st);
        s = enqueue_frames(p, window, dyn, translations, T_out, nw, nu, pk, st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess) s = DGSM_EHIP;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (c >= 0 && ms < best) {
            best = ms;
            best_nw = nw;
            best_units = nu;
            best_pack = pk;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->tile_waves = best_nw;
    p->split_units = best_units;
    p->pack = best_pack;
    p->tuned = true;
    if (s == DGSM_OK) {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[tune_key(p)] = TuneKnobs{best_nw, best_units, best_pack, p->static_waves, p->static_units};
    }
    return s;
}

// Knobs of an earlier plan with the same workload, if any.
bool tune_from_cache(dgsm_plan p) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(tune_key(p));
    if (it == g_tune.end()) return false;
    p->tile_waves = it->second.waves;
    p->split_units = it->second.units;
    p->pack = it->second.pack;
    p->static_waves = it->second.static_waves;
    p->static_units = it->second.static_units;
    p->tuned = true;
    p->tuned_cached = true;
    return true;
}

// Static set into the plan in spatial order (see bitonic_kernel); synchronous.
dgsm_status sort_static(dgsm_plan p, const dgsm_gaussians_t& src) {
    const int64_t n = src.n;
    int64_t npad = 1;
    while (npad < n) npad <<= 1;
    const int nparts = 256;
    float* part = nullptr;
    uint64_t* keys = nullptr;
    bool ok = dalloc(&part, sizeof(float) * 6 * nparts) == hipSuccess &&
              dalloc(&keys, sizeof(uint64_t) * (size_t)npad) == hipSuccess;
    if (ok) {
        bbox_partial_kernel<<<nparts, 256>>>(src.mean, n, part);
        morton_kernel<<<(unsigned)((npad + 255) / 256), 256>>>(src.mean, n, part, nparts, keys, npad);
        for (int64_t k = 2; k <= npad; k <<= 1)
            for (int64_t j = k >> 1; j > 0; j >>= 1)
                bitonic_kernel<<<(unsigned)((npad + 255) / 256), 256>>>(keys, npad, j, k);
        gather_static_kernel<<<(unsigned)((n + 255) / 256), 256>>>(src, keys, p->mean, p->scale, p->rot, p->opacity,
                                                                    p->out_index);
        ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
    if (part) (void)hipFree(part);
    if (keys) (void)hipFree(keys);
    return ok ? DGSM_OK : DGSM_EHIP;
}

// Static points per (light, tile) bucket of the tiles their lookups read
// (once, at plan creation: the points and lights never change).
dgsm_status bucket_static(dgsm_plan p) {
    const size_t nb = (size_t)p->L * p->g.ntiles;
    int* counts = nullptr;
    if (dalloc(&p->boffs, 4 * (nb + 1)) != hipSuccess || dalloc(&counts, 4 * nb) != hipSuccess) {
        if (counts) (void)hipFree(counts);
        return DGSM_EHIP;
    }
    std::vector<int> h(nb + 1, 0);
    bool ok = hipMemset(counts, 0, 4 * nb) == hipSuccess &&
              launch_point_buckets(p->g, p->lights, p->L, p->mean, p->ns, counts, nullptr, nullptr, nullptr) ==
                  hipSuccess &&
              hipMemcpy(h.data() + 1, counts, 4 * nb, hipMemcpyDeviceToHost) == hipSuccess;
    int64_t total = 0;
    for (size_t b = 0; ok && b < nb; ++b) {
        total += h[b + 1];
        h[b + 1] = (int)total;
    }
    std::vector<int2> chunks;
    for (size_t b = 0; ok && b < nb; ++b)
        for (int q = h[b]; q < h[b + 1]; q += 256) chunks.push_back(make_int2((int)b, q));
    p->nchunks = (int64_t)chunks.size();
    ok = ok && total < INT32_MAX && hipMemcpy(p->boffs, h.data(), 4 * (nb + 1), hipMemcpyHostToDevice) == hipSuccess &&
         dalloc(&p->bchunk, sizeof(int2) * std::max<size_t>(chunks.size(), 1)) == hipSuccess &&
         (chunks.empty() ||
          hipMemcpy(p->bchunk, chunks.data(), sizeof(int2) * chunks.size(), hipMemcpyHostToDevice) == hipSuccess) &&
         dalloc(&p->bidx, 4 * (size_t)std::max<int64_t>(total, 1)) == hipSuccess &&
         hipMemset(counts, 0, 4 * nb) == hipSuccess &&
         launch_point_buckets(p->g, p->lights, p->L, p->mean, p->ns, counts, p->boffs, p->bidx, nullptr) ==
             hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
    (void)hipFree(counts);
    return ok ? DGSM_OK : DGSM_EHIP;
}

// List entries the static set (in plan order) needs per light, the maximum
// over lights; a binning on a temporary minimal workspace; synchronous.
dgsm_status count_static_entries(dgsm_plan p, int64_t& entries) {
    entries = 0;
    if (p->ns == 0) return DGSM_OK;
    const BuildLayout Lc = build_layout(p->g, p->ns, p->L, 64 * (int64_t)p->g.S);
    unsigned char* ws = nullptr;
    if (dalloc(&ws, Lc.total) != hipSuccess) return DGSM_EHIP;
    const dgsm_lights_t lt{p->lights, p->L, p->kappa, p->beta_mode};
    dgsm_status s = enqueue_bin(p->g, Lc, ws, lt, p->desc.cull_eps, set_of(p, p->mean, 0, p->ns), nullptr, true);
    std::vector<int> need(2 * (size_t)p->L, 0);
    for (int l = 0; l < p->L && s == DGSM_OK; ++l)
        if (hipMemcpy(&need[2 * l], light_ws(ws, Lc, l).need, 2 * sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
            s = DGSM_EHIP;
    if (s == DGSM_OK && hipDeviceSynchronize() != hipSuccess) s = DGSM_EHIP;
    (void)hipFree(ws);
    for (int l = 0; l < p->L; ++l) entries = need[2 * l] > entries ? need[2 * l] : entries;
    return s;
}

}  // namespace

extern "C" dgsm_status dgsm_plan_create(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc,
                                        const dgsm_gaussians_t* static_set, int64_t n_dynamic,
                                        const dgsm_plan_opts_t* opts, dgsm_plan* out) {
    if (!out || !opts) return DGSM_EINVAL;
    *out = nullptr;
    dgsm_status st = validate_desc(desc);
    if (st != DGSM_OK) return st;
    if ((st = validate_lights(lights)) != DGSM_OK) return st;
    if ((st = validate_gaussians(static_set)) != DGSM_OK) return st;
    if (n_dynamic < 0 || opts->frames < 1) return DGSM_EINVAL;
    if (opts->chains < 0 || opts->chains > kMaxChains) return DGSM_EINVAL;
    if (opts->motion != DGSM_MOTION_RIGID && opts->motion != DGSM_MOTION_FREE) return DGSM_EINVAL;
    const int groups = opts->groups > 1 ? opts->groups : 1;
    if (opts->groups < 0 || groups > 65535) return DGSM_EINVAL;
    if (groups > 1) {   // ascending offsets covering the dynamic set
        if (!opts->group_start || opts->group_start[0] != 0 || opts->group_start[groups] != n_dynamic)
            return DGSM_EINVAL;
        for (int i = 0; i < groups; ++i)
            if (opts->group_start[i + 1] < opts->group_start[i]) return DGSM_EINVAL;
    }
    const int64_t np = static_set->n + n_dynamic;
    const Geom g = make_geom(*desc);
    if (np >= INT32_MAX || (np + 64) * (int64_t)g.S >= (int64_t)INT32_MAX) return DGSM_EUNSUPPORTED;
    dgsm_plan p = new (std::nothrow) dgsm_plan_s{};
    if (!p) return DGSM_EHIP;
    p->g = g;
    p->desc = *desc;
    p->L = lights->n;
    p->kappa = lights->kappa;
    p->beta_mode = lights->beta_mode;
    p->ns = static_set->n;
    p->nd = n_dynamic;
    p->np = np;
    p->frames = opts->frames;
    p->cache = opts->static_cache != 0;
    p->autotune = opts->autotune;
    p->tile_waves = (opts->tile_waves == 2 || opts->tile_waves == 4) ? opts->tile_waves : kDefaultTileWaves;
    p->split_units = opts->split_units == 0 ? kDefaultSplitUnits : (opts->split_units < 0 ? -1 : opts->split_units);
    p->motion = opts->motion;
    p->pack = p->cache && opts->packed ? 1 : 0;
    p->static_waves = kDefaultTileWaves;
    p->static_units = kDefaultSplitUnits;
    p->groups = groups;
    const size_t elem = desc->dtype == DGSM_F16 ? 2 : 4;
    const size_t table = (size_t)p->L * g.K * plane_elems(g, true);   // plan-internal: tile-major planes
    p->lay_b = build_layout(g, p->nd, p->L);
    p->ws_b_bytes = p->cache ? p->lay_b.total : 0;
    bool ok = dalloc(&p->lights, 12 * (size_t)p->L) == hipSuccess && dalloc(&p->mean, 12 * (size_t)np) == hipSuccess &&
              dalloc(&p->scale, 12 * (size_t)np) == hipSuccess && dalloc(&p->rot, 16 * (size_t)np) == hipSuccess &&
              dalloc(&p->opacity, 4 * (size_t)np) == hipSuccess && dalloc(&p->out_index, 4 * (size_t)np) == hipSuccess &&
              // the query staging and its gather index serve the uncached frame query only
              (p->cache || (dalloc(&p->in_pos, 4 * (size_t)np) == hipSuccess &&
                            dalloc(&p->tq, 4 * (size_t)np * p->L) == hipSuccess)) &&
              dalloc(&p->atlas, table * elem) == hipSuccess &&
              (!p->cache || (dalloc(&p->tau_static, table * 4) == hipSuccess &&
                             dalloc(&p->atlas_static, table * elem) == hipSuccess &&
                             dalloc(&p->ts, 4 * (size_t)std::max<int64_t>(p->ns, 1) * p->L) == hipSuccess &&
                             dalloc(&p->ws_b, p->ws_b_bytes) == hipSuccess));
    if (ok && groups > 1) {
        ok = dalloc(&p->group, 2 * (size_t)p->nd) == hipSuccess;
        for (int i = 0; i < groups && ok; ++i) {
            const int64_t a = opts->group_start[i], b = opts->group_start[i + 1];
            if (b > a) group_index_kernel<<<(unsigned)((b - a + 255) / 256), 256>>>(p->group, a, b, i);
            ok = hipGetLastError() == hipSuccess;
        }
    }
    p->chains = p->cache ? (p->frames < kMaxChains ? p->frames : kMaxChains) : 1;
    if (p->cache && opts->chains > 0 && opts->chains < p->chains) p->chains = opts->chains;
    p->cmean[0] = p->mean;
    p->ctq[0] = p->tq;
    p->catlas[0] = p->atlas;
    p->cws[0] = p->ws_b;
    // chains beyond the first exist in cache mode only, whose query needs no staging
    for (int c = 1; c < p->chains && ok; ++c)
        ok = dalloc(&p->cmean[c], 12 * (size_t)np) == hipSuccess &&
             dalloc(&p->catlas[c], table * elem) == hipSuccess && dalloc(&p->cws[c], p->ws_b_bytes) == hipSuccess &&
             hipStreamCreateWithFlags(&p->cstream[c], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&p->ev_join[c], hipEventDisableTiming) == hipSuccess;
    ok = ok && (p->chains < 2 || hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) == hipSuccess);
    const int64_t n = p->ns;
    ok = ok && hipMemcpy(p->lights, lights->pos, 12 * (size_t)p->L, hipMemcpyDeviceToDevice) == hipSuccess;
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    if (ok && n > 0) ok = sort_static(p, *static_set) == DGSM_OK;
    if (ok && p->cache) ok = bucket_static(p) == DGSM_OK;
    // The static set never changes, so its list entries are counted once here
    // and its workspace holds exactly them (the worst case, every Gaussian in
    // every supertile list, is far larger).  Without the cache the lists hold
    // the static entries plus the dynamic set's worst case.
    if (ok) {
        int64_t entries = 0;
        ok = count_static_entries(p, entries) == DGSM_OK;
        const int64_t worst = ((p->cache ? p->ns : np) + 64) * (int64_t)g.S;
        int64_t cap = p->cache ? entries : entries + (p->nd + 64) * (int64_t)g.S;
        cap = cap < worst ? cap : worst;
        cap = cap > 64 * (int64_t)g.S ? cap : 64 * (int64_t)g.S;
        p->lay_a = build_layout(g, p->cache ? p->ns : np, p->L, cap);
        p->ws_a_bytes = p->lay_a.total;
        ok = ok && dalloc(&p->ws_a, p->ws_a_bytes) == hipSuccess;
    }
    // the atlas cones never change: computed once into each workspace
    ok = ok && enqueue_cones(g, p->lay_a, p->ws_a, nullptr) == DGSM_OK;
    for (int c = 0; c < p->chains && ok && p->cache; ++c) ok = enqueue_cones(g, p->lay_b, p->cws[c], nullptr) == DGSM_OK;
    ok = ok && hipDeviceSynchronize() == hipSuccess;
    // every chain's means start with the static set in plan order
    for (int c = 1; c < p->chains && ok && n > 0; ++c)
        ok = hipMemcpy(p->cmean[c], p->mean, 12 * (size_t)n, hipMemcpyDeviceToDevice) == hipSuccess;
    if (ok && p->nd > 0) {
        iota_kernel<<<(unsigned)((p->nd + 255) / 256), 256>>>(p->out_index, p->ns, p->np);
        ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
    if (ok && np > 0 && !p->cache) {
        invert_kernel<<<(unsigned)((np + 255) / 256), 256>>>(p->out_index, np, p->in_pos);
        ok = hipGetLastError() == hipSuccess && hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        plan_free(p);
        return DGSM_EHIP;
    }
    *out = p;
    return DGSM_OK;
}

extern "C" dgsm_status dgsm_plan_run(dgsm_plan p, const dgsm_gaussians_t* dynamic_set, const float* translations,
                                     float* T_out, int32_t use_graph, void* stream) {
    if (!p || !dynamic_set || !T_out) return DGSM_EINVAL;
    if (p->motion == DGSM_MOTION_RIGID && p->nd > 0 && !translations) return DGSM_EINVAL;
    if (dynamic_set->n != p->nd) return DGSM_EINVAL;
    dgsm_status st = validate_gaussians(dynamic_set);
    if (st != DGSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (p->autotune && !p->tuned && !tune_from_cache(p) &&
        (st = autotune(p, dynamic_set, translations, T_out, s)) != DGSM_OK)
        return st;
    if (!use_graph) return enqueue_run(p, dynamic_set, translations, T_out, s);
    if (!s) return DGSM_EINVAL;   // the legacy default stream cannot be captured
    const void* key[6] = {dynamic_set->mean, dynamic_set->scale, dynamic_set->rot, dynamic_set->opacity,
                          translations, T_out};
    bool same = p->exec != nullptr;
    for (int i = 0; i < 6 && same; ++i) same = key[i] == p->cap_key[i];
    if (!same) {
        if (p->exec) {
            // a replay of the old graph may still run on the stream
            if (hipStreamSynchronize(s) != hipSuccess) return DGSM_EHIP;
            (void)hipGraphExecDestroy(p->exec);
            p->exec = nullptr;
        }
        hipGraph_t graph;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return DGSM_EHIP;
        st = enqueue_run(p, dynamic_set, translations, T_out, s);
        const hipError_t ec = hipStreamEndCapture(s, &graph);
        if (st != DGSM_OK) return st;
        if (ec != hipSuccess) return DGSM_EHIP;
        const hipError_t ei = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            p->exec = nullptr;
            return DGSM_EHIP;
        }
        for (int i = 0; i < 6; ++i) p->cap_key[i] = key[i];
    }
    return hipGraphLaunch(p->exec, s) == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

extern "C" dgsm_status dgsm_plan_time_frame(dgsm_plan p, const dgsm_gaussians_t* dynamic_set,
                                            const float* translations, float* T_out, float ms[5], void* stream) {
    if (!p || !dynamic_set || !T_out || !ms) return DGSM_EINVAL;
    if (dynamic_set->n != p->nd) return DGSM_EINVAL;
    if (p->motion == DGSM_MOTION_RIGID && p->nd > 0 && !translations) return DGSM_EINVAL;
    dgsm_status st = validate_gaussians(dynamic_set);
    if (st != DGSM_OK) return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipEvent_t ev[5] = {};
    for (int i = 0; i < 5; ++i)
        if (hipEventCreate(&ev[i]) != hipSuccess) st = DGSM_EHIP;
    if (st == DGSM_OK && p->nd > 0 && p->motion == DGSM_MOTION_RIGID) {
        const int64_t o = p->ns;
        if (hipMemcpyAsync(p->scale + 3 * o, dynamic_set->scale, 12 * p->nd, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(p->rot + 4 * o, dynamic_set->rot, 16 * p->nd, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipMemcpyAsync(p->opacity + o, dynamic_set->opacity, 4 * p->nd, hipMemcpyDeviceToDevice, s) != hipSuccess)
            st = DGSM_EHIP;
    }
    hipEvent_t es[2] = {};
    if (st == DGSM_OK && (hipEventCreate(&es[0]) != hipSuccess || hipEventCreate(&es[1]) != hipSuccess))
        st = DGSM_EHIP;
    if (st == DGSM_OK && p->cache) st = enqueue_static(p, p->static_waves, p->static_units, s, es);
    if (st == DGSM_OK)
        st = enqueue_frame(p, 0, 0, dynamic_set, translations, T_out, p->tile_waves, p->split_units, p->pack, s, ev);
    if (st == DGSM_OK && hipEventSynchronize(ev[4]) != hipSuccess) st = DGSM_EHIP;
    for (int i = 0; i < 4 && st == DGSM_OK; ++i)
        if (hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]) != hipSuccess) st = DGSM_EHIP;
    ms[4] = 0.f;
    if (st == DGSM_OK && p->cache && hipEventElapsedTime(&ms[4], es[0], es[1]) != hipSuccess) st = DGSM_EHIP;
    for (int i = 0; i < 5; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    for (int i = 0; i < 2; ++i)
        if (es[i]) (void)hipEventDestroy(es[i]);
    return st;
}

extern "C" int32_t dgsm_plan_tile_waves(const dgsm_plan p) { return p ? p->tile_waves : 0; }

extern "C" int32_t dgsm_plan_split_units(const dgsm_plan p) { return p ? p->split_units : 0; }

extern "C" int32_t dgsm_plan_packed(const dgsm_plan p) { return p ? p->pack : 0; }

extern "C" int32_t dgsm_plan_tuned_from_cache(const dgsm_plan p) { return p && p->tuned_cached ? 1 : 0; }

extern "C" int32_t dgsm_plan_static_knobs(const dgsm_plan p, int32_t out[2]) {
    if (!p || !out) return 0;
    out[0] = p->static_waves;
    out[1] = p->static_units;
    return 1;
}

extern "C" void dgsm_autotune_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune.clear();
}

extern "C" dgsm_status dgsm_plan_destroy(dgsm_plan p) {
    if (!p) return DGSM_EINVAL;
    plan_free(p);
    return DGSM_OK;
}
