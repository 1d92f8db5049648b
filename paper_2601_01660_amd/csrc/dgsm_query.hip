// DGSM sampling on gfx950 (Sec. 3.3): trilinear lookup of the octahedral x
// radial atlas at world points, one thread per (point, light); footprint
// sampling; and, for the batched plan, points that never move indexed by the
// atlas tiles their lookups read, so that a frame looks up again only the
// points under the tiles it changed.

#include <climits>

#include "dgsm_device.hpp"
#include "dgsm_host.hpp"

namespace dgsm {

// Element offset of texel (i, j), wrapped, in a shell plane (row-major, or
// tile-major with 8x8 tiles when tiled).
__device__ inline int wrap_offset(int i, int j, int H, int W, int TW, bool tiled) {
    wrap_texel(i, j, H, W);
    return tiled ? ((i >> 3) * TW + (j >> 3)) * kWave + (i & 7) * kTile + (j & 7) : i * W + j;
}

struct QueryArgs {
    Geom g;
    const float* lights;   // [L][3]
    int L;
    const void* atlas;     // [L][K][H][W]
    const float* points;   // [P][3]
    int64_t P;
    float* T;              // [L][P]
    float lr0, kscale;     // shell coordinate: geometric (log2 r - lr0) * kscale, uniform r * kscale - 1/2
    int tiled;             // plane order of the atlas (see wrap_offset)
    const int* out_index;  // optional [P]: point p's result goes to column out_index[p]
    int point_major;       // T [P][L] instead of [L][P]
    int64_t ld;            // light-major row stride of T (0: P)
};

// Texels and weights of a trilinear lookup: the four plane offsets of the
// 2x2 texel footprint (wrapped), its first shell and the fractions.
struct Foot {
    int o[4];   // (i0, j0), (i0, j0 + 1), (i0 + 1, j0), (i0 + 1, j0 + 1)
    int k0;
    float fi, fj, fk;
};

__device__ inline Foot footprint(const QueryArgs& a, int l, float x, float y, float z) {
    const Geom& g = a.g;
    const bool tiled = a.tiled != 0;
    const Cell c = query_cell(g, a.lr0, a.kscale, a.lights + 3 * l, x, y, z);
    Foot f;
    f.o[0] = wrap_offset(c.i0, c.j0, g.H, g.W, g.TW, tiled);
    f.o[1] = wrap_offset(c.i0, c.j0 + 1, g.H, g.W, g.TW, tiled);
    f.o[2] = wrap_offset(c.i0 + 1, c.j0, g.H, g.W, g.TW, tiled);
    f.o[3] = wrap_offset(c.i0 + 1, c.j0 + 1, g.H, g.W, g.TW, tiled);
    f.k0 = c.k0;
    f.fi = c.fi; f.fj = c.fj; f.fk = c.fk;
    return f;
}

template <typename InT>
__device__ inline float interp(const QueryArgs& a, int l, const Foot& f) {
    const Geom& g = a.g;
    const size_t plane = a.tiled ? (size_t)g.ntiles * kWave : (size_t)g.H * g.W;
    const InT* s0 = reinterpret_cast<const InT*>(a.atlas) + ((size_t)l * g.K + f.k0) * plane;
    const InT* s1 = s0 + plane;
    const float fi = f.fi, fj = f.fj, fk = f.fk;
    const float a0 = (1.f - fj) * Store<InT>::get(s0 + f.o[0]) + fj * Store<InT>::get(s0 + f.o[1]);
    const float b0 = (1.f - fj) * Store<InT>::get(s0 + f.o[2]) + fj * Store<InT>::get(s0 + f.o[3]);
    const float a1 = (1.f - fj) * Store<InT>::get(s1 + f.o[0]) + fj * Store<InT>::get(s1 + f.o[1]);
    const float b1 = (1.f - fj) * Store<InT>::get(s1 + f.o[2]) + fj * Store<InT>::get(s1 + f.o[3]);
    const float t0 = (1.f - fi) * a0 + fi * b0;
    const float t1 = (1.f - fi) * a1 + fi * b1;
    return (1.f - fk) * t0 + fk * t1;
}

// Trilinear lookup of light l's atlas at world point (x, y, z).
template <typename InT>
__device__ inline float lookup(const QueryArgs& a, int l, float x, float y, float z) {
    return interp<InT>(a, l, footprint(a, l, x, y, z));
}

// One thread per (point, light): blockIdx.y is the light, so the threads of a
// wave read 64 consecutive points and write 64 consecutive T values, and each
// thread has its 8 texel gathers in flight at once.
template <typename InT>
__global__ __launch_bounds__(256) void query_kernel(QueryArgs a) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.P) return;
    const int l = blockIdx.y;
    const float T = lookup<InT>(a, l, a.points[3 * p], a.points[3 * p + 1], a.points[3 * p + 2]);
    const int64_t col = a.out_index ? (int64_t)a.out_index[p] : p;
    a.T[a.point_major ? (size_t)col * a.L + l : (size_t)l * (a.ld ? a.ld : a.P) + col] = T;
}

// ---------------------------------------------------------------------------
// Points that never move, indexed by the atlas tiles their lookups read
// (tiled atlas: a plane offset is tile * 64 + texel in the tile).  For each
// light and tile, the points whose 2x2 footprint has a texel in the tile.

// Distinct tiles of a footprint, n of them in t.
__device__ inline int foot_tiles(const Foot& f, int t[4]) {
    int n = 0;
    for (int q = 0; q < 4; ++q) {
        const int tq = f.o[q] / kWave;
        bool seen = false;
        for (int r = 0; r < n; ++r) seen |= t[r] == tq;
        if (!seen) t[n++] = tq;
    }
    return n;
}

// fill == nullptr: count the entries of each (light, tile) bucket; else write
// point indices at offs[bucket] + the bucket's cursor.
__global__ __launch_bounds__(256) void bucket_kernel(QueryArgs a, int* __restrict__ counts,
                                                     const int* __restrict__ offs, int* __restrict__ fill) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.P) return;
    const int l = blockIdx.y;
    const Foot f = footprint(a, l, a.points[3 * p], a.points[3 * p + 1], a.points[3 * p + 2]);
    int t[4];
    const int n = foot_tiles(f, t);
    for (int r = 0; r < n; ++r) {
        const size_t b = (size_t)l * a.g.ntiles + t[r];
        const int slot = atomicAdd(counts + b, 1);
        if (fill) fill[offs[b] + slot] = (int)p;
    }
}

// One workgroup per 256-point chunk of a (light, tile) bucket: if the tile's
// count in hits is nonzero, look up every point of the chunk whose lowest
// reached footprint tile is this one (each point is written once) into
// T[l][out_col[p]] (row stride ld).
template <typename InT>
__global__ __launch_bounds__(256) void patch_kernel(QueryArgs a, const unsigned char* __restrict__ hits0,
                                                    size_t hits_stride, const int* __restrict__ offs,
                                                    const int2* __restrict__ chunks, const int* __restrict__ idx,
                                                    const int* __restrict__ out_col) {
    const int2 ch = chunks[blockIdx.x];   // {bucket, first entry}
    const int l = ch.x / a.g.ntiles, tile = ch.x - l * a.g.ntiles;
    const int* hits = reinterpret_cast<const int*>(hits0 + (size_t)l * hits_stride);
    if (hits[tile] == 0) return;
    const int q = ch.y + (int)threadIdx.x;
    if (q >= offs[ch.x + 1]) return;
    const int p = idx[q];
    const Foot f = footprint(a, l, a.points[3 * p], a.points[3 * p + 1], a.points[3 * p + 2]);
    int t[4];
    const int n = foot_tiles(f, t);
    int owner = INT_MAX;
    for (int r = 0; r < n; ++r)
        if (hits[t[r]] != 0) owner = min(owner, t[r]);
    if (owner == tile) a.T[(size_t)l * a.ld + out_col[p]] = interp<InT>(a, l, f);
}

// rows of src [rows][n] into dst with row stride ld
__global__ __launch_bounds__(256) void copy_rows_kernel(const float* __restrict__ src, int64_t n, int rows,
                                                        float* __restrict__ dst, int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    for (int r = 0; r < rows; ++r) dst[(size_t)r * ld + i] = src[(size_t)r * n + i];
}

// Footprint sampling (Sec. 3.3, Ablation A): T_g = sum_i w_i T(mu_g + R_g (s_g * z_i)),
// one thread per (Gaussian, light); offsets and weights in LDS.
constexpr int kMaxFootprint = 64;

struct FootArgs {
    QueryArgs q;
    dgsm_gaussians_t gs;
    const float* z;        // [n][3]
    const float* w;        // [n]
    int n;
};

template <typename InT>
__global__ __launch_bounds__(256) void footprint_kernel(FootArgs f) {
    __shared__ float sz[kMaxFootprint][3];
    __shared__ float sw[kMaxFootprint];
    for (int i = threadIdx.x; i < f.n; i += 256) {
        sz[i][0] = f.z[3 * i];
        sz[i][1] = f.z[3 * i + 1];
        sz[i][2] = f.z[3 * i + 2];
        sw[i] = f.w[i];
    }
    __syncthreads();
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= f.gs.n) return;
    const int l = blockIdx.y;
    float qw = f.gs.rot[4 * p], qx = f.gs.rot[4 * p + 1], qy = f.gs.rot[4 * p + 2], qz = f.gs.rot[4 * p + 3];
    const float qn = rsqrtf(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn; qx *= qn; qy *= qn; qz *= qn;
    // columns of R (principal axes) scaled by the standard deviations
    const float s0 = f.gs.scale[3 * p], s1 = f.gs.scale[3 * p + 1], s2 = f.gs.scale[3 * p + 2];
    const float c0x = (1.f - 2.f * (qy * qy + qz * qz)) * s0, c0y = 2.f * (qx * qy + qw * qz) * s0,
                c0z = 2.f * (qx * qz - qw * qy) * s0;
    const float c1x = 2.f * (qx * qy - qw * qz) * s1, c1y = (1.f - 2.f * (qx * qx + qz * qz)) * s1,
                c1z = 2.f * (qy * qz + qw * qx) * s1;
    const float c2x = 2.f * (qx * qz + qw * qy) * s2, c2y = 2.f * (qy * qz - qw * qx) * s2,
                c2z = (1.f - 2.f * (qx * qx + qy * qy)) * s2;
    const float mx = f.gs.mean[3 * p], my = f.gs.mean[3 * p + 1], mz = f.gs.mean[3 * p + 2];
    float acc = 0.f;
    for (int i = 0; i < f.n; ++i) {
        const float z0 = sz[i][0], z1 = sz[i][1], z2 = sz[i][2];
        const float x = mx + c0x * z0 + c1x * z1 + c2x * z2;
        const float y = my + c0y * z0 + c1y * z1 + c2y * z2;
        const float zz = mz + c0z * z0 + c1z * z1 + c2z * z2;
        acc += sw[i] * lookup<InT>(f.q, l, x, y, zz);
    }
    f.q.T[(size_t)l * f.gs.n + p] = acc;
}

namespace {
QueryArgs query_args(const Geom& g, const float* lights, int L, const void* atlas, const float* points, int64_t P,
                     float* T, bool tiled, const int* out_index, bool point_major, int64_t ld) {
    QueryArgs a{g, lights, L, atlas, points, P, T, 0.f, 0.f, tiled ? 1 : 0, out_index, point_major ? 1 : 0, ld};
    if (g.spacing == DGSM_SHELLS_GEOMETRIC) {
        a.lr0 = log2f(g.r0);
        a.kscale = (float)(g.K - 1) / log2f(g.r1 / g.r0);
    } else {
        a.kscale = (float)g.K / g.r1;
    }
    return a;
}
}  // namespace

hipError_t launch_query(const Geom& g, const float* lights, int L, const void* atlas, const float* points,
                        int64_t P, float* T, hipStream_t st, bool tiled, const int* out_index, bool point_major,
                        int64_t ld) {
    if (P == 0) return hipSuccess;
    const QueryArgs a = query_args(g, lights, L, atlas, points, P, T, tiled, out_index, point_major, ld);
    const dim3 grid((unsigned)((P + 255) / 256), L);
    if (g.dtype == DGSM_F16)
        query_kernel<__half><<<grid, 256, 0, st>>>(a);
    else
        query_kernel<float><<<grid, 256, 0, st>>>(a);
    return hipGetLastError();
}

hipError_t launch_point_buckets(const Geom& g, const float* lights, int L, const float* points, int64_t P,
                                int* counts, const int* offs, int* idx, hipStream_t st) {
    if (P == 0) return hipSuccess;
    const QueryArgs a = query_args(g, lights, L, nullptr, points, P, nullptr, true, nullptr, false, 0);
    bucket_kernel<<<dim3((unsigned)((P + 255) / 256), L), 256, 0, st>>>(a, counts, offs, idx);
    return hipGetLastError();
}

hipError_t launch_patch(const Geom& g, const float* lights, int L, const void* atlas, const float* points,
                        const unsigned char* hits0, size_t hits_stride, const int* offs, const int2* chunks,
                        int64_t nchunks, const int* idx, const int* out_col, float* T, int64_t ld, hipStream_t st) {
    if (nchunks == 0) return hipSuccess;
    const QueryArgs a = query_args(g, lights, L, atlas, points, 0, T, true, nullptr, false, ld);
    if (g.dtype == DGSM_F16)
        patch_kernel<__half><<<(unsigned)nchunks, 256, 0, st>>>(a, hits0, hits_stride, offs, chunks, idx, out_col);
    else
        patch_kernel<float><<<(unsigned)nchunks, 256, 0, st>>>(a, hits0, hits_stride, offs, chunks, idx, out_col);
    return hipGetLastError();
}

hipError_t launch_copy_rows(const float* src, int64_t n, int rows, float* dst, int64_t ld, hipStream_t st) {
    if (n == 0) return hipSuccess;
    copy_rows_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(src, n, rows, dst, ld);
    return hipGetLastError();
}

}  // namespace dgsm

using namespace dgsm;

extern "C" dgsm_status dgsm_query(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc, const void* atlas,
                                  const float* points, int64_t P, float* T, void* stream) {
    dgsm_status st = validate_desc(desc);
    if (st != DGSM_OK) return st;
    if ((st = validate_lights(lights)) != DGSM_OK) return st;
    if (P < 0 || (P > 0 && (!atlas || !points || !T))) return DGSM_EINVAL;
    const Geom g = make_geom(*desc);
    return launch_query(g, lights->pos, lights->n, atlas, points, P, T,
                        reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

extern "C" dgsm_status dgsm_query_footprint(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc,
                                            const void* atlas, const dgsm_gaussians_t* gaussians, const float* z,
                                            const float* w, int32_t n, float* T, void* stream) {
    dgsm_status st = validate_desc(desc);
    if (st != DGSM_OK) return st;
    if ((st = validate_lights(lights)) != DGSM_OK) return st;
    if ((st = validate_gaussians(gaussians)) != DGSM_OK) return st;
    if (n < 1 || n > kMaxFootprint || !z || !w) return DGSM_EINVAL;
    if (gaussians->n > 0 && (!atlas || !T)) return DGSM_EINVAL;
    if (gaussians->n == 0) return DGSM_OK;
    const Geom g = make_geom(*desc);
    FootArgs f{};
    f.q = QueryArgs{g, lights->pos, lights->n, atlas, nullptr, gaussians->n, T, 0.f, 0.f, 0, nullptr, 0, 0};
    if (g.spacing == DGSM_SHELLS_GEOMETRIC) {
        f.q.lr0 = log2f(g.r0);
        f.q.kscale = (float)(g.K - 1) / log2f(g.r1 / g.r0);
    } else {
        f.q.kscale = (float)g.K / g.r1;
    }
    f.gs = *gaussians;
    f.z = z;
    f.w = w;
    f.n = n;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)((gaussians->n + 255) / 256), lights->n);
    if (g.dtype == DGSM_F16)
        footprint_kernel<__half><<<grid, 256, 0, s>>>(f);
    else
        footprint_kernel<float><<<grid, 256, 0, s>>>(f);
    return hipGetLastError() == hipSuccess ? DGSM_OK : DGSM_EHIP;
}

extern "C" void dgsm_footprint_stencil7(float z[21], float w[7]) {
    for (int i = 0; i < 21; ++i) z[i] = 0.f;
    const double e = exp(-0.5);
    const double norm = 1.0 + 6.0 * e;
    w[0] = (float)(1.0 / norm);
    for (int j = 0; j < 3; ++j) {
        z[3 * (1 + 2 * j) + j] = 1.f;
        z[3 * (2 + 2 * j) + j] = -1.f;
        w[1 + 2 * j] = w[2 + 2 * j] = (float)(e / norm);
    }
}

extern "C" const char* dgsm_status_string(dgsm_status s) {
    switch (s) {
        case DGSM_OK: return "ok";
        case DGSM_EINVAL: return "invalid argument";
        case DGSM_EWORKSPACE: return "workspace missing or too small";
        case DGSM_EHIP: return "HIP runtime or kernel launch error";
        case DGSM_EUNSUPPORTED: return "unsupported by this build";
    }
    return "unknown status";
}
