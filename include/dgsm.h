/*
 * dgsm.h - C ABI of the MI355X (gfx950) Deep Gaussian Shadow Map library.
 *
 * Method: "Animated 3DGS Avatars in Diverse Scenes with Consistent Lighting
 * and Shadows" (arXiv 2601.01660), Sec. 3.2 (build), Sec. 3.3 (sampling) and
 * Sec. 3.5 (SH radiance transfer).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array pointers are DEVICE pointers owned by the caller, unless the
 *    comment says "host".  Arrays are dense, C order, float32 unless stated.
 *  - The library performs no device allocation inside dgsm_build, dgsm_query,
 *    sh_transfer or dgsm_alpha_centroid; scratch memory comes from a caller
 *    workspace sized by the matching *_workspace_size function.
 *  - Every call is asynchronous and stream ordered on `stream` (a hipStream_t;
 *    NULL is the legacy default stream).  Outputs are valid once the stream
 *    reaches the call.
 *  - Arguments are validated on the host before anything is enqueued.  A
 *    non-zero dgsm_status means nothing was enqueued (DGSM_EHIP: a HIP launch
 *    failed; earlier kernels of the same call may have run).
 *  - Calls on distinct output and workspace buffers may run concurrently on
 *    different streams.  The library holds no global mutable state except the
 *    per-GPU scratch array of dgsm_build_noalloc.
 *
 * Gaussian records (Sec. 3.2, first paragraph): mean mu, covariance
 * Sigma = R diag(s^2) R^T with R from a quaternion (w, x, y, z) that the
 * library normalises, precision A = Sigma^-1, opacity alpha in [0, 1).
 *
 * Atlas layout (Sec. 3.2 "Directional parameterization ... and storage"):
 * T[l][k][i][j], shell-major, light l, shell k, texel row i, column j.  Texel
 * (i, j) stores T at direction psi^-1(u, v) with u = -1 + (2j+1)/W and
 * v = -1 + (2i+1)/H (texel centres; sgn(0) = +1 in the octahedral fold) and at
 * radius t_k:
 *    uniform   t_k = (k + 1/2) * r1 / K                  (r0 unused)
 *    geometric t_k = r0 * (r1/r0)^(k/(K-1))
 */
#ifndef DGSM_H
#define DGSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DGSM_OK = 0,
    DGSM_EINVAL = 1,       /* invalid argument (null pointer, bad size, bad enum) */
    DGSM_EWORKSPACE = 2,   /* workspace pointer null or smaller than required */
    DGSM_EHIP = 3,         /* a HIP runtime call or kernel launch failed */
    DGSM_EUNSUPPORTED = 4  /* valid request this build does not implement */
} dgsm_status;

typedef enum { DGSM_SHELLS_UNIFORM = 0, DGSM_SHELLS_GEOMETRIC = 1 } dgsm_spacing;
typedef enum { DGSM_F32 = 0, DGSM_F16 = 1 } dgsm_dtype;

/* Gaussian set, structure of arrays, device memory.  n may be 0. */
typedef struct {
    const float* mean;     /* [n][3] metres */
    const float* scale;    /* [n][3] standard deviations s > 0 in metres */
    const float* rot;      /* [n][4] quaternion (w, x, y, z), any non-zero norm */
    const float* opacity;  /* [n]    alpha in [0, 1) */
    int64_t n;
} dgsm_gaussians_t;

/* Opacity-to-absorption mapping (Sec. 3.2 Eq. 5 and the alpha -> beta
 * ablation), with tau* = -ln(1 - alpha) and kappa the strength knob:
 *   DGSM_BETA_TRACE    beta = kappa tau* sqrt(tr(A)/3) / sqrt(2 pi)   (Eq. 5, default)
 *   DGSM_BETA_CONSTANT beta = kappa tau*
 *   DGSM_BETA_DENSITY  beta = kappa tau* / ((2 pi)^(3/2) s_x s_y s_z)
 *                      (the ablation's det-of-covariance and diagonal-scale
 *                      forms coincide: det of the covariance = (s_x s_y s_z)^2) */
typedef enum { DGSM_BETA_TRACE = 0, DGSM_BETA_CONSTANT = 1, DGSM_BETA_DENSITY = 2 } dgsm_beta_mode;

/* Point lights.  pos is a DEVICE pointer [n][3].  kappa is the global
 * strength knob of Eq. 5 (1 reproduces the 3DGS opacity in the far field);
 * beta_mode a dgsm_beta_mode (0 = Eq. 5). */
typedef struct {
    const float* pos;
    int32_t n;
    float kappa;
    int32_t beta_mode;
} dgsm_lights_t;

/* Direction parameterisation of the atlas.
 *   DGSM_PARAM_OCTAHEDRAL  the octahedral map of Sec. 3.2 (default): texel
 *       (i, j) has u = -1 + (2j+1)/W, v = -1 + (2i+1)/H; lookups wrap across
 *       the outer edges through the octahedral mirror (see dgsm_query).
 *   DGSM_PARAM_CUBEMAP  the six-face cube map the octahedral atlas is compared
 *       with (Ablation C).  Faces of F x F texels, H = 2F, W = 3F; face
 *       f = 2m + (0 for the + side, 1 for the - side) of major axis m in
 *       (x, y, z) sits at block row f / 3, block column f % 3.  Texel (b, a)
 *       inside face (m, sign) has face coordinates s = -1 + (2a+1)/F,
 *       t = -1 + (2b+1)/F and direction along d[m] = sign, d[(m+1) % 3] = s,
 *       d[(m+2) % 3] = t.  A lookup takes the face of the largest |component|
 *       of the FP32 offset (the first axis on ties) and interpolates
 *       bilinearly inside that face, clamped to its edge texels (no filtering
 *       across faces).  The learned field (dgsm_mlp_*) accepts only the
 *       octahedral atlas. */
typedef enum { DGSM_PARAM_OCTAHEDRAL = 0, DGSM_PARAM_CUBEMAP = 1 } dgsm_param;

/* Atlas description.  Octahedral: H and W even, >= 2.  Cube map: H = 2F,
 * W = 3F, F >= 2.  H, W <= 1024; K >= 2; r1 > 0, and 0 < r0 < r1
 * for geometric spacing.  cull_eps is the per-Gaussian contribution bound of
 * the light-space culling (Sec. 3.2 "Occluder culling"): a Gaussian is left
 * out of a tile only where its optical depth along every texel ray of the
 * tile is provably below cull_eps.  cull_eps = 0 disables culling (every
 * Gaussian is evaluated for every texel; the result then equals the plain
 * definition up to FP32 rounding).  Typical value 1e-8. */
typedef struct {
    int32_t H, W, K;
    int32_t spacing;       /* dgsm_spacing */
    float r0, r1;
    int32_t dtype;         /* dgsm_dtype of the stored T: FP32, or FP16 (RNE of the FP32 value) */
    float cull_eps;
    int32_t param;         /* dgsm_param */
} dgsm_atlas_desc_t;

/* Human-readable text for a status code (static storage). */
const char* dgsm_status_string(dgsm_status s);

/* Bytes of workspace dgsm_build needs for this atlas, n_gauss Gaussians and
 * n_lights lights.  Returns 0 if desc is invalid. */
size_t dgsm_build_workspace_size(const dgsm_atlas_desc_t* desc, int64_t n_gauss, int32_t n_lights);

/*
 * dgsm_build - tabulate T(d, t) = exp(-tau(d, t)) for every light (Sec. 3.2).
 *   tau(d, t) = sum_i beta_i int_0^t exp(-1/2 (x(s)-mu_i)^T A_i (x(s)-mu_i)) ds,
 *   x(s) = o_L + s d (Eqs. 1-2), each term in the erf closed form of Eq. 3,
 *   T by Eq. 4, beta_i = kappa (-ln(1-alpha_i)) sqrt(tr(A_i)/3) / sqrt(2 pi) (Eq. 5).
 * Every Gaussian passed is an occluder.  Computed in FP32 with the
 * cancellation-prone geometry (light-to-mean offsets, ray cross products and
 * the distance along the ray) in FP64.
 *   lights   : n >= 1 lights
 *   gaussians: any n >= 0 (n = 0 gives T = 1 everywhere)
 *   atlas    : device output [lights.n][K][H][W] of desc->dtype
 *   ws       : device workspace of >= dgsm_build_workspace_size(...) bytes; its
 *              contents on entry are ignored and on exit undefined
 * T is non-increasing in k at every texel and lies in [0, 1].
 */
dgsm_status dgsm_build(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                       const dgsm_atlas_desc_t* desc, void* atlas, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * Workspaces sized for a particular Gaussian set.  dgsm_build_workspace_size
 * covers the worst case, in which every Gaussian reaches every supertile of
 * the atlas (n S list entries per light, S = number of 64 x 64-texel
 * supertiles, up to 256): about 12 n S bytes per light, 98 GB for 4 M
 * Gaussians and 8 lights at 1024 x 1024.  Real sets need far fewer entries
 * (each Gaussian's light-space footprint covers a few supertiles), so every
 * call that takes a build workspace (dgsm_build, dgsm_bin, dgsm_accumulate,
 * dgsm_build_roi, dgsm_work_units, dgsm_list_entries) derives the list
 * capacity from ws_bytes: the worst case if ws_bytes holds it, otherwise the
 * largest capacity that fits (DGSM_EWORKSPACE if not even 64 S entries do).
 *
 * dgsm_build_workspace_size_entries - bytes of a workspace whose lists hold
 *   `entries` entries per light (rounded up to a multiple of 64, at least 64 S,
 *   at most the worst case); 0 if the arguments are invalid.
 * dgsm_count_entries - bins `gaussians` (Sec. 3.2 "Occluder culling") on ws
 *   and returns in *entries (host) the list entries the set needs, the maximum
 *   over lights: a workspace of dgsm_build_workspace_size_entries(desc, n, L,
 *   *entries) bytes then holds this set.  Any workspace of at least
 *   dgsm_build_workspace_size_entries(desc, n, L, 0) bytes will do.
 *   Synchronises `stream`.
 * dgsm_list_entries - out[0] = entries the last binning on ws needed for light
 *   `light`, out[1] = the capacity of ws.  When out[0] > out[1] that binning
 *   did not fit: the library then empties every list of the light (nothing is
 *   written past the workspace) and the atlas it builds is wrong.  Copies from
 *   the device and synchronises `stream`.
 */
size_t dgsm_build_workspace_size_entries(const dgsm_atlas_desc_t* desc, int64_t n_gauss, int32_t n_lights,
                                         int64_t entries);
dgsm_status dgsm_count_entries(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                               const dgsm_atlas_desc_t* desc, void* ws, size_t ws_bytes, int64_t* entries,
                               void* stream);
dgsm_status dgsm_list_entries(const dgsm_atlas_desc_t* desc, int64_t n_gauss, int32_t n_lights, const void* ws,
                              size_t ws_bytes, int32_t light, int64_t out[2], void* stream);

/*
 * dgsm_build_noalloc - dgsm_build for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, kernels and result as dgsm_build, but the
 * workspace is a fixed array inside the library instead of a caller buffer:
 * the call performs no hipMalloc, hipFree or other allocation.
 *   - Limit: the request must fit DGSM_BUILD_SCRATCH_BYTES (64 MiB), i.e.
 *     dgsm_build_workspace_size(desc, gaussians->n, lights->n) <= that
 *     (for example 50k Gaussians at 128 x 128 x 32, 20k at 256 x 256 x 64, one
 *     light); larger requests return DGSM_EWORKSPACE and enqueue nothing.
 *   - Each GPU holds its own copy of the array from the first call on it until
 *     the process ends; its address is looked up once per device, with that
 *     device current, on the first call there (DGSM_EHIP if the lookup fails).
 *   - Every call on one GPU shares that GPU's array.  Calls that overlap on one
 *     GPU (concurrent streams, or host threads enqueuing at once with no
 *     ordering between their streams) race on it and give undefined results;
 *     stream-ordered calls are safe.  Nothing the previous call left in the
 *     array is read.
 * dgsm_build_noalloc_max_bytes returns DGSM_BUILD_SCRATCH_BYTES.
 */
#define DGSM_BUILD_SCRATCH_BYTES (64u * 1024u * 1024u)
dgsm_status dgsm_build_noalloc(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                               const dgsm_atlas_desc_t* desc, void* atlas, void* stream);
size_t dgsm_build_noalloc_max_bytes(void);

/*
 * dgsm_build in two phases, for callers that schedule or time them apart.
 * dgsm_build(...) is exactly dgsm_bin(...) followed by dgsm_accumulate(...) on
 * the same workspace.
 *
 * dgsm_bin - light-space culling and bucketing of the occluders (Sec. 3.2
 * "Occluder culling via light-space footprints"): per light and Gaussian a
 * record of the Eq. 2-3 quantities and a conservative cone of directions
 * outside which its optical depth stays below desc->cull_eps; Gaussian ids are
 * bucketed, in ascending order, into lists of atlas supertiles (groups of 8x8
 * texel tiles) whose texel-centre directions the cone can reach.
 *
 * dgsm_accumulate - per 8x8 atlas tile, the Gaussians of its supertile list
 * whose cone reaches the tile are evaluated at every texel (Eq. 3), summed
 * over Gaussians in list order (Eq. 2; bitwise reproducible) and stored as T
 * (Eq. 4) in atlas.  n_gauss must equal the count passed to dgsm_bin.
 *   stats: optional device array [8] of counters the call ADDS to (zero it
 *   first): [0] texel-Gaussian pairs evaluated at tile granularity, [1] pairs
 *   whose prefactor exceeded cull_eps, [2] erf-ramp evaluations of those,
 *   [3] supertile list entries scanned, [4] (tile, Gaussian) pairs with no
 *   texel above cull_eps, [5] shell iterations of the ramp loops (one per
 *   wave and shell), [6] (tile, Gaussian) pairs, [7] idle pairs rejected by
 *   the distance pre-test (a subset of [4]).  NULL
 *   disables counting (the timed configuration).
 * A tile with far more Gaussian hits than the launch's mean is cut into
 * slices evaluated by separate workgroups whose fixed-point sums are added
 * afterwards; integer sums make the atlas bitwise the same as unsplit.
 *
 * dgsm_work_units - how the last dgsm_accumulate on this workspace cut its
 * tiles, for light `light`: out[0] extra slices, out[1] split tiles, out[2]
 * hits per slice (0: no splitting), out[3] total (tile, Gaussian) hits.
 * Copies from the device and synchronises `stream`.
 */
dgsm_status dgsm_bin(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                     const dgsm_atlas_desc_t* desc, void* ws, size_t ws_bytes, void* stream);
dgsm_status dgsm_accumulate(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc, int64_t n_gauss,
                            void* atlas, void* ws, size_t ws_bytes, unsigned long long* stats, void* stream);
/*
 * dgsm_accumulate_ex - dgsm_accumulate with the knobs of the tile accumulation
 * (the batched plan's autotuner chooses among them; the result is bitwise the
 * same for every choice):
 *   tile_waves   waves sharing one 8 x 8 tile's accumulators: 2, 4 or 8
 *   split_units  target work units per launch (0: default 32768; < 0: never
 *                cut a tile into slices)
 *   packed       0: every binned (tile, Gaussian) pair is evaluated at all 64
 *                texels of the tile at once; 1: packed walk -- each pair only
 *                runs the distance pre-test over the tile's texels, and the
 *                (texel, Gaussian) pairs that pass are evaluated 64 at a time,
 *                one per lane (faster for sets whose Gaussians cover few texels
 *                of a tile, such as an avatar seen from a light).  stats must be
 *                NULL with packed = 1.
 * dgsm_accumulate(...) equals dgsm_accumulate_ex with {8, 0, 0}.
 */
typedef struct {
    int32_t tile_waves;
    int32_t split_units;
    int32_t packed;
} dgsm_accum_opts_t;
dgsm_status dgsm_accumulate_ex(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc, int64_t n_gauss,
                               void* atlas, void* ws, size_t ws_bytes, const dgsm_accum_opts_t* opts,
                               unsigned long long* stats, void* stream);
dgsm_status dgsm_work_units(const dgsm_atlas_desc_t* desc, int64_t n_gauss, int32_t n_lights, const void* ws,
                            size_t ws_bytes, int32_t light, int32_t out[4], void* stream);

/*
 * dgsm_build_roi - dgsm_build restricted to a receiver-driven region of
 * interest (Sec. 3.2 "Receiver-driven region of interest"): receivers are the
 * points of `receivers` inside the box
 *   |x - cx| <= half, |y - cy| <= half, zmin <= z <= zmax
 * (half <= 0: every point is a receiver; cx, cy typically the alpha-weighted
 * avatar centroid from dgsm_alpha_centroid, half the radius R of the paper,
 * zmin / zmax robust height bounds).  Per light, the region is the set of
 * texels each receiver's trilinear lookup reads (its cell of dgsm_query, four
 * texels with the octahedral wrap) times the shell range [k_min, k_max] of
 * all receivers (each lookup reads shells k0 and k0 + 1).  T equals the full
 * build inside the region and is 1 outside it, by construction; queries at
 * receivers therefore equal queries of the full atlas (up to FP32 rounding of
 * the per-shell sums).  Tiles without receiver texels do no accumulation.
 *   receivers: device [n_receivers][3] (n_receivers = 0: T = 1 everywhere)
 *   box      : host
 *   atlas, ws: as dgsm_build (the same workspace size)
 */
typedef struct {
    float cx, cy, half, zmin, zmax;
} dgsm_roi_box_t;

dgsm_status dgsm_build_roi(const dgsm_lights_t* lights, const dgsm_gaussians_t* gaussians,
                           const dgsm_atlas_desc_t* desc, const float* receivers, int64_t n_receivers,
                           const dgsm_roi_box_t* box, void* atlas, void* ws, size_t ws_bytes, void* stream);

/*
 * dgsm_query - sample the atlas at world points (Sec. 3.3): for each light l
 * and point x, r = |x - o_L|, d = (x - o_L)/r (d = +z when r = 0), continuous
 * texel coordinates j_f = (u+1) W/2 - 1/2, i_f = (v+1) H/2 - 1/2 of (u, v) =
 * psi(d), fractional shell k_f = (K-1) ln(r/r0)/ln(r1/r0) (geometric) or
 * r K / r1 - 1/2 (uniform) clamped to [0, K-1]; trilinear interpolation of T.
 * Texel neighbours outside the grid follow the octahedral mirror wrap: a
 * column beyond the left/right edge maps to column 0 / W-1 at row H-1-i, then
 * a row beyond the top/bottom edge maps to row 0 / H-1 at column W-1-j.
 * A cube-map atlas (desc->param) takes the in-face coordinates instead:
 * a_f = (s+1) F/2 - 1/2 and b_f = (t+1) F/2 - 1/2 clamped to [0, F-1], with
 * both neighbours inside the face.
 *   atlas : device [lights.n][K][H][W] of desc->dtype (as written by dgsm_build)
 *   points: device [P][3];  T: device output [lights.n][P] float32.  P may be 0.
 */
dgsm_status dgsm_query(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc, const void* atlas,
                       const float* points, int64_t P, float* T, void* stream);

/*
 * dgsm_query_footprint - per-receiver transmittance averaged over a footprint
 * around each Gaussian (Sec. 3.3 sampling; Ablation A "footprint sampling"):
 *   T_g = sum_i w[i] T(mu_g + R_g (s_g * z[i])),
 * R_g the rotation of the unit quaternion, s_g the standard deviations, z[i]
 * offsets in the principal-axes frame, T the trilinear lookup of dgsm_query.
 * Monte Carlo sampling passes standard-normal draws z and w = 1/n; the
 * deterministic stencil is dgsm_footprint_stencil7.
 *   z: device [n][3], w: device [n] (sum 1 expected, not checked), 1 <= n <= 64
 *   T: device output [lights.n][gaussians.n] float32
 */
dgsm_status dgsm_query_footprint(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc, const void* atlas,
                                 const dgsm_gaussians_t* gaussians, const float* z, const float* w, int32_t n,
                                 float* T, void* stream);

/* The 7-point footprint stencil (host arrays): z = 0 and +-e_j (one standard
 * deviation along each principal axis), weights proportional to the Gaussian
 * kernel exp(-|z|^2 / 2) at the offsets, normalised to sum 1.  The paper
 * names the stencil without its offsets or weights; this is the reading used. */
void dgsm_footprint_stencil7(float z[21], float w[7]);

/* Parameters of the SH radiance transfer (Sec. 3.5).  The lat-long grid has
 * cell centres theta_a = (a + 1/2) pi / n_theta, phi_b = (b + 1/2) 2 pi / n_phi,
 * direction (sin th cos ph, sin th sin ph, cos th) and weight sin(theta).
 * Defaults used by the workloads: 32 x 64, q = 1, clip_max = 4, eps = 1e-6,
 * gamma = 1. */
typedef struct {
    int32_t n_theta, n_phi;   /* >= 1 each */
    float q;                  /* lobe exponent, > 0 (1 = Lambertian) */
    float clip_max;           /* t_max of the clip, > 0 */
    float eps;                /* denominator epsilon, >= 0 */
    float gamma;              /* global intensity */
    const float* centroid;    /* device [3]: point the normals face away from */
} dgsm_sh_params_t;

/*
 * sh_transfer - per-Gaussian radiance transfer (Sec. 3.4 evaluation and 3.5).
 *   L(w) = B(w) A with the probe A = probe_sh [Kp][3] (Kp in {1, 4, 9, 16});
 *   B is the real orthonormal SH basis, index k = l^2 + l + m, WITHOUT the
 *   Condon-Shortley phase (Y_1,-1 ~ +y, Y_1,0 ~ +z, Y_1,1 ~ +x).
 *   n = column of R for the smallest scale (ties: lowest axis), negated when
 *   n . (mu - centroid) < 0.  S_j = max(0, <w_j, n>)^q.
 *   s_c = clip_[0, clip_max]( sum_j w_j L_c(w_j) S_j / (sum_j w_j S_j + eps) ).
 *   scale_out     : device [n][3] = s
 *   colour_sh     : device [n][16][3] SH colour coefficients, or NULL
 *   colour_sh_out : device [n][16][3] = gamma s_c f (no clamp), or NULL
 *   rgb_out       : device [n][3] = max(0, gamma (0.5 + C0 f_0) s) with
 *                   C0 = 1/(2 sqrt(pi)) (the DC colour), or NULL
 *   colour_sh_out and rgb_out require colour_sh.
 *   ws            : device workspace of >= sh_transfer_workspace_size(n_theta,
 *                   n_phi) bytes, 16-byte aligned (16 bytes per grid
 *                   direction with the columns padded to a multiple of 16,
 *                   plus the row and column sines and cosines): the probe's
 *                   weighted radiance and weight on the grid, evaluated once
 *                   per call and then read by every Gaussian's sum.
 *                   DGSM_EINVAL if ws is not 16-byte aligned.
 * The sums run in FP32 in a fixed order, bitwise reproducible: the grid is
 * cut into eight parts; within a part, of every 16 directions 12 go to two
 * matrix-core partial sums (alternating) and 4 to a vector partial sum, each
 * in direction order; the three are added, then the parts in order.
 */
size_t sh_transfer_workspace_size(int32_t n_theta, int32_t n_phi);
dgsm_status sh_transfer(const float* probe_sh, int32_t Kp, const dgsm_gaussians_t* gaussians,
                        const float* colour_sh, const dgsm_sh_params_t* params, float* scale_out,
                        float* colour_sh_out, float* rgb_out, void* ws, size_t ws_bytes, void* stream);

/*
 * Batched build + query over animation frames (a plan).
 *
 * A plan serves a scene made of a STATIC Gaussian set (copied into the plan at
 * creation; the caller's arrays may be freed afterwards) and a DYNAMIC set of
 * n_dynamic Gaussians (avatars, re-posed every frame) that moves in one of two
 * ways (opts->motion):
 *   DGSM_MOTION_RIGID  the dynamic set is cut into opts->groups consecutive
 *       groups (one per avatar; group g holds Gaussians [group_start[g],
 *       group_start[g+1])), each translated rigidly: in frame f the means of
 *       group g are base_mean + translations[f][g] (one FP32 addition per
 *       coordinate), scales, rotations and opacities fixed;
 *   DGSM_MOTION_FREE   every frame brings its own dynamic Gaussians: the
 *       dynamic_set arrays of dgsm_plan_run hold F frames (mean [F][n][3],
 *       scale [F][n][3], rot [F][n][4], opacity [F][n], n = n_dynamic) and
 *       translations is ignored (a skinned avatar).
 * One dgsm_plan_run evaluates every frame:
 * the atlas of every light from all static + dynamic Gaussians (exactly what
 * dgsm_build computes on the union) and a dgsm_query of every light at all
 * Gaussian centres (static first, then dynamic) into T_out[f][light][point].
 *
 * dgsm_plan_opts_t:
 *   frames        F >= 1 frames per run
 *   static_cache  1: the static optical depth is built once per run and each
 *                 frame adds only the dynamic Gaussians to it (tau is a sum over
 *                 Gaussians, Eq. 2); 0: every frame rebuilds from all Gaussians
 *   autotune      1: the first run (unless the tuning cache below holds this
 *                 workload) times the knobs of the tile accumulation on the
 *                 real workload -- in cache mode a window of frames dealt to
 *                 the chains as a run deals them, else frame 0 -- and keeps
 *                 the fastest combination: waves per tile (4, 8), work units
 *                 per launch (8192, 32768, 131072) and, in cache mode, the
 *                 packed walk (see dgsm_accumulate_ex) on or off; in cache mode they
 *                 apply to the per-frame dynamic accumulation, and the
 *                 once-per-run static build gets its own waves per tile and
 *                 work units, timed on the static set (tile walk); without
 *                 autotuning the static build takes the defaults (8, 32768)
 *   tile_waves    waves sharing one 8x8 tile when autotune = 0 (2, 4 or 8; else 8)
 *   split_units   target number of work units per accumulation when
 *                 autotune = 0: a tile with more hits than (total hits /
 *                 split_units) is cut into slices run by separate blocks
 *                 (results are bitwise the same); 0 = default (32768),
 *                 negative = never split
 *   packed        packed walk for the dynamic accumulation when autotune = 0
 *                 (cache mode only)
 *   chains        frame chains in cache mode (see below): 0 = min(F, 3),
 *                 else 1..3 (fewer chains, less memory)
 *   motion        dgsm_motion (DGSM_MOTION_RIGID = 0, DGSM_MOTION_FREE = 1)
 *   groups        rigid groups (0 or 1: the whole dynamic set is one group)
 *   group_start   host [groups + 1], ascending from 0 to n_dynamic (read at
 *                 creation only); NULL when groups <= 1
 *
 * Memory: the static set's supertile lists are counted once at creation (a
 * binning of the static set, synchronous) and its workspace holds exactly
 * those entries; the dynamic set's workspaces hold its worst case (n_dynamic
 * times the supertile count per light), since it moves.  In cache mode the
 * static points are also indexed at creation by the atlas tiles their
 * lookups read (per light and tile; about 1.3 four-byte entries per point
 * and light), and each run queries them once in the static-only atlas: a
 * frame then looks up again only the static points under tiles the dynamic
 * set reaches and copies the others' run-wide values (the tiles it does not
 * reach hold the static-only atlas, so those values are the lookups' own).
 *
 * dgsm_plan_create allocates all device memory the plan needs (the only
 * allocating entry points are create and destroy) and synchronises the device;
 * dgsm_plan_destroy synchronises the device (a run may still be in flight)
 * before it frees the plan's buffers, streams and events.
 * dgsm_plan_run enqueues on `stream`; with use_graph = 1 the whole run (static
 * build + all frames) is captured once into a hipGraph and replayed (stream
 * must then be a created stream, not NULL; a run with different dynamic or
 * output pointers recaptures).  Runs of one plan must not overlap.  In cache
 * mode with F >= 2 the frames are dealt round-robin to min(F, 3) chains of
 * buffers; frame f runs on chain f mod chains, chain 0 on `stream` and the
 * others on streams the plan owns, forked from `stream` after the static
 * build and joined back into it before the run ends, so work enqueued on
 * `stream` afterwards sees every frame.
 *   dynamic_set : rigid: device arrays of the dynamic set at its base pose
 *                 (n = n_dynamic); free: device arrays of all F frames (above)
 *   translations: rigid: device [F][groups][3]; free: ignored (may be NULL)
 *   T_out       : device [F][lights.n][n_static + n_dynamic] float32
 */
typedef struct dgsm_plan_s* dgsm_plan;
typedef enum { DGSM_MOTION_RIGID = 0, DGSM_MOTION_FREE = 1 } dgsm_motion;
typedef struct {
    int32_t frames;
    int32_t static_cache;
    int32_t autotune;
    int32_t tile_waves;
    int32_t split_units;
    int32_t chains;
    int32_t motion;
    int32_t groups;
    const int64_t* group_start;
    int32_t packed;
} dgsm_plan_opts_t;

dgsm_status dgsm_plan_create(const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc,
                             const dgsm_gaussians_t* static_set, int64_t n_dynamic,
                             const dgsm_plan_opts_t* opts, dgsm_plan* out);
dgsm_status dgsm_plan_run(dgsm_plan plan, const dgsm_gaussians_t* dynamic_set, const float* translations,
                          float* T_out, int32_t use_graph, void* stream);
/* dgsm_plan_time_frame - one frame of the plan (frame 0, on the caller's
 * stream, eagerly, after the static build in cache mode) with HIP events
 * between its phases: ms[0] dynamic binning (the whole set without the cache),
 * ms[1] tile accumulation (work-unit planning, tile build, finish of split
 * tiles), ms[2] query and reordering into T_out, ms[3] restore of the reached
 * tiles (cache mode), ms[4] the static set's accumulation into its cached
 * optical depth (cache mode; 0 otherwise).  Writes T_out[0]; synchronises
 * `stream`.  For measuring the launches; results as dgsm_plan_run. */
dgsm_status dgsm_plan_time_frame(dgsm_plan plan, const dgsm_gaussians_t* dynamic_set, const float* translations,
                                 float* T_out, float ms[5], void* stream);

/* The knobs in use (after autotuning, if enabled): waves per tile, work
 * units per accumulation (-1: never split), packed walk (1) or not (0). */
int32_t dgsm_plan_tile_waves(const dgsm_plan plan);
int32_t dgsm_plan_split_units(const dgsm_plan plan);
int32_t dgsm_plan_packed(const dgsm_plan plan);
/* Tuning cache: the autotuner's choice is kept for the process, keyed by the
 * workload (atlas H, W, K, spacing, storage type and parameterisation, light
 * count, cache mode, motion, and the static and dynamic Gaussian counts to the
 * nearest power of two); a later plan with the same key takes it without
 * timing.  The cache is guarded by a mutex (plans may be created and run from
 * several host threads).  dgsm_plan_tuned_from_cache: 1 if this plan's knobs
 * came from the cache; dgsm_autotune_cache_clear empties it. */
int32_t dgsm_plan_tuned_from_cache(const dgsm_plan plan);
/* out = {waves per tile, work units} of the static build; returns 1 (0 if plan or out is NULL). */
int32_t dgsm_plan_static_knobs(const dgsm_plan plan, int32_t out[2]);
void dgsm_autotune_cache_clear(void);
dgsm_status dgsm_plan_destroy(dgsm_plan plan);

/*
 * Learned per-light transmittance field (a surrogate of one light's atlas).
 *
 * Network: features phi(u, v, rho) -> 4 hidden layers of 128 ReLU units ->
 * z -> T = sigmoid(-z) (log T = -softplus(z)).  (u, v) is the octahedral code
 * of the direction from the light, rho in [-1, 1] the atlas radius coordinate
 * (geometric: 2 ln(r/r0)/ln(r1/r0) - 1; uniform: 2 r/r1 - 1; clamped).
 * phi[128] = u, v, rho, then for i = 0..15 and f_i = pi (W/4)^(i/15) (W the
 * atlas width): sin(f_i u), cos(f_i u), sin(f_i v), cos(f_i v), sin(f_i rho),
 * cos(f_i rho); zeros from index 99.  The sines take the phase f_i x / (2 pi)
 * formed in FP64 and reduced to [-1/2, 1/2] turns; training, gradients and checks
 * evaluate them in FP64, inference in FP32.  Matrix products run on BF16 MFMA with
 * FP32 accumulation: weights, features, hidden activations and back-propagated
 * pre-activation gradients are rounded to BF16 (nearest even) where they enter
 * the matrix units; biases, the output layer and all accumulations are FP32.
 *
 * Parameters: FP32 device array of DGSM_MLP_PARAMS values, per layer l = 0..3
 * W_l [128 out][128 in] row-major then b_l [128], then w4 [128], then b4.
 * Adam state: FP32 [2][DGSM_MLP_PARAMS] (first then second moments), zero it
 * before the first step.  Loss: mean over the batch of (T - T_target)^2.
 */
#define DGSM_MLP_PARAMS 66177

typedef struct {
    int64_t batch;       /* samples per step, multiple of 32 */
    int32_t steps;       /* steps in this call */
    int32_t step0;       /* Adam steps already taken (bias correction continues) */
    float lr0, lr1;      /* learning rate, cosine decay from lr0 to lr1 over the call */
    uint32_t seed;       /* sample stream */
    float beta1, beta2, eps;
} dgsm_mlp_train_t;

/* Workspace for dgsm_mlp_grad / dgsm_mlp_train at this batch (0 if invalid). */
size_t dgsm_mlp_workspace_size(int64_t batch);
/* Workspace for dgsm_mlp_infer with n_lights parameter sets; dgsm_mlp_check
 * needs dgsm_mlp_infer_workspace_size(1) plus 16 bytes per check sample
 * (rounded up to 256). */
size_t dgsm_mlp_infer_workspace_size(int32_t n_lights);

/* Gradient of the loss at params on B given samples uvrt [B][4] = (u, v, rho,
 * T_target), without an update.  grad: device [DGSM_MLP_PARAMS]; loss: device
 * [1] or NULL.  B multiple of 32.  desc supplies W (frequencies). */
dgsm_status dgsm_mlp_grad(const float* params, const float* uvrt, int64_t B, const dgsm_atlas_desc_t* desc,
                          float* grad, float* loss, void* ws, size_t ws_bytes, void* stream);

/* opt->steps Adam steps on batches sampled from one light's atlas atlas_l
 * [K][H][W] (desc->dtype): half of each batch at texel centres and shell radii
 * (exact table values), half uniform in (u, v, rho) with trilinear targets.
 * loss_out: device [steps] or NULL. */
dgsm_status dgsm_mlp_train(float* params, float* adam_mv, const dgsm_atlas_desc_t* desc, const void* atlas_l,
                           const dgsm_mlp_train_t* opt, float* loss_out, void* ws, size_t ws_bytes, void* stream);

/* Held-out check: n_check samples drawn like the training samples from the
 * stream `seed`; sets mask[region] = 1 for every sample with |T - T_atlas| >
 * thresh, region = (k0/8, i0/8, j0/8) of its floor texel, mask laid out
 * [ceil(K/8)][H/8 tiles][W/8 tiles] (zero it first).  stats: device uint [2]
 * (zero it first): flagged samples, max |T - T_atlas| as float bits. */
dgsm_status dgsm_mlp_check(const float* params, const dgsm_atlas_desc_t* desc, const void* atlas_l,
                           int64_t n_check, uint32_t seed, float thresh, unsigned char* mask, unsigned int* stats,
                           void* ws, size_t ws_bytes, void* stream);

/* Exhaustive check of one light's network over its atlas, for a fallback mask
 * that does not depend on a random held-out draw: the network is compared with
 * the table at every texel centre and shell radius (H W K samples, exact table
 * values) and at n_per_region points drawn uniformly (stream `seed`) inside
 * each fallback region's domain -- the continuous texel and shell coordinates
 * whose trilinear cell lies in the region -- against the trilinear atlas value.
 * A node that misses by more than thresh flags the regions of all (up to 8)
 * cells it is a corner of; a random point flags the region of its own cell.
 * mask and stats as dgsm_mlp_check (zero them first).  The samples are staged
 * in passes of at most 4M rows; ws >= dgsm_mlp_check_grid_workspace_size(desc,
 * n_per_region) bytes (0 if desc is invalid or n_per_region < 0). */
size_t dgsm_mlp_check_grid_workspace_size(const dgsm_atlas_desc_t* desc, int32_t n_per_region);
dgsm_status dgsm_mlp_check_grid(const float* params, const dgsm_atlas_desc_t* desc, const void* atlas_l,
                                int32_t n_per_region, uint32_t seed, float thresh, unsigned char* mask,
                                unsigned int* stats, void* ws, size_t ws_bytes, void* stream);

/* T[l][p] of each light's network at world points [P][3] (params [L][DGSM_MLP_PARAMS]).
 * With mask (layout of dgsm_mlp_check, [L][regions]) and atlas ([L][K][H][W]),
 * points whose floor texel lies in a flagged region take the trilinear atlas
 * value instead (the plain method as fallback). */
dgsm_status dgsm_mlp_infer(const float* params, const dgsm_lights_t* lights, const dgsm_atlas_desc_t* desc,
                           const void* atlas, const unsigned char* mask, const float* points, int64_t P, float* T,
                           void* ws, size_t ws_bytes, void* stream);

/*
 * Checkpoint of one light's learned field (HOST memory, no device work): the
 * parameters [DGSM_MLP_PARAMS], optionally the Adam moments [2][DGSM_MLP_PARAMS]
 * and the Adam step count (the step0 to resume dgsm_mlp_train with), and the
 * atlas geometry the network was trained for (H, W, K, spacing, r0, r1; the
 * Fourier frequencies follow W).  File: the line "DGSM-MLP 1", a line with a
 * JSON object {"params", "adam", "step", "H", "W", "K", "spacing", "r0", "r1"},
 * then the float32 values, little endian (parameters, then the moments).
 *   dgsm_mlp_save: adam_mv may be NULL (no moments written).  DGSM_EINVAL if
 *     the file cannot be written.
 *   dgsm_mlp_load: params required; adam_mv NULL skips the moments (DGSM_EINVAL
 *     if asked for moments the file lacks); step and desc may be NULL (desc gets
 *     the stored geometry, octahedral, FP32, cull_eps 0).  DGSM_EINVAL on a
 *     missing or malformed file or a different parameter count.
 */
dgsm_status dgsm_mlp_save(const char* path, const float* params, const float* adam_mv, int32_t step,
                          const dgsm_atlas_desc_t* desc);
dgsm_status dgsm_mlp_load(const char* path, float* params, float* adam_mv, int32_t* step,
                          dgsm_atlas_desc_t* desc);

/*
 * dgsm_probe_fit - SH coefficients of an approximate environment probe by
 * weighted ridge least squares (Sec. 3.4):
 *   A = argmin ||W^(1/2) (B A - Y)||_F^2 + lambda ||A||_F^2,
 *   (B^T W B + lambda I) A = B^T W Y,
 * B [n][Kp] the real orthonormal SH basis (the convention of sh_transfer) at
 * the sample directions, W = diag(w).  Accumulated in FP64 in a fixed order
 * and solved by Cholesky in FP64 (B^T W B + lambda I must be positive
 * definite: lambda > 0, or samples that determine every coefficient).
 *   Y : device [n][3] radiance samples (RGB)
 *   D : device [n][3] unit directions;  w: device [n] weights (e.g. the solid
 *       angles of cube-map pixels)
 *   Kp: 1, 4, 9 or 16 (SH degree 0..3);  lambda >= 0
 *   A : device output [Kp][3] float32 (the probe sh_transfer consumes)
 *   ws: device workspace of >= dgsm_probe_fit_workspace_size(Kp) bytes
 */
size_t dgsm_probe_fit_workspace_size(int32_t Kp);
dgsm_status dgsm_probe_fit(const float* Y, const float* D, const float* w, int64_t n, int32_t Kp, float lambda,
                           float* A, void* ws, size_t ws_bytes, void* stream);

/* dgsm_alpha_centroid - c = sum_i alpha_i mu_i / sum_i alpha_i (Sec. 3.2
 * "Receiver-driven region", the alpha-weighted avatar centroid), accumulated
 * in FP64 in a fixed order (bitwise reproducible).  centroid: device [3].
 * n >= 1 and sum alpha > 0 required for a finite result. */
dgsm_status dgsm_alpha_centroid(const dgsm_gaussians_t* gaussians, float* centroid, void* stream);

/* dgsm_check_gaussians - count the Gaussians outside the domain of Eqs. 1-5:
 * a non-finite mean, scale, rotation or opacity, a scale <= 0, an opacity
 * outside [0, 1) (Eq. 5 takes -ln(1 - alpha)), or a zero quaternion.  The
 * build does not check its inputs on the device (timing); callers that load
 * untrusted data run this first.  counter: device int64 scratch (overwritten);
 * *n_bad: host result.  Synchronises `stream`. */
dgsm_status dgsm_check_gaussians(const dgsm_gaussians_t* gaussians, long long* counter, long long* n_bad,
                                 void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DGSM_H */
