"""FP64 oracle: Deep Gaussian Shadow Map build and query.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every quantity is
float64; inputs given as float32 are widened exactly.  No culling, no
tiling, no reordering: the atlas is the plain definition of Sec. 3.2,

    tau(d, t) = sum_i beta_i * int_0^t exp(-1/2 (a_i s^2 + 2 b_i s + c_i)) ds   (Eq. 2)
    T(d, t)   = exp(-tau(d, t))                                              (Eq. 4)

evaluated with the erf primitive of Eq. 3 at every texel centre of the
octahedral atlas and every radial shell.  The only shortcut is an exact skip
of pairs whose whole-ray contribution is below 1e-15 (|erf difference| <= 2),
which bounds the total error by N * 1e-15.

Conventions (readings of the paper where it is silent):
* texel (row i, column j) has u = -1 + (2j+1)/W, v = -1 + (2i+1)/H  (Sec. 3.2,
  "pixel centers"); u runs along columns, v along rows.
* sgn(0) = +1 in the octahedral fold.
* shells: uniform centres t_k = (k + 1/2) t_max / K (Sec. 3.2) or geometric
  radii r_k = r0 (r1/r0)^(k/(K-1)) (the workload configurations).
* query: bilinear in texel space with the octahedral mirror wrap across the
  outer edges, times linear in the fractional shell index, applied to T.
* cube-map atlas (Ablation C, param="cubemap"): see the cube-map section.
"""
from __future__ import annotations

import numpy as np
from scipy import special

SKIP = 1e-15


# ---------------------------------------------------------------------------
# Gaussian parameters (Sec. 3.2 first paragraph, Eq. 5)
# ---------------------------------------------------------------------------

def quaternion_to_matrix(q):
    """Rotation matrices [..., 3, 3] of quaternions (w, x, y, z), normalised first."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def precision_matrix(scale, rot):
    """A_i = Sigma_i^-1 = R diag(s^-2) R^T for Sigma_i = R diag(s^2) R^T (Sec. 3.2)."""
    R = quaternion_to_matrix(rot)
    s = np.asarray(scale, dtype=np.float64)
    return np.einsum("nij,nj,nkj->nik", R, 1.0 / (s * s), R)


def absorption_amplitude(opacity, A, kappa=1.0, beta="trace"):
    """Opacity to absorption, tau* = -ln(1 - alpha):
    "trace"    Eq. 5: beta_i = kappa tau*_i sqrt(tr(A_i)/3) / sqrt(2 pi)
    "constant" beta_i = kappa tau*_i                        (ablation B, mapping 1)
    "density"  beta_i = kappa tau*_i sqrt(det A_i) / (2 pi)^(3/2)
               (ablation B, mappings 3 and 4: A is the precision here, so
               sqrt(det A) = 1 / (s_x s_y s_z); the absorption then integrates
               to kappa tau*_i over space)."""
    alpha = np.asarray(opacity, dtype=np.float64)
    tau_star = -np.log1p(-alpha)
    if beta == "constant":
        return kappa * tau_star
    if beta == "density":
        return kappa * tau_star * np.sqrt(np.linalg.det(A)) / (2.0 * np.pi) ** 1.5
    tr = np.trace(A, axis1=-2, axis2=-1)
    return kappa * tau_star * np.sqrt(tr / 3.0) / np.sqrt(2.0 * np.pi)


def absorption(x, mean, A, beta):
    """Eq. 1: sigma(x) = sum_i beta_i exp(-1/2 (x - mu_i)^T A_i (x - mu_i)), x [..., 3]."""
    x = np.asarray(x, dtype=np.float64)
    diff = x[..., None, :] - np.asarray(mean, dtype=np.float64)
    q = np.einsum("...ni,nij,...nj->...n", diff, A, diff)
    return np.sum(beta * np.exp(-0.5 * q), axis=-1)


# ---------------------------------------------------------------------------
# Closed-form line integral (Eqs. 2-3)
# ---------------------------------------------------------------------------

def ray_quadratic(d, o_L, mean, A):
    """Eq. 2 coefficients for directions d [P,3] and Gaussians [N]: a, b [P,N], c [N].

    a = d^T A d, b = d^T A (o_L - mu), c = (o_L - mu)^T A (o_L - mu).
    """
    d = np.asarray(d, dtype=np.float64)
    m = np.asarray(o_L, dtype=np.float64)[None, :] - np.asarray(mean, dtype=np.float64)
    dd = (d[:, :, None] * d[:, None, :]).reshape(d.shape[0], 9)
    a = dd @ A.reshape(-1, 9).T
    Am = np.einsum("nij,nj->ni", A, m)
    b = d @ Am.T
    c = np.einsum("ni,ni->n", m, Am)
    return a, b, c


def erf_difference(x1, x0):
    """erf(x1) - erf(x0) for x1 >= x0, switching to erfc where both tails agree."""
    x1, x0 = np.broadcast_arrays(np.atleast_1d(np.asarray(x1, dtype=np.float64)),
                                 np.atleast_1d(np.asarray(x0, dtype=np.float64)))
    out = np.array(special.erf(x1) - special.erf(x0))
    pos = x0 > 0
    out[pos] = special.erfc(x0[pos]) - special.erfc(x1[pos])
    neg = x1 < 0
    out[neg] = special.erfc(-x1[neg]) - special.erfc(-x0[neg])
    return out


def line_integral(a, b, c, t):
    """Eq. 3: int_0^t exp(-1/2 (a s^2 + 2 b s + c)) ds, broadcasting a, b, c against t."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    pref = np.sqrt(np.pi / (2 * a)) * np.exp(-0.5 * (c - b * b / a))
    ra = np.sqrt(a / 2)
    return pref * erf_difference(ra * (t + b / a), ra * (b / a))


# ---------------------------------------------------------------------------
# Octahedral parameterisation and shells (Sec. 3.2, "Directional parameterization")
# ---------------------------------------------------------------------------

def _sgn(x):
    return np.where(x >= 0, 1.0, -1.0)


def octahedral_encode(d):
    """psi: unit vectors [..., 3] -> (u, v) in [-1, 1]^2, with sgn(0) = +1."""
    d = np.asarray(d, dtype=np.float64)
    q = d / np.sum(np.abs(d), axis=-1, keepdims=True)
    qx, qy, qz = q[..., 0], q[..., 1], q[..., 2]
    u = np.where(qz >= 0, qx, _sgn(qx) * (1 - np.abs(qy)))
    v = np.where(qz >= 0, qy, _sgn(qy) * (1 - np.abs(qx)))
    return u, v


def octahedral_decode(u, v):
    """psi^-1: undo the fold, z = 1 - |u| - |v|, normalise."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    z = 1 - np.abs(u) - np.abs(v)
    x = np.where(z < 0, _sgn(u) * (1 - np.abs(v)), u)
    y = np.where(z < 0, _sgn(v) * (1 - np.abs(u)), v)
    d = np.stack([x, y, z], axis=-1)
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def texel_uv(H, W):
    """(u, v) of every texel centre, arrays [H, W]."""
    j = np.arange(W, dtype=np.float64)
    i = np.arange(H, dtype=np.float64)
    u = -1 + (2 * j + 1) / W
    v = -1 + (2 * i + 1) / H
    return np.broadcast_to(u[None, :], (H, W)), np.broadcast_to(v[:, None], (H, W))


def texel_directions(H, W, param="octahedral"):
    """Unit direction of every texel centre, [H, W, 3]."""
    if param == "cubemap":
        return cube_texel_directions(H, W)
    if param != "octahedral":
        raise ValueError(param)
    u, v = texel_uv(H, W)
    return octahedral_decode(u, v)


# ---------------------------------------------------------------------------
# Cube-map parameterisation (Ablation C)
# ---------------------------------------------------------------------------
# The paper compares its octahedral atlas with a six-face cube map but does
# not fix the cube map's layout or filtering; the reading used here:
# * faces of F x F texels, face f = 2 m + (0 for the + side, 1 for the - side)
#   of major axis m in (x, y, z), stored in a 2F x 3F atlas (H = 2F, W = 3F)
#   at block row f // 3, block column f % 3;
# * on face (m, sign) texel (b, a) (row b, column a inside the face) has face
#   coordinates s = -1 + (2a + 1)/F, t = -1 + (2b + 1)/F and the direction
#   proportional to d[m] = sign, d[(m+1) % 3] = s, d[(m+2) % 3] = t;
# * a lookup picks the face of the largest |component| (the first axis on
#   ties) and interpolates bilinearly inside that face, clamped to the face's
#   edge texels: nothing is filtered across faces (the seams the ablation
#   measures).

def cube_decode(face, s, t):
    """Unit direction of face coordinates (s, t) in [-1, 1] on the given faces."""
    face = np.asarray(face, dtype=np.int64)
    s, t = np.broadcast_arrays(np.asarray(s, dtype=np.float64), np.asarray(t, dtype=np.float64))
    face = np.broadcast_to(face, s.shape)
    m = face // 2
    sign = np.where(face % 2 == 0, 1.0, -1.0)
    d = np.zeros(s.shape + (3,))
    for axis in range(3):
        sel = m == axis
        d[sel, axis] = sign[sel]
        d[sel, (axis + 1) % 3] = s[sel]
        d[sel, (axis + 2) % 3] = t[sel]
    return d / np.linalg.norm(d, axis=-1, keepdims=True)


def cube_face(d):
    """Face of each direction d [..., 3] (FP64): the axis of the largest
    |component| (the first on ties) and its sign.  Points within rounding of a
    tie can land on the other face in a lower precision; tests leave them out."""
    d = np.asarray(d, dtype=np.float64)
    a = np.abs(d)
    m = np.where((a[..., 0] >= a[..., 1]) & (a[..., 0] >= a[..., 2]), 0, np.where(a[..., 1] >= a[..., 2], 1, 2))
    comp = np.take_along_axis(d, m[..., None], axis=-1)[..., 0]
    return 2 * m + (comp < 0)


def cube_encode(d, face):
    """Face coordinates (s, t) of directions d [..., 3] on the given faces."""
    d = np.asarray(d, dtype=np.float64)
    m = np.asarray(face) // 2
    major = np.abs(np.take_along_axis(d, m[..., None], axis=-1)[..., 0])
    s = np.take_along_axis(d, ((m + 1) % 3)[..., None], axis=-1)[..., 0] / major
    t = np.take_along_axis(d, ((m + 2) % 3)[..., None], axis=-1)[..., 0] / major
    return s, t


def cube_texel_directions(H, W):
    """Unit direction of every texel centre of a 2F x 3F cube-map atlas, [H, W, 3]."""
    F = H // 2
    if H != 2 * F or W != 3 * F or F < 2:
        raise ValueError("cube-map atlas must be 2F x 3F with F >= 2")
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    face = 3 * (i // F) + j // F
    s = -1 + (2 * (j % F) + 1) / F
    t = -1 + (2 * (i % F) + 1) / F
    return cube_decode(face, s, t)


def shell_radii(K, spacing="geometric", r0=0.05, r1=8.0):
    """Radial sample distances t_k [K]."""
    k = np.arange(K, dtype=np.float64)
    if spacing == "geometric":
        return r0 * (r1 / r0) ** (k / (K - 1))
    if spacing == "uniform":
        return (k + 0.5) * r1 / K
    raise ValueError(spacing)


# ---------------------------------------------------------------------------
# Build
# ---------------------------------------------------------------------------

def gaussian_terms(g, kappa=1.0, beta="trace"):
    """(mean, A, beta) in float64 for a Gaussian set with .mean/.scale/.rot/.opacity."""
    A = precision_matrix(g.scale, g.rot)
    beta = absorption_amplitude(g.opacity, A, kappa, beta)
    return np.asarray(g.mean, dtype=np.float64), A, beta


def optical_depth(dirs, t, o_L, mean, A, beta, chunk=2048):
    """tau(d_p, t_k) [P, K] for unit directions dirs [P, 3] (Eqs. 2-3)."""
    dirs = np.asarray(dirs, dtype=np.float64).reshape(-1, 3)
    t = np.asarray(t, dtype=np.float64)
    P, K = dirs.shape[0], t.shape[0]
    tau = np.zeros((P, K))
    for s in range(0, mean.shape[0], chunk):
        e = slice(s, s + chunk)
        a, b, c = ray_quadratic(dirs, o_L, mean[e], A[e])
        pref = beta[e][None, :] * np.sqrt(np.pi / (2 * a)) * np.exp(-0.5 * (c[None, :] - b * b / a))
        p_idx, n_idx = np.nonzero(2 * pref >= SKIP)
        if p_idx.size == 0:
            continue
        aa, bb = a[p_idx, n_idx], b[p_idx, n_idx]
        ra = np.sqrt(aa / 2)[:, None]
        boa = (bb / aa)[:, None]
        vals = pref[p_idx, n_idx][:, None] * erf_difference(ra * (t[None, :] + boa), ra * boa)
        np.add.at(tau, p_idx, vals)
    return tau


def build(light, gaussians, H, W, K, spacing="geometric", r0=0.05, r1=8.0, kappa=1.0, beta="trace",
          param="octahedral"):
    """Transmittance atlas T[K, H, W] for one point light (Eqs. 2-4, Sec. 3.2)."""
    mean, A, beta = gaussian_terms(gaussians, kappa, beta)
    dirs = texel_directions(H, W, param).reshape(-1, 3)
    t = shell_radii(K, spacing, r0, r1)
    tau = optical_depth(dirs, t, light, mean, A, beta)
    return np.exp(-tau).T.reshape(K, H, W)


def build_texels(light, gaussians, rows, cols, K, spacing="geometric", r0=0.05, r1=8.0,
                 kappa=1.0, H=None, W=None, param="octahedral"):
    """T[len(rows), K] at the given texels of an H x W atlas (sampled parity)."""
    mean, A, beta = gaussian_terms(gaussians, kappa)
    dirs = _texel_dirs_at(rows, cols, H, W, param)
    t = shell_radii(K, spacing, r0, r1)
    return np.exp(-optical_depth(dirs, t, light, mean, A, beta))


def _texel_dirs_at(rows, cols, H, W, param):
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if param == "cubemap":
        return cube_texel_directions(H, W)[rows, cols]
    u = -1 + (2 * cols + 1) / W
    v = -1 + (2 * rows + 1) / H
    return octahedral_decode(u, v)


def transmittance_at(light, gaussians, points, kappa=1.0, chunk=4096):
    """Exact T(d, r) = exp(-tau(d, r)) at world points (Eqs. 2-4 at the point itself,
    no atlas): d = (x - o_L)/|x - o_L|, r = |x - o_L|."""
    mean, A, beta = gaussian_terms(gaussians, kappa)
    diff = np.asarray(points, dtype=np.float64) - np.asarray(light, dtype=np.float64)
    r = np.linalg.norm(diff, axis=1)
    dirs = diff / r[:, None]
    tau = np.zeros(r.shape[0])
    for s in range(0, mean.shape[0], chunk):
        e = slice(s, s + chunk)
        a, b, c = ray_quadratic(dirs, light, mean[e], A[e])
        pref = beta[e][None, :] * np.sqrt(np.pi / (2 * a)) * np.exp(-0.5 * (c[None, :] - b * b / a))
        ra = np.sqrt(a / 2)
        boa = b / a
        tau += np.sum(pref * erf_difference(ra * (r[:, None] + boa), ra * boa), axis=1)
    return np.exp(-tau)


def dropped_depth_bound(light, gaussians, rows, cols, H, W, eps, kappa=1.0, param="octahedral", chunk=65536):
    """Error budget of a culled build at the given texels (Sec. 3.2 "Occluder
    culling via light-space footprints").  A shell's optical depth integrates
    Eq. 2 along the texel ray from the light (t >= 0), so leaving Gaussian i
    out along direction d lowers every shell by at most its depth along the
    whole ray, beta_i times Eq. 3 with t -> inf; a culled build may leave a
    Gaussian out only where that depth is at most eps.  Returns per texel (the
    sum of the ray depths at or below eps -- the most optical depth such a
    build can drop there -- and the number of Gaussians above eps, each of
    which a build evaluates)."""
    mean, A, beta = gaussian_terms(gaussians, kappa)
    dirs = _texel_dirs_at(rows, cols, H, W, param)
    dropped = np.zeros(dirs.shape[0])
    kept = np.zeros(dirs.shape[0], dtype=np.int64)
    for s in range(0, mean.shape[0], chunk):
        e = slice(s, s + chunk)
        a, b, c = ray_quadratic(dirs, light, mean[e], A[e])
        ray = beta[e][None, :] * line_integral(a, b, c[None, :], np.inf)
        small = ray <= eps
        dropped += np.where(small, ray, 0.0).sum(axis=1)
        kept += (~small).sum(axis=1)
    return dropped, kept


# ---------------------------------------------------------------------------
# Query (Sec. 3.3)
# ---------------------------------------------------------------------------

def wrap_texel(i, j, H, W):
    """Octahedral mirror wrap of integer texel indices (possibly one step outside).

    Across the left/right edge (u = -+1) the map identifies (u, v) with (u, -v);
    across the top/bottom edge (v = -+1) it identifies (u, v) with (-u, v).
    """
    i = np.asarray(i).copy()
    j = np.asarray(j).copy()
    out = j < 0
    j[out], i[out] = 0, H - 1 - i[out]
    out = j >= W
    j[out], i[out] = W - 1, H - 1 - i[out]
    out = i < 0
    i[out], j[out] = 0, W - 1 - j[out]
    out = i >= H
    i[out], j[out] = H - 1, W - 1 - j[out]
    return i, j


def query_coords(light, points, H, W, K, spacing="geometric", r0=0.05, r1=8.0):
    """Continuous texel coordinates (i_f, j_f) and fractional shell k_f of points."""
    diff = np.asarray(points, dtype=np.float64) - np.asarray(light, dtype=np.float64)
    r = np.linalg.norm(diff, axis=-1)
    diff = np.where(r[:, None] > 0, diff, np.array([0.0, 0.0, 1.0]))
    u, v = octahedral_encode(diff)
    jf = (u + 1) * W / 2 - 0.5
    i_f = (v + 1) * H / 2 - 0.5
    if spacing == "geometric":
        with np.errstate(divide="ignore"):
            kf = (K - 1) * np.log(np.maximum(r, 1e-300) / r0) / np.log(r1 / r0)
    else:
        kf = r * K / r1 - 0.5
    kf = np.clip(kf, 0.0, K - 1)
    return i_f, jf, kf


def _corner_weights(i_f, jf, kf, K):
    i0 = np.floor(i_f).astype(np.int64)
    j0 = np.floor(jf).astype(np.int64)
    k0 = np.minimum(np.floor(kf).astype(np.int64), K - 2)
    return i0, j0, k0, i_f - i0, jf - j0, kf - k0


def _shell_coord(r, K, spacing, r0, r1):
    if spacing == "geometric":
        with np.errstate(divide="ignore"):
            kf = (K - 1) * np.log(np.maximum(r, 1e-300) / r0) / np.log(r1 / r0)
    else:
        kf = r * K / r1 - 0.5
    return np.clip(kf, 0.0, K - 1)


def cube_cells(light, points, H, W, K, spacing="geometric", r0=0.05, r1=8.0):
    """Cube-map lookup cells: floor texel (i0, j0) with i0 + 1, j0 + 1 inside the
    same face, lower shell k0 and the fractions (fi, fj, fk)."""
    F = H // 2
    diff = np.asarray(points, dtype=np.float64).reshape(-1, 3) - np.asarray(light, dtype=np.float64)
    r = np.linalg.norm(diff, axis=-1)
    diff = np.where(r[:, None] > 0, diff, np.array([0.0, 0.0, 1.0]))
    face = cube_face(diff)
    s, t = cube_encode(diff, face)

    def axis(c):
        cf = np.clip((c + 1) * F / 2 - 0.5, 0.0, F - 1)
        c0 = np.minimum(np.floor(cf).astype(np.int64), F - 2)
        return c0, cf - c0

    a0, fa = axis(s)
    b0, fb = axis(t)
    kf = _shell_coord(r, K, spacing, r0, r1)
    k0 = np.minimum(np.floor(kf).astype(np.int64), K - 2)
    return (face // 3) * F + b0, (face % 3) * F + a0, k0, fb, fa, kf - k0


def _cells(light, points, H, W, K, spacing, r0, r1, param):
    """(i0, j0, k0, fi, fj, fk) of the trilinear cell of each point."""
    if param == "cubemap":
        return cube_cells(light, points, H, W, K, spacing, r0, r1)
    if param != "octahedral":
        raise ValueError(param)
    i_f, jf, kf = query_coords(light, points, H, W, K, spacing, r0, r1)
    return _corner_weights(i_f, jf, kf, K)


def _neighbour(i, j, H, W, param):
    """Texel read at integer (i, j): octahedral wrap, identity inside a cube face."""
    if param == "cubemap":
        return np.asarray(i), np.asarray(j)
    return wrap_texel(i, j, H, W)


def query(table, light, points, spacing="geometric", r0=0.05, r1=8.0, param="octahedral"):
    """Trilinear lookup of T[K, H, W] at world points [P, 3] (Sec. 3.3)."""
    K, H, W = table.shape
    i0, j0, k0, fi, fj, fk = _cells(light, points, H, W, K, spacing, r0, r1, param)
    out = np.zeros(i0.shape)
    for di, wi in ((0, 1 - fi), (1, fi)):
        for dj, wj in ((0, 1 - fj), (1, fj)):
            ii, jj = _neighbour(i0 + di, j0 + dj, H, W, param)
            for dk, wk in ((0, 1 - fk), (1, fk)):
                out += wi * wj * wk * table[k0 + dk, ii, jj]
    return out


def roi_region(light, receivers, H, W, K, box=None, spacing="geometric", r0=0.05, r1=8.0, param="octahedral"):
    """Receiver-driven region of interest (Sec. 3.2): receivers inside the box
    B = {|x - cx| <= R, |y - cy| <= R, zmin <= z <= zmax} (box = (cx, cy, R,
    zmin, zmax); None or R <= 0 keeps every point) mark the texels their
    trilinear lookup reads (the floor texel and its three neighbours, wrapped);
    the radial range is [min k0, max k0 + 1] over the receivers.
    Returns (texel mask [H, W] bool, k_min, k_max); k_min > k_max if empty."""
    pts = np.asarray(receivers, dtype=np.float64).reshape(-1, 3)
    if box is not None and box[2] > 0:
        cx, cy, R, zmin, zmax = box
        keep = (np.abs(pts[:, 0] - cx) <= R) & (np.abs(pts[:, 1] - cy) <= R) & (pts[:, 2] >= zmin) & \
               (pts[:, 2] <= zmax)
        pts = pts[keep]
    mask = np.zeros((H, W), dtype=bool)
    if pts.shape[0] == 0:
        return mask, K, -1
    i0, j0, k0, _, _, _ = _cells(light, pts, H, W, K, spacing, r0, r1, param)
    for di in (0, 1):
        for dj in (0, 1):
            ii, jj = _neighbour(i0 + di, j0 + dj, H, W, param)
            mask[ii, jj] = True
    return mask, int(k0.min()), int(k0.max() + 1)


def build_roi(light, gaussians, H, W, K, receivers, box=None, spacing="geometric", r0=0.05, r1=8.0,
              kappa=1.0, param="octahedral"):
    """T[K, H, W] of the full build inside the receiver region, 1 outside it."""
    mask, k_lo, k_hi = roi_region(light, receivers, H, W, K, box, spacing, r0, r1, param)
    T = build(light, gaussians, H, W, K, spacing, r0, r1, kappa, param=param)
    keep = mask[None, :, :] & (np.arange(K)[:, None, None] >= k_lo) & (np.arange(K)[:, None, None] <= k_hi)
    return np.where(keep, T, 1.0)


def footprint_stencil7():
    """Deterministic 7-point footprint stencil (Sec. 3.3, Ablation A): offsets
    in the principal-axes frame z = 0 and +-e_j (one standard deviation along
    each axis), weights proportional to the Gaussian kernel exp(-|z|^2 / 2) at
    each offset, normalised to sum 1.  (The paper names the stencil but not its
    offsets or weights; this is the reading used throughout.)"""
    z = np.zeros((7, 3))
    for j in range(3):
        z[1 + 2 * j, j] = 1.0
        z[2 + 2 * j, j] = -1.0
    k = np.exp(-0.5 * np.sum(z * z, axis=1))
    return z, k / k.sum()


def query_footprint(table, light, gaussians, z, w, spacing="geometric", r0=0.05, r1=8.0, param="octahedral"):
    """Footprint-averaged transmittance of each Gaussian (Sec. 3.3, Ablation A):
    T_g = sum_i w_i T(mu_g + R_g (s_g * z_i)), with T the trilinear atlas
    lookup.  z [n, 3] offsets in the principal-axes frame (standard-normal
    draws for Monte Carlo sampling, or a stencil), w [n] weights summing to 1."""
    z = np.asarray(z, np.float64).reshape(-1, 3)
    w = np.asarray(w, np.float64).reshape(-1)
    mu = gaussians.mean.astype(np.float64)
    R = quaternion_to_matrix(gaussians.rot)
    s = gaussians.scale.astype(np.float64)
    out = np.zeros(gaussians.n)
    for zi, wi in zip(z, w):
        x = mu + np.einsum("nij,nj->ni", R, s * zi)
        out += wi * query(table, light, x, spacing, r0, r1, param)
    return out


def query_exact(light, gaussians, points, H, W, K, spacing="geometric", r0=0.05, r1=8.0,
                kappa=1.0, param="octahedral"):
    """Query at points without a stored atlas: the 8 texel values each point
    interpolates are computed from Eqs. 2-4 directly (for full-size sampling)."""
    mean, A, beta = gaussian_terms(gaussians, kappa)
    i0, j0, k0, fi, fj, fk = _cells(light, points, H, W, K, spacing, r0, r1, param)
    t_all = shell_radii(K, spacing, r0, r1)
    out = np.zeros(i0.shape)
    for di, wi in ((0, 1 - fi), (1, fi)):
        for dj, wj in ((0, 1 - fj), (1, fj)):
            ii, jj = _neighbour(i0 + di, j0 + dj, H, W, param)
            dirs = _texel_dirs_at(ii, jj, H, W, param)
            tau = optical_depth(dirs, t_all, light, mean, A, beta)
            T = np.exp(-tau)
            rows = np.arange(len(ii))
            for dk, wk in ((0, 1 - fk), (1, fk)):
                out += wi * wj * wk * T[rows, k0 + dk]
    return out
