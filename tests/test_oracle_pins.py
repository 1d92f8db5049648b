"""Pins for the FP64 oracle: checks against what the paper and mathematics fix.

None of these re-types an oracle formula.  They use numerical quadrature of
the absorption field (Eq. 1), closed forms derived by hand, exact symmetries
and invariants of Eqs. 2-5, library routines for special cases (scipy's
rotations, complex spherical harmonics, adaptive quadrature) and brute force
on tiny inputs.
"""
import math

import numpy as np
import pytest
from scipy import integrate, special
from scipy.spatial.transform import Rotation

from oracle import dgsm as od
from oracle import sh as osh
import synth


def tiny_scene(seed=0, n=3, lo=0.6, hi=1.6, median=0.15):
    rng = np.random.default_rng(seed)
    return synth.random_gaussians(rng, rng.uniform(lo, hi, (n, 3)), median)


# ---------------------------------------------------------------------------
# Gaussian parameters
# ---------------------------------------------------------------------------

def test_quaternion_matches_scipy_rotation():
    rng = np.random.default_rng(1)
    q = rng.standard_normal((50, 4))
    R = od.quaternion_to_matrix(q)
    ref = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()  # scipy is scalar-last
    assert np.max(np.abs(R - ref)) < 1e-14


def test_precision_eigenvalues_are_inverse_variances():
    g = tiny_scene(2, n=20)
    A = od.precision_matrix(g.scale, g.rot)
    for k in range(g.n):
        ev = np.linalg.eigvalsh(A[k])
        ref = np.sort(1.0 / g.scale[k].astype(np.float64) ** 2)
        assert np.allclose(ev, ref, rtol=1e-12)


# ---------------------------------------------------------------------------
# Eq. 3 against quadrature of Eq. 2 / Eq. 1
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(6))
def test_closed_form_matches_quadrature_of_quadratic(seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 50.0)
    tc = rng.uniform(-2, 3)                 # centre of the Gaussian along the ray
    b = -a * tc
    c = b * b / a + rng.uniform(0, 4)       # c - b^2/a >= 0 for a PSD form
    for t in (0.1, 0.7, 2.5, 6.0):
        got = od.line_integral(a, b, c, t)
        ref, _ = integrate.quad(lambda s: math.exp(-0.5 * (a * s * s + 2 * b * s + c)), 0.0, t,
                                epsabs=0, epsrel=1e-13, limit=200, points=[min(max(tc, 0), t)])
        assert abs(got - ref) <= 1e-10 * max(abs(ref), 1e-300) + 1e-300


def test_optical_depth_matches_quadrature_of_absorption_field():
    """Chain Eq. 1 -> Eq. 2 -> Eq. 3 for anisotropic Gaussians on random rays."""
    g = tiny_scene(3, n=6)
    mean, A, beta = od.gaussian_terms(g)
    o_L = np.array([0.1, -0.2, 0.05])
    rng = np.random.default_rng(4)
    # aim the rays at the Gaussians so that the integrals are not negligible
    targets = mean[rng.integers(0, g.n, 5)] + 0.05 * rng.standard_normal((5, 3))
    dirs = targets - o_L
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    t = np.array([0.3, 1.0, 1.7, 2.4, 5.0])
    tau = od.optical_depth(dirs, t, o_L, mean, A, beta)
    for p in range(dirs.shape[0]):
        for k, tk in enumerate(t):
            ref, _ = integrate.quad(lambda s: od.absorption(o_L + s * dirs[p], mean, A, beta), 0.0, tk,
                                    epsabs=1e-14, epsrel=1e-12, limit=400)
            assert abs(tau[p, k] - ref) <= 1e-9 * max(ref, 1e-6)


# ---------------------------------------------------------------------------
# Eq. 5 calibration: isotropic, on-axis closed form
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("alpha,s,D,kappa", [(0.7, 0.05, 2.0, 1.0), (0.3, 0.2, 1.0, 1.0),
                                             (0.95, 0.02, 3.0, 0.5), (0.5, 0.1, 0.15, 2.0)])
def test_isotropic_on_axis_closed_form(alpha, s, D, kappa):
    # tau(t) = kappa tau*/2 [erf((t - D)/(s sqrt2)) + erf(D/(s sqrt2))], derived by hand
    g = synth.Gaussians(np.array([[0.0, 0.0, D]], np.float32), np.full((1, 3), s, np.float32),
                        np.array([[1, 0, 0, 0]], np.float32), np.array([alpha], np.float32))
    mean, A, beta = od.gaussian_terms(g, kappa)
    a32 = float(np.float32(alpha))
    s = float(np.float32(s))
    D = float(np.float32(D))
    tau_star = -math.log1p(-a32)
    t = np.array([0.5 * D, D, D + s, D + 10 * s, 50.0])
    tau = od.optical_depth(np.array([[0.0, 0.0, 1.0]]), t, np.zeros(3), mean, A, beta)[0]
    ref = kappa * tau_star / 2 * (special.erf((t - D) / (s * math.sqrt(2))) + special.erf(D / (s * math.sqrt(2))))
    assert np.allclose(tau, ref, rtol=1e-12, atol=1e-15)
    if D > 8 * s:   # far field: T(inf) = (1 - alpha)^kappa, the 3DGS opacity
        assert abs(math.exp(-tau[-1]) - (1 - a32) ** kappa) < 1e-12


# ---------------------------------------------------------------------------
# Whole-build invariants and special cases
# ---------------------------------------------------------------------------

ATL = dict(H=8, W=8, K=6, spacing="geometric", r0=0.05, r1=8.0)


def test_empty_and_transparent_scene_is_fully_lit():
    T = od.build(np.zeros(3), synth.Gaussians.empty(), **ATL)
    assert T.shape == (6, 8, 8) and np.all(T == 1.0)
    g = tiny_scene(5, n=4)
    g.opacity[:] = 0.0
    assert np.all(od.build(np.zeros(3), g, **ATL) == 1.0)


def test_transmittance_monotone_in_radius():
    g = tiny_scene(6, n=30, lo=-2, hi=2, median=0.2)
    T = od.build(np.array([0.05, 0.02, -0.03]), g, 16, 16, 12)
    assert np.all(np.diff(T, axis=0) <= 0)
    assert np.all((T > 0) & (T <= 1))


def test_additivity_over_gaussian_sets():
    g = tiny_scene(7, n=12, lo=-2, hi=2, median=0.2)
    light = np.array([0.1, 0.0, 0.0])
    T = od.build(light, g, **ATL)
    T1 = od.build(light, g.subset(np.arange(0, 5)), **ATL)
    T2 = od.build(light, g.subset(np.arange(5, 12)), **ATL)
    assert np.allclose(T, T1 * T2, rtol=1e-12, atol=1e-15)


def test_kappa_power_law():
    g = tiny_scene(8, n=10, lo=-2, hi=2, median=0.2)
    light = np.array([0.0, 0.1, 0.0])
    T1 = od.build(light, g, **ATL)
    T3 = od.build(light, g, **ATL, kappa=2.5)
    assert np.allclose(T3, T1 ** 2.5, rtol=1e-11, atol=1e-15)


def test_length_scale_invariance():
    g = tiny_scene(9, n=10, lo=-2, hi=2, median=0.2)
    light = np.array([0.05, 0.0, 0.1])
    lam = 4.0   # a power of two keeps the float32 inputs exact
    g2 = synth.Gaussians(g.mean * lam, g.scale * lam, g.rot, g.opacity)
    T1 = od.build(light, g, 8, 8, 6, r0=0.05, r1=8.0)
    T2 = od.build(light * lam, g2, 8, 8, 6, r0=0.05 * lam, r1=8.0 * lam)
    assert np.allclose(T1, T2, rtol=1e-12, atol=1e-14)


def test_brute_force_quadrature_on_tiny_atlas():
    g = tiny_scene(10, n=3, lo=-1.2, hi=1.2, median=0.25)
    light = np.zeros(3)
    H = W = 4
    K = 4
    T = od.build(light, g, H, W, K, r0=0.3, r1=3.0)
    mean, A, beta = od.gaussian_terms(g)
    t = 0.3 * (10.0 ** (np.arange(K) / (K - 1)))
    for i in range(H):
        for j in range(W):
            u = -1 + (2 * j + 1) / W
            v = -1 + (2 * i + 1) / H
            z = 1 - abs(u) - abs(v)
            x, y = (u, v) if z >= 0 else (math.copysign(1 - abs(v), u), math.copysign(1 - abs(u), v))
            d = np.array([x, y, z]) / math.sqrt(x * x + y * y + z * z)
            for k in range(K):
                tau, _ = integrate.quad(lambda s: od.absorption(s * d, mean, A, beta), 0, t[k],
                                        epsabs=1e-13, epsrel=1e-11, limit=400)
                assert abs(T[k, i, j] - math.exp(-tau)) < 1e-10


# ---------------------------------------------------------------------------
# Octahedral map: round trip and exact symmetries of the atlas
# ---------------------------------------------------------------------------

def test_octahedral_round_trip_at_texel_centres():
    for H, W in ((8, 8), (6, 10), (32, 32)):
        u, v = od.texel_uv(H, W)
        uu, vv = od.octahedral_encode(od.octahedral_decode(u, v))
        assert np.max(np.abs(uu - u)) < 1e-14 and np.max(np.abs(vv - v)) < 1e-14


def test_octahedral_encode_is_onto_the_square_and_folds_lower_hemisphere():
    rng = np.random.default_rng(11)
    d = rng.standard_normal((2000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    u, v = od.octahedral_encode(d)
    assert np.all(np.abs(u) <= 1) and np.all(np.abs(v) <= 1)
    up = d[:, 2] >= 0
    assert np.all(np.abs(u[up]) + np.abs(v[up]) <= 1 + 1e-15)
    assert np.all(np.abs(u[~up]) + np.abs(v[~up]) >= 1 - 1e-15)


def _rotated_scene(g, rot: Rotation):
    mean = rot.apply(g.mean.astype(np.float64)).astype(np.float32)
    q = (rot * Rotation.from_quat(g.rot[:, [1, 2, 3, 0]].astype(np.float64))).as_quat()
    return synth.Gaussians(mean, g.scale, q[:, [3, 0, 1, 2]].astype(np.float32), g.opacity)


def test_atlas_symmetry_mirror_x_is_column_flip():
    g = tiny_scene(12, n=15, lo=-2, hi=2, median=0.2)
    gm = synth.Gaussians(g.mean * np.array([-1, 1, 1], np.float32), g.scale,
                         g.rot * np.array([1, 1, -1, -1], np.float32), g.opacity)  # reflect x
    T = od.build(np.zeros(3), g, 8, 8, 5)
    Tm = od.build(np.zeros(3), gm, 8, 8, 5)
    assert np.allclose(Tm, T[:, :, ::-1], rtol=1e-9, atol=1e-12)


def test_atlas_symmetry_quarter_turn_about_z():
    g = tiny_scene(13, n=15, lo=-2, hi=2, median=0.2)
    # exact float32 quarter turn: (x, y, z) -> (-y, x, z)
    rot = Rotation.from_euler("z", 90, degrees=True)
    gr = _rotated_scene(g, rot)
    gr.mean[:] = np.stack([-g.mean[:, 1], g.mean[:, 0], g.mean[:, 2]], 1)
    T = od.build(np.zeros(3), g, 8, 8, 5)
    Tr = od.build(np.zeros(3), gr, 8, 8, 5)
    # (u, v) -> (-v, u): texel (i, j) -> (j, W-1-i)
    W = 8
    ref = np.empty_like(T)
    for i in range(8):
        for j in range(8):
            ref[:, j, W - 1 - i] = T[:, i, j]
    assert np.allclose(Tr, ref, rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------------------
# Query
# ---------------------------------------------------------------------------

def _random_table(K, H, W, seed=14):
    rng = np.random.default_rng(seed)
    return rng.uniform(0, 1, (K, H, W))


def test_query_reproduces_texel_values_at_centres_and_shells():
    K, H, W = 5, 8, 8
    table = _random_table(K, H, W)
    t = od.shell_radii(K, "geometric", 0.05, 8.0)
    d = od.texel_directions(H, W)
    light = np.array([0.3, -0.2, 0.1])
    for k in range(K):
        pts = light + t[k] * d.reshape(-1, 3)
        got = od.query(table, light, pts)
        assert np.allclose(got, table[k].reshape(-1), atol=1e-10)


def test_query_partition_of_unity_and_bounds():
    K, H, W = 6, 8, 8
    rng = np.random.default_rng(15)
    pts = rng.uniform(-6, 6, (4000, 3))
    assert np.allclose(od.query(np.full((K, H, W), 0.37), np.zeros(3), pts), 0.37, atol=1e-14)
    table = _random_table(K, H, W)
    got = od.query(table, np.zeros(3), pts)
    assert np.all(got >= table.min() - 1e-12) and np.all(got <= table.max() + 1e-12)


def test_query_is_continuous_across_the_octahedral_seams():
    K, H, W = 4, 8, 8
    table = _random_table(K, H, W, seed=16)
    rng = np.random.default_rng(17)
    for _ in range(200):
        # a direction on the lower-hemisphere seam y = 0 (the u = +-1 edge) or x = 0
        a = rng.uniform(0.05, 0.95)
        sx = rng.choice([-1, 1])
        if rng.uniform() < 0.5:
            base = np.array([sx * a, 0.0, -(1 - a)])
            eps = np.array([0.0, 1e-9, 0.0])
        else:
            base = np.array([0.0, sx * a, -(1 - a)])
            eps = np.array([1e-9, 0.0, 0.0])
        r = rng.uniform(0.1, 7.0)
        p1 = r * (base + eps) / np.linalg.norm(base + eps)
        p2 = r * (base - eps) / np.linalg.norm(base - eps)
        v1, v2 = od.query(table, np.zeros(3), np.stack([p1, p2]))
        assert abs(v1 - v2) < 1e-6


def test_wrap_maps_corners_to_the_opposite_corner():
    i, j = od.wrap_texel(np.array([-1, 8, -1, 8]), np.array([-1, 8, 8, -1]), 8, 8)
    assert list(zip(i, j)) == [(7, 7), (0, 0), (7, 0), (0, 7)]


# ---------------------------------------------------------------------------
# SH basis and radiance transfer
# ---------------------------------------------------------------------------

def test_real_sh_matches_scipy_complex_harmonics():
    rng = np.random.default_rng(18)
    d = rng.standard_normal((300, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    th = np.arccos(np.clip(d[:, 2], -1, 1))
    ph = np.arctan2(d[:, 1], d[:, 0])
    B = osh.real_sh(4, d)
    for l in range(5):
        for m in range(-l, l + 1):
            Y = special.sph_harm_y(l, abs(m), th, ph)   # includes the Condon-Shortley phase
            if m > 0:
                ref = math.sqrt(2) * (-1) ** m * Y.real
            elif m < 0:
                ref = math.sqrt(2) * (-1) ** abs(m) * Y.imag
            else:
                ref = Y.real
            assert np.max(np.abs(B[:, l * l + l + m] - ref)) < 1e-12


def test_real_sh_orthonormal_by_quadrature():
    x, wx = np.polynomial.legendre.leggauss(40)
    nph = 80
    ph = (np.arange(nph) + 0.5) * 2 * math.pi / nph
    X, P = np.meshgrid(x, ph, indexing="ij")
    st = np.sqrt(1 - X * X)
    d = np.stack([st * np.cos(P), st * np.sin(P), X], -1).reshape(-1, 3)
    w = (wx[:, None] * np.full(nph, 2 * math.pi / nph)[None, :]).reshape(-1)
    B = osh.real_sh(3, d)
    G = (B * w[:, None]).T @ B
    assert np.max(np.abs(G - np.eye(16))) < 1e-12


def test_transfer_constant_probe_special_case():
    rng = np.random.default_rng(19)
    probe = np.zeros((16, 3))
    probe[0] = [0.9, 1.3, 0.4]
    n = rng.standard_normal((50, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    eps = 1e-3
    s = osh.transfer_scale(probe, n, 16, 32, q=1.0, clip_max=10.0, eps=eps)
    L = probe[0] * osh.C0                     # Y_00 = 1/(2 sqrt(pi))
    dirs, w = osh.latlong_grid(16, 32)
    S = np.maximum(0, n @ dirs.T)
    den = (S * w).sum(1)
    assert np.allclose(s, L[None, :] * (den / (den + eps))[:, None], rtol=1e-13)


def test_transfer_lambertian_limit_matches_irradiance_convolution():
    """q = 1 and a fine grid: s_c(n) -> E_c(n) / pi with the clamped-cosine SH
    convolution A_0 = pi, A_1 = 2 pi / 3, A_2 = pi / 4, A_3 = 0."""
    rng = np.random.default_rng(20)
    probe = rng.normal(0, 0.3, (16, 3))
    probe[0] = rng.uniform(2.0, 3.0, 3)          # keep E > 0 so no clip engages
    n = rng.standard_normal((20, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    s = osh.transfer_scale(probe, n, 400, 800, q=1.0, clip_max=100.0, eps=0.0)
    Ahat = np.array([math.pi] + [2 * math.pi / 3] * 3 + [math.pi / 4] * 5 + [0.0] * 7)
    E = osh.real_sh(3, n) @ (Ahat[:, None] * probe)
    assert np.max(np.abs(s - E / math.pi)) < 2e-4


def test_transfer_glossy_denominator_funk_hecke():
    # sum_j w_j max(0, <w_j, n>)^q -> 2 pi / (q + 1) (times the grid cell area)
    for q in (1.0, 4.0, 16.0):
        dirs, w = osh.latlong_grid(400, 800)
        cell = (math.pi / 400) * (2 * math.pi / 800)
        n = np.array([0.3, -0.5, 0.81])
        n /= np.linalg.norm(n)
        den = (np.maximum(0, dirs @ n) ** q * w).sum() * cell
        assert abs(den - 2 * math.pi / (q + 1)) < 2e-4


def test_normals_are_smallest_axis_and_face_outward():
    g = tiny_scene(21, n=40, lo=-1, hi=1)
    c = osh.alpha_centroid(g.mean, g.opacity)
    n = osh.normals(g.rot, g.scale, g.mean, c)
    R = Rotation.from_quat(g.rot[:, [1, 2, 3, 0]].astype(np.float64)).as_matrix()
    for k in range(g.n):
        ax = int(np.argmin(g.scale[k]))
        assert abs(abs(n[k] @ R[k][:, ax]) - 1) < 1e-12
        assert n[k] @ (g.mean[k] - c) >= 0


def test_transmittance_at_points_equals_table_at_texel_centres_and_shells():
    g = tiny_scene(22, n=20, lo=-2, hi=2, median=0.2)
    light = np.array([0.05, -0.03, 0.02])
    H = W = 8
    K = 6
    T = od.build(light, g, H, W, K)
    t = od.shell_radii(K)
    d = od.texel_directions(H, W).reshape(-1, 3)
    for k in (0, 3, 5):
        pts = light + t[k] * d
        assert np.allclose(od.transmittance_at(light, g, pts), T[k].reshape(-1), rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------
# Footprint sampling (Sec. 3.3, Ablation A)
# ---------------------------------------------------------------------------

def _footprint_case(seed=21):
    rng = np.random.default_rng(seed)
    g = synth.random_gaussians(rng, rng.uniform(-1.5, 1.5, (300, 3)) + [0, 0, 2.0], 0.05)
    light = np.array([0.2, -0.1, 0.0])
    T = od.build(light, g, 16, 16, 8)
    return g, light, T


def test_footprint_single_centre_sample_is_the_point_query():
    g, light, T = _footprint_case()
    got = od.query_footprint(T, light, g, np.zeros((1, 3)), np.ones(1))
    assert np.array_equal(got, od.query(T, light, g.mean))


def test_footprint_of_a_constant_atlas_is_that_constant():
    g, light, _ = _footprint_case()
    z = np.random.default_rng(4).normal(size=(9, 3))
    got = od.query_footprint(np.full((8, 16, 16), 0.37), light, g, z, np.full(9, 1 / 9))
    assert np.allclose(got, 0.37, rtol=0, atol=1e-15)


def test_footprint_points_follow_the_principal_axes():
    """A sample at z = e_j lands one standard deviation along the j-th principal
    axis, mu + s_j R e_j (R e_j the j-th column of the rotation): compared with a
    point query there."""
    g, light, T = _footprint_case()
    R = od.quaternion_to_matrix(g.rot)
    for j in range(3):
        zj = np.zeros((1, 3))
        zj[0, j] = 1.0
        pts = g.mean + R[:, :, j] * g.scale[:, j:j + 1]
        assert np.allclose(od.query_footprint(T, light, g, zj, np.ones(1)), od.query(T, light, pts),
                           rtol=0, atol=1e-15)


def test_stencil7_weights_and_symmetry():
    z, w = od.footprint_stencil7()
    assert z.shape == (7, 3) and abs(w.sum() - 1) < 1e-15
    assert np.allclose(z.sum(axis=0), 0) and np.allclose((w[:, None] * z).sum(axis=0), 0)
    # Gaussian kernel ratio between an axis point and the centre
    assert abs(w[1] / w[0] - np.exp(-0.5)) < 1e-15 and np.allclose(w[1:], w[1])


def test_footprint_is_a_weighted_average_invariant_to_sample_order():
    g, light, T = _footprint_case()
    rng = np.random.default_rng(8)
    z = rng.normal(size=(6, 3))
    w = rng.uniform(0.1, 1, 6)
    w /= w.sum()
    a = od.query_footprint(T, light, g, z, w)
    perm = rng.permutation(6)
    b = od.query_footprint(T, light, g, z[perm], w[perm])
    assert np.allclose(a, b, rtol=0, atol=1e-15)
    lo = np.min([od.query_footprint(T, light, g, z[i:i + 1], [1.0]) for i in range(6)], axis=0)
    hi = np.max([od.query_footprint(T, light, g, z[i:i + 1], [1.0]) for i in range(6)], axis=0)
    assert np.all(a >= lo - 1e-15) and np.all(a <= hi + 1e-15)


# ---------------------------------------------------------------------------
# Receiver-driven region of interest (Sec. 3.2)
# ---------------------------------------------------------------------------

def test_roi_queries_at_receivers_equal_full_queries():
    """Every value a receiver's lookup reads lies in the region, so its query is
    the full atlas's query exactly (the point of marking the lookup's cell)."""
    g, light, T = _footprint_case(31)
    rng = np.random.default_rng(3)
    rec = rng.uniform(-1.5, 1.5, (200, 3)) + [0, 0, 2.0]
    Troi = od.build_roi(light, g, 16, 16, 8, rec)
    assert np.array_equal(od.query(Troi, light, rec), od.query(T, light, rec))
    assert np.any(Troi == 1.0) and np.any(Troi < 1.0)


def test_roi_without_receivers_is_transparent():
    g, light, _ = _footprint_case(31)
    assert np.all(od.build_roi(light, g, 16, 16, 8, np.zeros((0, 3))) == 1.0)


def test_roi_box_keeps_only_receivers_inside():
    g, light, _ = _footprint_case(31)
    rec = np.array([[0.5, 0.5, 1.5], [-1.0, -1.0, 2.5]])
    m1, k1a, k1b = od.roi_region(light, rec[:1], 16, 16, 8)
    mb, kba, kbb = od.roi_region(light, rec, 16, 16, 8, box=(0.5, 0.5, 0.2, 1.0, 2.0))
    assert np.array_equal(m1, mb) and (k1a, k1b) == (kba, kbb)
    assert m1.sum() <= 4 and k1b == k1a + 1


# ---------------------------------------------------------------------------
# Opacity to absorption mappings (ablation B)
# ---------------------------------------------------------------------------

def test_beta_constant_mapping_is_kappa_tau():
    rng = np.random.default_rng(2)
    g = synth.random_gaussians(rng, rng.uniform(-1, 1, (50, 3)), 0.05)
    A = od.precision_matrix(g.scale, g.rot)
    b = od.absorption_amplitude(g.opacity, A, kappa=0.7, beta="constant")
    assert np.allclose(b, -0.7 * np.log(1 - g.opacity.astype(np.float64)), rtol=1e-15, atol=0)


def test_beta_density_mapping_integrates_to_kappa_tau():
    """With the density mapping the absorption of one Gaussian integrates to
    kappa tau* over space (a Riemann sum over a box of +-7 sigma)."""
    g = synth.Gaussians(np.zeros((1, 3), np.float32), np.float32([[0.02, 0.05, 0.03]]),
                        np.float32([[0.9, 0.1, -0.3, 0.2]]) / np.float32(np.linalg.norm([0.9, 0.1, -0.3, 0.2])),
                        np.float32([0.6]))
    mean, A, beta = od.gaussian_terms(g, kappa=1.3, beta="density")
    n = 121
    ax = np.linspace(-0.35, 0.35, n)
    X = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    total = od.absorption(X, mean, A, beta).sum() * (ax[1] - ax[0]) ** 3
    assert abs(total - 1.3 * -np.log(1 - 0.6)) < 1e-6


def test_beta_trace_mapping_is_equation_5_for_isotropic():
    s = 0.04
    A = np.eye(3)[None] / s ** 2
    b = od.absorption_amplitude(np.array([0.5]), A, beta="trace")
    assert abs(b[0] - np.log(2) * (1 / s) / np.sqrt(2 * np.pi)) < 1e-12


# ---------------------------------------------------------------------------
# Approximate HDRI probe fit (Sec. 3.4)
# ---------------------------------------------------------------------------

def test_cubemap_solid_angles_cover_the_sphere():
    D, w = synth.cubemap_directions(16)
    assert D.shape == (6 * 256, 3) and np.allclose(np.linalg.norm(D, axis=1), 1.0, atol=1e-15)
    assert abs(w.sum() - 4 * np.pi) < 1e-12
    # face centres are the largest pixels, corners the smallest: ratio 3^(3/2) in the limit
    assert w.max() / w.min() > 4.0


def test_cubemap_quadrature_makes_the_sh_basis_orthonormal():
    D, w = synth.cubemap_directions(64)
    B = osh.real_sh(3, D)
    G = B.T @ (w[:, None] * B)
    assert np.abs(G - np.eye(16)).max() < 2e-3


@pytest.mark.parametrize("l_max", [2, 3])
def test_probe_fit_recovers_a_known_probe(l_max):
    rng = np.random.default_rng(13)
    K = (l_max + 1) ** 2
    A = rng.normal(size=(K, 3))
    D, w = synth.cubemap_directions(12)
    Y = osh.real_sh(l_max, D) @ A
    assert np.allclose(osh.probe_fit(Y, D, w, l_max, 0.0), A, rtol=0, atol=1e-10)


def test_probe_fit_ridge_limit():
    rng = np.random.default_rng(14)
    D, w = synth.cubemap_directions(8)
    Y = rng.uniform(0, 2, (D.shape[0], 3))
    lam = 1e9
    A = osh.probe_fit(Y, D, w, 3, lam)
    B = osh.real_sh(3, D)
    assert np.allclose(A * lam, B.T @ (w[:, None] * Y), rtol=1e-6, atol=0)


# ---------------------------------------------------------------------------
# Cube-map atlas (Ablation C)
# ---------------------------------------------------------------------------

def test_cube_texels_are_the_cube_map_render_directions():
    """The texel centres of the 2F x 3F cube-map atlas are, as a set, the pixel
    centres of a six-face 90-degree cube-map render (an independent generator
    with its own face bases)."""
    F = 6
    a = np.round(od.cube_texel_directions(2 * F, 3 * F).reshape(-1, 3), 12)
    b = np.round(synth.cubemap_directions(F)[0], 12)
    a = a[np.lexsort(a.T)]
    b = b[np.lexsort(b.T)]
    assert np.array_equal(a, b)


def test_cube_face_centres_are_the_signed_axes():
    for f in range(6):
        d = od.cube_decode(np.array([f]), np.array([0.0]), np.array([0.0]))[0]
        e = np.zeros(3)
        e[f // 2] = 1.0 if f % 2 == 0 else -1.0
        assert np.array_equal(d, e)
        assert od.cube_face(e.astype(np.float32)[None])[0] == f


def test_cube_encode_inverts_decode_at_texel_centres():
    F = 5
    H, W = 2 * F, 3 * F
    d = od.cube_texel_directions(H, W)
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    face = od.cube_face(d.astype(np.float32))
    assert np.array_equal(face, 3 * (i // F) + j // F)
    s, t = od.cube_encode(d, face)
    assert np.allclose(s, -1 + (2 * (j % F) + 1) / F, atol=1e-14)
    assert np.allclose(t, -1 + (2 * (i % F) + 1) / F, atol=1e-14)


def test_cube_query_reproduces_texel_values_at_centres_and_shells():
    K, F = 5, 4
    H, W = 2 * F, 3 * F
    table = _random_table(K, H, W)
    t = od.shell_radii(K, "geometric", 0.05, 8.0)
    d = od.texel_directions(H, W, "cubemap").reshape(-1, 3)
    light = np.array([0.25, -0.5, 0.125], np.float32)
    for k in range(K):
        pts = light + t[k] * d
        got = od.query(table, light, pts, param="cubemap")
        assert np.allclose(got, table[k].reshape(-1), atol=1e-6)


def test_cube_query_partition_of_unity_and_bounds():
    K, F = 6, 4
    rng = np.random.default_rng(16)
    pts = rng.uniform(-6, 6, (4000, 3))
    got = od.query(np.full((K, 2 * F, 3 * F), 0.37), np.zeros(3), pts, param="cubemap")
    assert np.allclose(got, 0.37, atol=1e-14)
    table = _random_table(K, 2 * F, 3 * F)
    got = od.query(table, np.zeros(3), pts, param="cubemap")
    assert np.all(got >= table.min() - 1e-12) and np.all(got <= table.max() + 1e-12)


def test_cube_query_interpolates_linearly_between_face_texel_centres():
    """A table affine in the in-face texel indices (a, b) is reproduced exactly
    between the first and last texel centres of every face."""
    K, F = 3, 6
    H, W = 2 * F, 3 * F
    i, j = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    face = 3 * (i // F) + j // F
    c = np.array([0.1, 0.2, 0.3, 0.4, 0.5, 0.6])
    table = np.broadcast_to(c[face] + 0.03 * (j % F) - 0.02 * (i % F), (K, H, W)).copy()
    rng = np.random.default_rng(17)
    n = 600
    f = rng.integers(0, 6, n)
    alpha = rng.uniform(0, F - 1, n)
    beta = rng.uniform(0, F - 1, n)
    # face coordinate of the continuous texel index x: the centre map s(x) = -1 + (2x + 1)/F
    d = od.cube_decode(f, -1 + (2 * alpha + 1) / F, -1 + (2 * beta + 1) / F)
    got = od.query(table, np.zeros(3), 2.0 * d, param="cubemap")
    assert np.allclose(got, c[f] + 0.03 * alpha - 0.02 * beta, atol=1e-6)


def test_cube_query_clamps_to_the_face_at_its_edges():
    """Beyond the outermost texel centres the lookup holds the edge texels of
    the face it is in: nothing is blended across the cube edges."""
    K, F = 2, 4
    table = _random_table(K, 2 * F, 3 * F)
    # +x face (block 0, 0): s = +1 at the face edge, t at the centre of in-face row 1
    t1 = -1 + 3 / F
    d = np.array([[1.0, 1.0 - 1e-6, t1]])
    got = od.query(table, np.zeros(3), 2.0 * d / np.linalg.norm(d), param="cubemap")
    tk = od.shell_radii(K)
    fk = (np.log(2.0 / tk[0]) / np.log(tk[1] / tk[0]))
    want = (1 - fk) * table[0, 1, F - 1] + fk * table[1, 1, F - 1]
    assert np.allclose(got, want, atol=1e-5)
    # on the cube edge x = y the tie goes to the first axis (+x face)
    e = np.array([[1.0, 1.0, t1]], np.float32)
    assert od.cube_face(e)[0] == 0 and od.cube_face(-e)[0] == 1


def test_cube_build_is_the_transmittance_at_texel_centres():
    g = tiny_scene(23, n=20, lo=-2, hi=2, median=0.2)
    light = np.array([0.05, -0.03, 0.02])
    F, K = 4, 6
    T = od.build(light, g, 2 * F, 3 * F, K, param="cubemap")
    t = od.shell_radii(K)
    d = od.cube_texel_directions(2 * F, 3 * F).reshape(-1, 3)
    for k in (0, 2, 5):
        assert np.allclose(od.transmittance_at(light, g, light + t[k] * d), T[k].reshape(-1), rtol=1e-12,
                           atol=1e-14)
    assert T.min() < 0.9


def test_cube_roi_queries_at_receivers_equal_full_queries():
    rng = np.random.default_rng(33)
    g = synth.random_gaussians(rng, rng.uniform(-1.5, 1.5, (200, 3)) + [0, 0, 2.0], 0.05)
    light = np.array([0.2, -0.1, 0.0], np.float32)
    F, K = 6, 8
    T = od.build(light, g, 2 * F, 3 * F, K, param="cubemap")
    rec = rng.uniform(-1.5, 1.5, (150, 3)) + [0, 0, 2.0]
    Troi = od.build_roi(light, g, 2 * F, 3 * F, K, rec, param="cubemap")
    assert np.array_equal(od.query(Troi, light, rec, param="cubemap"), od.query(T, light, rec, param="cubemap"))
    assert np.any(Troi == 1.0) and np.any(Troi < 1.0)


# ---------------------------------------------------------------------------
# Uniform radial bins (Sec. 3.2 "Directional parameterization": K uniform bins
# of [0, t_max] sampled at their centres t_k = (k + 1/2) t_max / K)
# ---------------------------------------------------------------------------

def test_uniform_build_samples_the_bin_centres():
    """Shell k of a uniform atlas holds the exact transmittance at the centre of
    radial bin k; a table sampled at the bin edges k t_max / K (the plausible
    slip) differs wherever T varies along the ray."""
    g = tiny_scene(31, n=30, lo=-2.2, hi=2.2, median=0.25)
    light = np.array([0.05, -0.03, 0.02])
    H, W, K, r1 = 8, 12, 7, 5.0
    T = od.build(light, g, H, W, K, spacing="uniform", r1=r1)
    d = od.texel_directions(H, W).reshape(-1, 3)
    varied = 0
    for k in range(K):
        centre = light + ((k + 0.5) * r1 / K) * d
        edge = light + (k * r1 / K + 1e-3) * d
        exact_c = od.transmittance_at(light, g, centre)
        assert np.allclose(T[k].reshape(-1), exact_c, rtol=1e-12, atol=1e-14)
        varied += np.abs(od.transmittance_at(light, g, edge) - exact_c).max() > 1e-3
    assert varied >= K - 1


def test_uniform_query_reads_bin_centres_and_interpolates_linearly_between_them():
    K, H, W, r1 = 6, 8, 8, 4.0
    table = _random_table(K, H, W, seed=41)
    light = np.array([0.2, 0.1, -0.3])
    d = od.texel_directions(H, W).reshape(-1, 3)
    for k in range(K):
        got = od.query(table, light, light + ((k + 0.5) * r1 / K) * d, spacing="uniform", r1=r1)
        assert np.allclose(got, table[k].reshape(-1), atol=1e-12)
    for k in range(K - 1):        # bin edge between two centres: the mean of the two shells
        got = od.query(table, light, light + ((k + 1) * r1 / K) * d, spacing="uniform", r1=r1)
        assert np.allclose(got, 0.5 * (table[k] + table[k + 1]).reshape(-1), atol=1e-12)
    # inside the first half bin and beyond the last centre: clamped to the end shells
    assert np.allclose(od.query(table, light, light + 0.2 * r1 / K * d, spacing="uniform", r1=r1),
                       table[0].reshape(-1), atol=1e-12)
    assert np.allclose(od.query(table, light, light + 1.3 * r1 * d, spacing="uniform", r1=r1),
                       table[K - 1].reshape(-1), atol=1e-12)


def test_geometric_query_is_linear_in_log_radius():
    """Between two geometric shells the lookup is linear in the fractional shell
    index, i.e. in log r: the geometric mean of two radii gives the mean value."""
    K, H, W = 5, 8, 8
    table = _random_table(K, H, W, seed=42)
    light = np.zeros(3)
    d = od.texel_directions(H, W).reshape(-1, 3)
    r = 0.05 * 160.0 ** (np.arange(K) / (K - 1))      # 0.05 .. 8 m
    for k in range(K - 1):
        got = od.query(table, light, math.sqrt(r[k] * r[k + 1]) * d)
        assert np.allclose(got, 0.5 * (table[k] + table[k + 1]).reshape(-1), atol=1e-12)


# ---------------------------------------------------------------------------
# The sampled-texel and point paths the full-size GPU checks use, against the
# full table on a small atlas that includes the folded (lower-hemisphere) texels
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("spacing", ["geometric", "uniform"])
@pytest.mark.parametrize("param,H,W", [("octahedral", 8, 12), ("octahedral", 10, 6), ("cubemap", 8, 12)])
def test_build_texels_equals_the_full_table(spacing, param, H, W):
    g = tiny_scene(43, n=40, lo=-2.0, hi=2.0, median=0.25)       # occluders in every direction
    light = np.array([0.1, 0.05, -0.07])
    K = 6
    T = od.build(light, g, H, W, K, spacing=spacing, r1=6.0, param=param)
    rows, cols = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    rows, cols = rows.ravel(), cols.ravel()
    got = od.build_texels(light, g, rows, cols, K, spacing=spacing, r1=6.0, H=H, W=W, param=param)
    assert got.shape == (H * W, K)
    assert np.allclose(got, T[:, rows, cols].T, rtol=1e-12, atol=1e-15)
    if param == "octahedral":
        u, v = od.texel_uv(H, W)
        assert (np.abs(u) + np.abs(v) > 1).sum() > 0.3 * H * W          # folded texels are covered
        assert T.min() < 0.5 and (T < 0.999).mean() > 0.2                # and the table is not flat


@pytest.mark.parametrize("spacing", ["geometric", "uniform"])
@pytest.mark.parametrize("param,H,W", [("octahedral", 8, 12), ("cubemap", 8, 12)])
def test_query_exact_equals_query_of_the_full_table(spacing, param, H, W):
    g = tiny_scene(44, n=40, lo=-2.0, hi=2.0, median=0.25)
    light = np.array([-0.1, 0.05, 0.08])
    K = 6
    rng = np.random.default_rng(45)
    pts = light + rng.normal(size=(400, 3)) * rng.uniform(0.05, 3.0, (400, 1))
    # points on the octahedral seams of the lower hemisphere (x = 0 or y = 0, z < 0)
    seam = rng.normal(size=(60, 3))
    seam[:30, 0] = 0.0
    seam[30:, 1] = 0.0
    seam[:, 2] = -np.abs(seam[:, 2])
    pts = np.concatenate([pts, light + seam])
    T = od.build(light, g, H, W, K, spacing=spacing, r1=6.0, param=param)
    ref = od.query(T, light, pts, spacing=spacing, r1=6.0, param=param)
    got = od.query_exact(light, g, pts, H, W, K, spacing=spacing, r1=6.0, param=param)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-14)
    assert ref.min() < 0.7


# ---------------------------------------------------------------------------
# Relighting outputs (Sec. 3.5, the relit colour) on a hand-computed case
# ---------------------------------------------------------------------------

def test_relight_hand_computed_constant_probe():
    """A probe with only the DC coefficient A_0c = 2 sqrt(pi) L_c radiates L_c in
    every direction (Y_00 = 1 / (2 sqrt(pi))); with eps = 0 the per-channel scale
    is s_c = clip(L_c, 0, t_max) whatever the normal.  L = (0.8, 2.5, 5.0),
    t_max = 4, gamma = 1.7:
      s      = (0.8, 2.5, 4.0)
      f'     = gamma s_c f            (every SH coefficient, no clamp)
      rgb'   = max(0, gamma (0.5 + f_0 / (2 sqrt(pi))) s_c)
    for f_0 = (-2, 0.3, 1):  f'_0 = (-2.72, 1.275, 6.8) and
      rgb' = (0,  1.7 * (0.5 + 0.3 * 0.28209479177387814) * 2.5,
                  1.7 * (0.5 + 0.28209479177387814) * 4)
           = (0, 2.4846708595116946, 5.318244584062371)."""
    L = np.array([0.8, 2.5, 5.0])
    probe = np.zeros((9, 3))
    probe[0] = 2.0 * math.sqrt(math.pi) * L
    rng = np.random.default_rng(46)
    g = synth.random_gaussians(rng, rng.normal(size=(4, 3)), 0.05)
    f = np.zeros((4, 16, 3))
    f[:, 0] = [-2.0, 0.3, 1.0]
    f[:, 5] = [1.0, -2.0, 3.0]
    s, f_out, rgb = osh.relight(probe, g, f, clip_max=4.0, eps=0.0, gamma=1.7)
    assert np.allclose(s, [0.8, 2.5, 4.0], rtol=0, atol=1e-12)
    assert np.allclose(f_out[:, 0], [-2.72, 1.275, 6.8], rtol=0, atol=1e-12)
    assert np.allclose(f_out[:, 5], [1.7 * 0.8, -1.7 * 5.0, 1.7 * 12.0], rtol=0, atol=1e-12)
    assert np.all(f_out[:, 1:5] == 0) and np.all(f_out[:, 6:] == 0)
    assert np.allclose(rgb, [0.0, 2.4846708595116946, 5.318244584062371], rtol=0, atol=1e-12)
