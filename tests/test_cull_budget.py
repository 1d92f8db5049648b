"""Culling error budget at the 2.15M-Gaussian workload (CPU only).

The build drops a (texel, Gaussian) pair only where the Gaussian's optical
depth along the texel ray from the light is at most cull_eps (the cone and
separating-plane tile tests bound it along the ray; the pre-test and the
prefactor test bound the whole-line depth, which is larger), and cuts each
evaluated erf ramp where the remaining step is below 1e-10 at either end
(Sec. 3.2 "Occluder culling via light-space footprints"; Eq. 3).  The optical
depth a build can lose at a texel is therefore at most the sum of the ray
depths of the Gaussians at or below cull_eps plus 2e-10 per evaluated
Gaussian.  This checks
that sum, per texel, against a 1e-5 budget (a tenth of the 1e-4 parity bar) on
texels of all four lights, half of them aimed at Gaussian centres.
"""
import numpy as np

import synth
from oracle import dgsm as od

CULL_EPS = 1e-8      # the build's default cull_eps in every workload
RAMP_EPS = 1e-10     # per ramp end


def _texels_towards(points, light, H, W):
    u, v = od.octahedral_encode(np.asarray(points, np.float64) - np.asarray(light, np.float64))
    return (np.clip(np.floor((v + 1) * H / 2).astype(int), 0, H - 1),
            np.clip(np.floor((u + 1) * W / 2).astype(int), 0, W - 1))


def test_ray_depth_of_an_isotropic_gaussian_ahead_of_and_behind_the_light():
    """Pin of the per-pair quantity: for an isotropic Gaussian of scale s whose
    centre lies on the texel ray at distance D ahead of the light, Eq. 5 gives
    beta = tau* / (s sqrt(2 pi)) and the depth along the ray is
    tau*/2 (1 + erf(D / (s sqrt 2))); centred D behind the light it is
    tau*/2 erfc(D / (s sqrt 2)) (the whole line would give tau* for both)."""
    from scipy.special import erf, erfc
    H = W = 16
    i, j = np.array([5]), np.array([11])
    d = od.texel_directions(H, W)[5, 11]
    light = np.array([0.3, -0.2, 0.7])
    s, D, alpha = 0.02, 0.06, 0.6
    tau = -np.log1p(-alpha)
    for sign, want in ((1.0, 0.5 * tau * (1 + erf(D / (s * np.sqrt(2))))),
                       (-1.0, 0.5 * tau * erfc(D / (s * np.sqrt(2))))):
        g = synth.Gaussians((light + sign * D * d)[None].astype(np.float32), np.full((1, 3), s, np.float32),
                            np.array([[1, 0, 0, 0]], np.float32), np.array([alpha], np.float32))
        mean32 = g.mean[0].astype(np.float64)
        off = np.linalg.norm(np.cross(mean32 - light, d))      # float32 rounding of the centre: off the ray
        want = want * np.exp(-0.5 * (off / s) ** 2)
        dropped, kept = od.dropped_depth_bound(light, g, i, j, H, W, eps=1.0)
        assert kept[0] == 0 and abs(dropped[0] - want) <= 1e-6 * want, (sign, dropped[0], want)
        dropped, kept = od.dropped_depth_bound(light, g, i, j, H, W, eps=0.5 * want)
        assert kept[0] == 1 and dropped[0] == 0.0


def test_dropped_optical_depth_stays_within_budget_at_the_full_workload():
    c = synth.cfg3(frames=1)
    g = synth.Gaussians.concat([c["scene"], c["avatar"].translated(c["trajectory"][0])])
    spec = c["atlas"]
    worst = 0.0
    for l, light in enumerate(c["lights"]):
        rng = np.random.default_rng(60 + l)
        i1, j1 = _texels_towards(g.mean[rng.choice(g.n, 8, replace=False)], light, spec.H, spec.W)
        i = np.concatenate([i1, rng.integers(0, spec.H, 8)])
        j = np.concatenate([j1, rng.integers(0, spec.W, 8)])
        dropped, kept = od.dropped_depth_bound(light, g, i, j, spec.H, spec.W, CULL_EPS)
        budget = dropped + 2 * RAMP_EPS * kept
        worst = max(worst, float(budget.max()))
        print(f"[cull] light {l}: dropped depth max {dropped.max():.2e} (mean {dropped.mean():.2e}), "
              f"evaluated Gaussians per texel max {kept.max()}, budget max {budget.max():.2e}", flush=True)
    assert worst <= 1e-5
