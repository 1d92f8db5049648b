"""Culling error budget at the 2.15M-Gaussian workload (CPU only).

The build drops a (texel, Gaussian) pair only where the Gaussian's whole-line
optical depth along the texel ray is at most cull_eps (the cone, pre-test and
prefactor tests are all bounds of that quantity), and cuts each evaluated erf
ramp where the remaining step is below 1e-10 at either end (Sec. 3.2 "Occluder
culling via light-space footprints"; Eq. 3).  The optical depth a build can
lose at a texel is therefore at most the sum of the whole-line depths of the
Gaussians at or below cull_eps plus 2e-10 per evaluated Gaussian.  This checks
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
