"""GPU: the receiver-driven region of interest (Sec. 3.2).

Inside the region the atlas is the full build (FP32 bar against the oracle),
outside it T = 1, and queries at the receivers equal queries of the full atlas.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import dgsm as od

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def roi_case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_01660_amd as P
    P.lib()
    c = synth.cfg1(n=3000)
    rng = np.random.default_rng(44)
    receivers = c["gaussians"].mean[rng.choice(c["gaussians"].n, 300, replace=False)]
    return c, receivers


@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_roi_queries_equal_full_build_queries(roi_case, dtype):
    import paper_2601_01660_amd as P
    c, rec = roi_case
    a = c["atlas"]
    atlas = P.Atlas.from_spec(a, dtype=dtype)
    lights = torch.from_numpy(c["lights"])
    gs = P.GaussianSet.from_host(c["gaussians"])
    full = P.dgsm_build(lights, gs, atlas)
    roi = P.dgsm_build_roi(lights, gs, atlas, torch.from_numpy(rec))
    qf = P.dgsm_query(lights, atlas, full, torch.from_numpy(rec))
    qr = P.dgsm_query(lights, atlas, roi, torch.from_numpy(rec))
    torch.cuda.synchronize()
    err = (qf - qr).abs().max().item()
    frac = (roi == 1).float().mean().item()
    print(f"[roi] {dtype}: receivers' queries roi vs full max|dT| {err:.3e}; T == 1 on {frac:.3f} of the atlas")
    assert err <= (1e-6 if dtype == "f32" else 1e-3)
    assert 0.2 < frac < 1.0


def test_roi_atlas_matches_oracle(roi_case):
    import paper_2601_01660_amd as P
    c, rec = roi_case
    a = c["atlas"]
    box = (2.5, 2.5, 1.2, 0.5, 3.0)
    atlas = P.Atlas.from_spec(a, dtype="f32")
    got = P.dgsm_build_roi(torch.from_numpy(c["lights"]), P.GaussianSet.from_host(c["gaussians"]), atlas,
                           torch.from_numpy(rec), box=box)[0].cpu().numpy().astype(np.float64)
    ref = od.build_roi(c["lights"][0], c["gaussians"], a.H, a.W, a.K, rec, box, a.spacing, a.r0, a.r1)
    mask, k_lo, k_hi = od.roi_region(c["lights"][0], rec, a.H, a.W, a.K, box, a.spacing, a.r0, a.r1)
    # the device picks the lookup cell in FP32: a receiver within rounding of a
    # texel or shell boundary may mark a neighbouring cell; such entries are few
    bad = np.abs(got - ref) > 1e-4
    print(f"[roi] region {mask.sum()} texels, shells [{k_lo}, {k_hi}]; entries off by > 1e-4: {bad.sum()}")
    assert mask.sum() > 0 and bad.sum() <= 2 * a.K
