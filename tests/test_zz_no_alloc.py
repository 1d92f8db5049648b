"""The allocation-free build entry point against dgsm_build, through the C ABI.

dgsm_build_noalloc runs dgsm_build's kernels on a fixed scratch array inside the
library; its atlas must equal dgsm_build's bit for bit (the build's sums are
fixed-point integer sums in a fixed order).  Two calls in a row, the second
with a smaller input, check that nothing the first call left in the shared
array is read; a request beyond the array's size is refused before any launch.
"""
import numpy as np
import pytest
import torch

import paper_2601_01660_amd as P
import synth

pytestmark = pytest.mark.gpu


def _case(n, H, W, K, n_lights, dtype):
    c = synth.cfg1(n)
    lights = np.asarray(c["lights"], np.float32)
    if n_lights > 1:
        lights = np.concatenate([lights, lights + np.float32([[0.3, -0.2, 0.4]])])[:n_lights]
    atlas = P.Atlas(H, W, K, dtype=dtype)
    return P.GaussianSet.from_host(c["gaussians"]), torch.from_numpy(np.ascontiguousarray(lights)), atlas


def _both(gs, lights, atlas):
    ref = P.dgsm_build(lights, gs, atlas)
    out = torch.full_like(ref, float("nan"))
    P.dgsm_build_noalloc(lights, gs, atlas, out)
    torch.cuda.synchronize()
    return ref, out


def test_noalloc_equals_build_on_two_calls_in_a_row():
    torch.cuda.set_device(0)
    big = _case(6000, 96, 96, 24, 2, "f32")
    small = _case(900, 48, 64, 16, 1, "f16")
    for gs, lights, atlas in (big, small):
        ws = P.dgsm_build_workspace_size(atlas, gs.n, int(lights.shape[0]))
        assert 0 < ws <= P.dgsm_build_noalloc_max_bytes()
        print(f"[noalloc] n={gs.n} lights={int(lights.shape[0])} {atlas.H}x{atlas.W}x{atlas.K} {atlas.dtype}",
              flush=True)
        ref, out = _both(gs, lights, atlas)
        assert torch.equal(ref, out), float((ref.float() - out.float()).abs().max())


def test_noalloc_refuses_requests_beyond_its_array():
    """A valid build whose workspace exceeds the array is refused, and nothing is
    written to the output."""
    torch.cuda.set_device(0)
    gs, lights, _ = _case(200_000, 32, 32, 16, 1, "f32")
    atlas = P.Atlas(256, 256, 64)
    assert P.dgsm_build_workspace_size(atlas, gs.n, 1) > P.dgsm_build_noalloc_max_bytes()
    out = torch.full((1, 64, 256, 256), float("nan"), device="cuda")
    with pytest.raises(P.DGSMError, match="status 2"):
        P.dgsm_build_noalloc(lights, gs, atlas, out)
    torch.cuda.synchronize()
    assert bool(torch.isnan(out).all())
