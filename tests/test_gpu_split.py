"""GPU: tiles cut into work units.

A dense cluster seen from the light lands in a handful of atlas tiles with
thousands of Gaussian hits each; the accumulation cuts such tiles into slices
run by separate workgroups.  The fixed-point sums are integers, so the atlas
must be bitwise the same as with unsplit tiles, and within the FP32 bar of the
FP64 oracle.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import dgsm as od

pytestmark = pytest.mark.gpu

H, W, K = 48, 48, 16


@pytest.fixture(scope="module")
def cluster():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_01660_amd as P
    P.lib()
    rng = np.random.default_rng(91)
    dense = synth.random_gaussians(rng, rng.uniform(-0.15, 0.15, (12000, 3)) + [1.1, 0.5, 0.3], 0.01)
    bg = synth.random_gaussians(rng, rng.uniform(-2.5, 2.5, (1500, 3)) * [1, 1, 0.3] + [0, 0, -0.5], 0.05)
    light = np.array([[0.1, -0.2, 1.6]], np.float32)
    traj = synth.random_walk(rng, 3, step=0.05, start=(0.0, 0.0))
    return dict(dense=dense, bg=bg, light=light, traj=traj)


def test_split_tiles_match_oracle(cluster):
    import paper_2601_01660_amd as P
    g = synth.Gaussians.concat([cluster["bg"], cluster["dense"]])
    lights = torch.from_numpy(cluster["light"]).cuda()
    atlas = P.Atlas(H, W, K, dtype="f32")
    gs = P.GaussianSet.from_host(g)
    ws = torch.empty(P.dgsm_build_workspace_size(atlas, g.n, 1), dtype=torch.uint8, device="cuda")
    T = torch.empty((1, K, H, W), dtype=torch.float32, device="cuda")
    P.dgsm_bin(lights, gs, atlas, ws)
    P.dgsm_accumulate(lights, atlas, g.n, T, ws)
    extra, nsplit, per, total = P.dgsm_work_units(atlas, g.n, 1, ws, 0)
    print(f"[split] extra slices {extra}, split tiles {nsplit}, hits/slice {per}, total hits {total}")
    assert nsplit >= 1 and extra >= nsplit and per > 0
    # texels aimed at the cluster (the split tiles) and a few uniform ones
    rng = np.random.default_rng(5)
    import gpu_util
    idx = rng.choice(cluster["dense"].n, 40, replace=False)
    i1, j1 = gpu_util.texels_towards(cluster["dense"].mean[idx], cluster["light"][0], H, W)
    i = np.concatenate([i1, rng.integers(0, H, 8)])
    j = np.concatenate([j1, rng.integers(0, W, 8)])
    ref = od.build_texels(cluster["light"][0], g, i, j, K, H=H, W=W)
    got = T[0].cpu().numpy()[:, i, j].T.astype(np.float64)
    err = np.abs(got - ref).max()
    print(f"[split] vs oracle at {len(i)} texels: max|dT| {err:.3e} (min T {ref.min():.3f})")
    assert ref.min() < 0.5           # the sampled rays do cross the cluster
    assert err <= 1e-4


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("cache", [True, False])
def test_split_is_bitwise_unsplit(cluster, dtype, cache):
    import paper_2601_01660_amd as P
    atlas = P.Atlas(H, W, K, dtype=dtype)
    lights = torch.from_numpy(cluster["light"]).cuda()
    static = P.GaussianSet.from_host(cluster["bg"])
    dyn = P.GaussianSet.from_host(cluster["dense"])
    tr = torch.from_numpy(cluster["traj"]).cuda()
    outs = []
    for units in (-1, 100000):
        plan = P.Plan(lights, atlas, static, cluster["dense"].n, cluster["traj"].shape[0], static_cache=cache,
                      autotune=False, tile_waves=4, split_units=units)
        assert plan.split_units == units
        outs.append(plan.run(dyn, tr, use_graph=False))
        torch.cuda.synchronize()
        plan.close()
    assert outs[0].min().item() < 0.5
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("spacing", ["geometric", "uniform"])
def test_packed_walk_is_bitwise_the_tile_walk(cluster, dtype, spacing):
    """The packed walk (only pairs past the distance pre-test, 64 per wave)
    adds exactly the increments of the tile walk: the atlas is bitwise the same
    for every number of waves per tile, with and without split tiles."""
    import paper_2601_01660_amd as P
    g = synth.Gaussians.concat([cluster["bg"], cluster["dense"]])
    lights = torch.from_numpy(np.array([[0.1, -0.2, 1.6], [-1.0, 0.7, 1.2]], np.float32)).cuda()
    atlas = P.Atlas(H, W, K, spacing=spacing, dtype=dtype)
    gs = P.GaussianSet.from_host(g)
    ws = torch.empty(P.dgsm_build_workspace_size(atlas, g.n, 2), dtype=torch.uint8, device="cuda")
    P.dgsm_bin(lights, gs, atlas, ws)
    ref = P.dgsm_accumulate(lights, atlas, g.n, torch.empty((2, K, H, W), dtype=atlas.torch_dtype,
                                                          device="cuda"), ws)
    for nw in (2, 4, 8):
        for units in (-1, 0, 2000):
            for packed in (False, True):
                out = torch.empty_like(ref)
                P.dgsm_accumulate_ex(lights, atlas, g.n, out, ws, tile_waves=nw, split_units=units, packed=packed)
                torch.cuda.synchronize()
                assert torch.equal(out, ref), (nw, units, packed)
    assert ref.min().item() < 0.5
    print(f"[split] packed walk bitwise equal to the tile walk ({spacing}, {dtype})", flush=True)


@pytest.mark.parametrize("cache", [True, False])
def test_plan_packed_walk_is_bitwise_unpacked(cluster, cache):
    import paper_2601_01660_amd as P
    atlas = P.Atlas(H, W, K, dtype="f16")
    lights = torch.from_numpy(cluster["light"]).cuda()
    static = P.GaussianSet.from_host(cluster["bg"])
    dyn = P.GaussianSet.from_host(cluster["dense"])
    tr = torch.from_numpy(cluster["traj"]).cuda()
    outs = []
    for packed in (False, True):
        plan = P.Plan(lights, atlas, static, cluster["dense"].n, cluster["traj"].shape[0], static_cache=cache,
                      autotune=False, tile_waves=8, packed=packed)
        assert plan.packed == (packed and cache)
        outs.append(plan.run(dyn, tr, use_graph=False).clone())
        torch.cuda.synchronize()
        plan.close()
    assert torch.equal(outs[0], outs[1])
