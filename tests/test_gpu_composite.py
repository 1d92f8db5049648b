"""GPU: the full composite workload at its real size -- a 6M-Gaussian room, 8
avatars x 200k Gaussians on their own seeded walks, 8 lights, 1024 x 1024 x 128
geometric shells -- against the FP64 oracle on sampled texels and centres.

FP32 build of frame 0 on a workspace sized for the set's list entries: sampled
texels within 1e-4 of the oracle.  FP16 batched plan (static cache, one rigid
group per avatar): frame 2 at sampled centres within 1e-2 of the oracle's query
from exactly computed texel columns."""
import numpy as np
import pytest
import torch

import synth
from oracle import dgsm as od

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def comp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_01660_amd as P
    P.lib()
    c = synth.cfg5(frames=3)
    c["tr"] = np.stack(c["trajectories"], axis=1).astype(np.float32)     # [F][avatars][3]
    c["dyn"] = synth.Gaussians.concat(c["avatars"])
    c["starts"] = np.cumsum([0] + [a.n for a in c["avatars"]])
    return c


def _frame(c, f):
    return synth.Gaussians.concat([c["scene"]] + [a.translated(c["tr"][f, i]) for i, a in enumerate(c["avatars"])])


def _texels_towards(points, light, H, W):
    u, v = od.octahedral_encode(np.asarray(points, np.float64) - np.asarray(light, np.float64))
    return (np.clip(np.floor((v + 1) * H / 2).astype(int), 0, H - 1),
            np.clip(np.floor((u + 1) * W / 2).astype(int), 0, W - 1))


def test_composite_fp32_build_sampled_texels(comp):
    import paper_2601_01660_amd as P
    spec = comp["atlas"]
    g = _frame(comp, 0)
    gs = P.GaussianSet.from_host(g)
    lights = torch.from_numpy(comp["lights"]).cuda()
    atlas = P.Atlas.from_spec(spec, dtype="f32", cull_eps=1e-8)
    L = lights.shape[0]
    entries = P.dgsm_count_entries(lights, gs, atlas)
    ws = torch.empty(P.dgsm_build_workspace_size_entries(atlas, g.n, L, entries), dtype=torch.uint8, device="cuda")
    T = P.dgsm_build(lights, gs, atlas, workspace=ws)
    torch.cuda.synchronize()
    for l in range(L):
        need, cap = P.dgsm_list_entries(atlas, g.n, L, ws, l)
        assert need <= cap
    del ws
    rng = np.random.default_rng(91)
    worst = 0.0
    for l in range(L):
        light = comp["lights"][l]
        # one texel towards an avatar centre, one towards a room centre, one at random
        ia, ja = _texels_towards(g.mean[[comp["scene"].n + rng.integers(comp["dyn"].n)]], light, spec.H, spec.W)
        ir, jr = _texels_towards(g.mean[[rng.integers(comp["scene"].n)]], light, spec.H, spec.W)
        i = np.concatenate([ia, ir, rng.integers(0, spec.H, 1)])
        j = np.concatenate([ja, jr, rng.integers(0, spec.W, 1)])
        ref = od.build_texels(light, g, i, j, spec.K, spec.spacing, spec.r0, spec.r1, H=spec.H, W=spec.W)
        got = T[l][:, torch.from_numpy(i).cuda(), torch.from_numpy(j).cuda()].T.cpu().numpy()
        err = np.abs(got - ref).max()
        worst = max(worst, err)
        print(f"[composite] fp32 light {l} texels {list(zip(i.tolist(), j.tolist()))}: max|dT| {err:.2e} "
              f"(T from {ref.min():.3f} to {ref.max():.3f})", flush=True)
        assert err <= 1e-4
    print(f"[composite] fp32 sampled texels over {L} lights: max|dT| {worst:.2e}", flush=True)


def test_composite_batched_plan_sampled_centres(comp):
    import paper_2601_01660_amd as P
    spec = comp["atlas"]
    lights = torch.from_numpy(comp["lights"]).cuda()
    atlas = P.Atlas.from_spec(spec, dtype="f16", cull_eps=1e-8)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        plan = P.Plan(lights, atlas, P.GaussianSet.from_host(comp["scene"]), comp["dyn"].n, 3, static_cache=True,
                      autotune=False, tile_waves=8, split_units=131072, chains=1, group_start=comp["starts"])
        out = plan.run(P.GaussianSet.from_host(comp["dyn"]), torch.from_numpy(comp["tr"]).cuda(), use_graph=True)
        side.synchronize()
        f = 2
        rng = np.random.default_rng(92)
        g = _frame(comp, f)
        ns = comp["scene"].n
        for l in (0, 5):
            light = comp["lights"][l]
            near = np.argsort(np.linalg.norm(g.mean[:ns] - light, axis=1))[:200:40]
            idx = np.concatenate([near, ns + rng.choice(comp["dyn"].n, 4, replace=False)])
            got = out[f, l, torch.from_numpy(idx).cuda()].cpu().numpy()
            ref = od.query_exact(light, g, g.mean[idx], spec.H, spec.W, spec.K, spec.spacing, spec.r0, spec.r1)
            err = np.abs(got - ref).max()
            print(f"[composite] plan frame {f} light {l}: max|dT| {err:.2e} over {len(idx)} centres "
                  f"(T from {ref.min():.3f} to {ref.max():.3f})", flush=True)
            assert err <= 1e-2
        plan.close()
