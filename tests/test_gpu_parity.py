"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: FP32 transmittance within 1e-4 absolute of the oracle (table and
queries); FP16 storage within 1e-2; SH transfer within 1e-4 relative.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import dgsm as od
from oracle import sh as osh

pytestmark = pytest.mark.gpu

TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_01660_amd as P
    P.lib()   # raises if the HIP library is missing


def _util():
    import gpu_util
    return gpu_util


def _report(name, err):
    print(f"[parity] {name}: max|dT| = {err:.3e}", flush=True)


# ---------------------------------------------------------------------------
# Plain build + query at the 5k-Gaussian workload (32 x 32 x 16)
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cfg1():
    c = synth.cfg1()
    a = c["atlas"]
    c["oracle_T"] = od.build(c["lights"][0], c["gaussians"], a.H, a.W, a.K, a.spacing, a.r0, a.r1)
    return c


def test_cfg1_build_matches_oracle(cfg1):
    U = _util()
    T, _ = U.gpu_build(cfg1["gaussians"], cfg1["lights"], cfg1["atlas"])
    got = T[0].cpu().numpy().astype(np.float64)
    err = np.abs(got - cfg1["oracle_T"]).max()
    _report("cfg1 build", err)
    assert err <= TOL


def test_cfg1_query_matches_oracle(cfg1):
    U = _util()
    T, atlas = U.gpu_build(cfg1["gaussians"], cfg1["lights"], cfg1["atlas"])
    got = U.gpu_query(cfg1["lights"], atlas, T, cfg1["points"])[0]
    ref = od.query(cfg1["oracle_T"], cfg1["lights"][0], cfg1["points"])
    err = np.abs(got - ref).max()
    _report("cfg1 query", err)
    assert err <= TOL
    # the query kernel alone: FP64 trilinear of the GPU's own table
    own = od.query(T[0].cpu().numpy().astype(np.float64), cfg1["lights"][0], cfg1["points"])
    assert np.abs(got - own).max() <= 2e-5


@pytest.mark.parametrize("spacing", ["geometric", "uniform"])
def test_octahedral_query_edge_cases_on_a_random_table(spacing):
    """Random table (an input, not a build) on a non-square atlas: points on the
    fold seams (x = 0 or y = 0 below the light), straight below it (the corner
    of the map), on the horizon plane z = 0 (the inner diamond), on the inner
    coordinate planes, beside the outer edges (wrapped neighbours), at the
    light (r = 0), inside r0 and beyond r1; FP32 lookup against the FP64 oracle."""
    U = _util()
    import paper_2601_01660_amd as P
    H, W, K = 24, 40, 12
    r0, r1 = 0.05, 8.0
    rng = np.random.default_rng(17)
    light = np.array([[0.25, -0.5, 1.0]], np.float32)          # exact in FP32
    table = rng.uniform(0, 1, (1, K, H, W)).astype(np.float32)
    n = 400
    rad = rng.uniform(0.02, 12.0, (n, 1))
    a, b = rng.uniform(-1, 1, (n, 1)), rng.uniform(-1, 1, (n, 1))
    down = -np.abs(rng.uniform(0.05, 1, (n, 1)))
    offs = {
        "random": rng.normal(size=(n, 3)) * rad,
        "seam x=0, z<0": np.hstack([0 * a, a, down]) * rad,
        "seam y=0, z<0": np.hstack([a, 0 * a, down]) * rad,
        "straight below": np.hstack([0 * a, 0 * a, down]) * rad,
        "horizon z=0": np.hstack([a, b, 0 * a]) * rad,
        "plane x=0, z>0": np.hstack([0 * a, a, -down]) * rad,
        "plane y=0, z>0": np.hstack([a, 0 * a, -down]) * rad,
        "near outer edge": np.hstack([np.sign(a) * (1 - 1e-3 * np.abs(b)), 1e-3 * b, -np.ones_like(a)]) * rad,
        "at the light": np.zeros((4, 3)),
        "inside r0": rng.normal(size=(n, 3)) * 0.01,
        "beyond r1": rng.normal(size=(n, 3)) * 40.0,
    }
    atlas = P.Atlas(H, W, K, spacing=spacing, r0=r0, r1=r1)
    Tt = torch.from_numpy(table).cuda()
    worst = 0.0
    for name, o in offs.items():
        pts = (light[0] + o.astype(np.float32)).astype(np.float32)
        got = U.gpu_query(light, atlas, Tt, pts)[0]
        ref = od.query(table[0].astype(np.float64), light[0].astype(np.float64), pts.astype(np.float64),
                       spacing, r0, r1)
        err = np.abs(got - ref).max()
        worst = max(worst, err)
        print(f"[parity] octahedral query {spacing} {name}: max|dT| = {err:.2e}", flush=True)
        assert err <= 2e-5, name
    _report(f"octahedral query edge cases, {spacing}", worst)


def test_cfg1_denser_ragged_two_lights():
    """The 5k scene at 36 x 36 (ragged 8x8 tiles) x 24 shells, two lights, one inside the cloud."""
    U = _util()
    c = synth.cfg1()
    g = c["gaussians"]
    lights = np.array([[0.0, 0.0, 0.0], [2.5, 2.5, 2.5]], np.float32)
    spec = synth.AtlasSpec(36, 36, 24)
    T, atlas = U.gpu_build(g, lights, spec)
    got = T.cpu().numpy().astype(np.float64)
    for l in range(2):
        ref = od.build(lights[l], g, spec.H, spec.W, spec.K)
        err = np.abs(got[l] - ref).max()
        _report(f"36x36x24 light {l}", err)
        assert err <= TOL
        pts = g.mean[::7]
        q = U.gpu_query(lights, atlas, T, pts)[l]
        assert np.abs(q - od.query(ref, lights[l], pts)).max() <= TOL


def test_partial_supertiles_and_tile_order_tail():
    """80 x 76 texels: 10 x 10 tiles in four supertiles, three of them partial;
    100 tile blocks, so the XCD-aware tile order covers whole groups of 64 and
    a tail.  Every texel and shell against the oracle."""
    U = _util()
    c = synth.cfg1()
    g = c["gaussians"]
    lights = np.array([[0.3, -0.2, 0.4]], np.float32)
    spec = synth.AtlasSpec(76, 80, 8)
    T, atlas = U.gpu_build(g, lights, spec)
    ref = od.build(lights[0], g, spec.H, spec.W, spec.K)
    err = np.abs(T[0].cpu().numpy().astype(np.float64) - ref).max()
    _report("76x80x8 partial supertiles", err)
    assert ref.min() < 0.5 and err <= TOL


def test_uniform_shells_and_kappa():
    U = _util()
    c = synth.cfg1(1500)
    g = c["gaussians"]
    spec = synth.AtlasSpec(16, 24, 10, spacing="uniform", r0=0.05, r1=8.0)
    T, atlas = U.gpu_build(g, c["lights"], spec, kappa=1.7)
    ref = od.build(c["lights"][0], g, spec.H, spec.W, spec.K, "uniform", spec.r0, spec.r1, kappa=1.7)
    err = np.abs(T[0].cpu().numpy() - ref).max()
    _report("uniform shells kappa 1.7", err)
    assert err <= TOL
    q = U.gpu_query(c["lights"], atlas, T, g.mean)[0]
    assert np.abs(q - od.query(ref, c["lights"][0], g.mean, "uniform", spec.r0, spec.r1)).max() <= TOL


def test_light_inside_gaussians_and_large_scales():
    """Gaussians that contain the light (global culling cones) and wide ramps."""
    U = _util()
    rng = np.random.default_rng(5)
    g = synth.random_gaussians(rng, rng.uniform(-0.6, 0.6, (300, 3)), 0.25)
    lights = np.array([[0.01, -0.02, 0.03]], np.float32)
    spec = synth.AtlasSpec(24, 24, 20, r0=0.02, r1=3.0)
    T, _ = U.gpu_build(g, lights, spec)
    ref = od.build(lights[0], g, spec.H, spec.W, spec.K, spec.spacing, spec.r0, spec.r1)
    err = np.abs(T[0].cpu().numpy() - ref).max()
    _report("light inside", err)
    assert err <= TOL


# ---------------------------------------------------------------------------
# Special cases and invariants on the GPU
# ---------------------------------------------------------------------------

def test_empty_and_transparent_scene():
    U = _util()
    spec = synth.AtlasSpec(16, 16, 8)
    lights = np.zeros((1, 3), np.float32)
    T, atlas = U.gpu_build(synth.Gaussians.empty(), lights, spec)
    assert torch.all(T == 1.0)
    g = synth.cfg1(200)["gaussians"]
    g.opacity[:] = 0.0
    T, _ = U.gpu_build(g, lights, spec)
    assert torch.all(T == 1.0)
    q = U.gpu_query(lights, atlas, T, np.random.default_rng(1).uniform(-5, 5, (1000, 3)))
    assert np.all(q == 1.0)


def test_build_does_not_depend_on_gaussian_order():
    """tau is a sum over Gaussians (Eq. 2) accumulated in fixed point, and
    every culling decision is taken per Gaussian: the atlas of a 400k-Gaussian
    room under 4 lights is bitwise the same for the caller's order, a random
    permutation and a spatially sorted order (the binning waves then hold
    different mixes of entries)."""
    U = _util()
    rng = np.random.default_rng(2024)
    g = synth.random_gaussians(rng, synth.room_centres(rng, 400_000), 0.03)
    lights = synth.CFG3_LIGHTS
    spec = synth.AtlasSpec(256, 256, 32)
    T0, _ = U.gpu_build(g, lights, spec, dtype="f16")
    perm = rng.permutation(g.n)
    zyx = np.lexsort((g.mean[:, 0], g.mean[:, 1], np.floor(g.mean[:, 2] * 4)))
    for order in (perm, zyx):
        T1, _ = U.gpu_build(g.subset(order), lights, spec, dtype="f16")
        assert torch.equal(T0, T1)
    assert T0.float().min().item() < 0.5


def test_binding_rejects_buffers_of_the_wrong_shape(cfg1):
    """Outputs, tables, points and translations reach the library as raw
    pointers: a tensor of the wrong shape or dtype is refused before any launch."""
    import paper_2601_01660_amd as P
    g, lights = cfg1["gaussians"], cfg1["lights"]
    atlas = P.Atlas(32, 32, 16, dtype="f32")
    gs = P.GaussianSet.from_host(g)
    lt = torch.from_numpy(np.ascontiguousarray(lights, dtype=np.float32)).cuda()
    L = lt.shape[0]
    T = P.dgsm_build(lt, gs, atlas)
    with pytest.raises(ValueError):
        P.dgsm_build(lt, gs, atlas, out=torch.empty((L, 16, 32, 16), device="cuda"))
    with pytest.raises(ValueError):
        P.dgsm_build(lt, gs, atlas, out=torch.empty((L, 16, 32, 32), dtype=torch.float16, device="cuda"))
    pts = torch.zeros((10, 3), device="cuda")
    with pytest.raises(ValueError):
        P.dgsm_query(lt, atlas, T, pts, out=torch.empty((L, 5), device="cuda"))
    with pytest.raises(ValueError):
        P.dgsm_query(lt, atlas, T[:, :8].contiguous(), pts)
    with pytest.raises(ValueError):
        P.dgsm_query(lt, atlas, T, torch.zeros((10, 4), device="cuda"))
    plan = P.Plan(lt, atlas, gs, 0, 3, static_cache=True, autotune=False)
    empty = P.GaussianSet.from_host(synth.Gaussians.empty())
    with pytest.raises(ValueError):
        plan.run(empty, torch.zeros((2, 3), device="cuda"))
    with pytest.raises(ValueError):
        plan.run(empty, torch.zeros((3, 3), device="cuda"), out=torch.empty((3, L, 7), device="cuda"))
    out = plan.run(empty, torch.zeros((3, 3), device="cuda"), use_graph=False)
    torch.cuda.synchronize()
    assert out.shape == (3, L, g.n)
    plan.close()
    # no dynamic Gaussians: every frame is the static set's own query (the
    # frame query copies the once-per-run static results, no tile reached)
    ref = P.dgsm_query(lt, atlas, T, gs.mean).cpu()
    for f in range(3):
        assert (out[f].cpu() - ref).abs().max().item() <= 2e-6
    # no static Gaussians: every frame is the dynamic set's own build and query
    plan = P.Plan(lt, atlas, empty, g.n, 2, static_cache=True, autotune=False)
    out = plan.run(gs, torch.zeros((2, 3), device="cuda"), use_graph=False)
    torch.cuda.synchronize()
    assert out.shape == (2, L, g.n)
    for f in range(2):
        assert (out[f].cpu() - ref).abs().max().item() <= 2e-6
    plan.close()


def test_monotone_bounded_and_deterministic(cfg1):
    U = _util()
    spec = synth.AtlasSpec(64, 64, 32)
    T1, _ = U.gpu_build(cfg1["gaussians"], cfg1["lights"], spec)
    T2, _ = U.gpu_build(cfg1["gaussians"], cfg1["lights"], spec)
    assert torch.equal(T1, T2)
    assert torch.all(T1[:, 1:] <= T1[:, :-1])
    assert torch.all((T1 >= 0) & (T1 <= 1))


def test_culling_matches_unculled(cfg1):
    U = _util()
    spec = synth.AtlasSpec(64, 64, 16)
    Tc, _ = U.gpu_build(cfg1["gaussians"], cfg1["lights"], spec, cull_eps=1e-8)
    Tn, _ = U.gpu_build(cfg1["gaussians"], cfg1["lights"], spec, cull_eps=0.0)
    err = (Tc - Tn).abs().max().item()
    _report("culled vs unculled", err)
    assert err <= 1e-6


def test_culling_matches_unculled_around_the_light():
    """Anisotropic Gaussians on every side of a light, some within a few
    centimetres of it (the tile tests' separating plane and cone face Gaussians
    ahead of, beside and behind the light): culled vs unculled within the
    culling budget of 1e-5, on a 64x64 atlas (8x8-texel tiles of about 0.1 rad)
    and a 256x256 one (0.025 rad)."""
    U = _util()
    rng = np.random.default_rng(321)
    light = np.array([[0.2, -0.1, 1.3]], np.float32)
    far = rng.uniform(-3, 3, (15000, 3)) + light[0]
    near = rng.normal(0, 0.15, (500, 3)) + light[0]
    g = synth.random_gaussians(rng, np.concatenate([far, near]).astype(np.float32), 0.03)
    for spec in (synth.AtlasSpec(64, 64, 16), synth.AtlasSpec(256, 256, 16)):
        Tc, _ = U.gpu_build(g, light, spec, cull_eps=1e-8)
        Tn, _ = U.gpu_build(g, light, spec, cull_eps=0.0)
        err = (Tc - Tn).abs().max().item()
        _report(f"culled vs unculled around the light {spec.H}x{spec.W}", err)
        assert Tn.min().item() < 0.5
        assert err <= 1e-5


def test_additivity_on_gpu(cfg1):
    U = _util()
    g = cfg1["gaussians"]
    spec = synth.AtlasSpec(32, 32, 16)
    T, _ = U.gpu_build(g, cfg1["lights"], spec)
    T1, _ = U.gpu_build(g.subset(np.arange(0, 2000)), cfg1["lights"], spec)
    T2, _ = U.gpu_build(g.subset(np.arange(2000, g.n)), cfg1["lights"], spec)
    assert (T - T1 * T2).abs().max().item() <= 1e-5


def test_fp16_storage_within_bar(cfg1):
    U = _util()
    spec = synth.AtlasSpec(64, 64, 16)
    T32, a32 = U.gpu_build(cfg1["gaussians"], cfg1["lights"], spec, dtype="f32")
    T16, a16 = U.gpu_build(cfg1["gaussians"], cfg1["lights"], spec, dtype="f16")
    assert T16.dtype == torch.float16
    assert (T16.float() - T32).abs().max().item() <= 1e-2
    assert torch.equal(T16, T32.half())       # RNE of the FP32 value
    q32 = U.gpu_query(cfg1["lights"], a32, T32, cfg1["points"])
    q16 = U.gpu_query(cfg1["lights"], a16, T16, cfg1["points"])
    assert np.abs(q32 - q16).max() <= 1e-2


def test_minimal_atlas():
    U = _util()
    c = synth.cfg1(300)
    spec = synth.AtlasSpec(2, 2, 2)
    T, atlas = U.gpu_build(c["gaussians"], c["lights"], spec)
    ref = od.build(c["lights"][0], c["gaussians"], 2, 2, 2)
    assert np.abs(T[0].cpu().numpy() - ref).max() <= TOL
    q = U.gpu_query(c["lights"], atlas, T, c["points"])[0]
    assert np.abs(q - od.query(ref, c["lights"][0], c["points"])).max() <= TOL


# ---------------------------------------------------------------------------
# Full-size workloads, sampled against the oracle
# ---------------------------------------------------------------------------

def test_cfg2_full_size_sampled():
    U = _util()
    c = synth.cfg2()
    g, spec, light = c["gaussians"], c["atlas"], c["lights"][0]
    T, atlas = U.gpu_build(g, c["lights"], spec)
    i, j = U.sample_texels(g, light, spec.H, spec.W, 64, seed=21)
    ref = od.build_texels(light, g, i, j, spec.K, spec.spacing, spec.r0, spec.r1, H=spec.H, W=spec.W)
    got = T[0].cpu().numpy()[:, i, j].T
    err = np.abs(got - ref).max()
    _report("cfg2 sampled texels", err)
    assert err <= TOL
    pts = g.mean[np.random.default_rng(22).choice(g.n, 12, replace=False)]
    q = U.gpu_query(c["lights"], atlas, T, pts)[0]
    qref = od.query_exact(light, g, pts, spec.H, spec.W, spec.K, spec.spacing, spec.r0, spec.r1)
    err = np.abs(q - qref).max()
    _report("cfg2 sampled queries", err)
    assert err <= TOL
    # the query kernel at every Gaussian centre: FP64 trilinear of the GPU's own table
    qall = U.gpu_query(c["lights"], atlas, T, g.mean)[0]
    own = od.query(T[0].cpu().numpy().astype(np.float64), light, g.mean, spec.spacing, spec.r0, spec.r1)
    err = np.abs(qall - own).max()
    _report(f"cfg2 query of all {g.n} centres vs FP64 trilinear of the GPU table", err)
    assert err <= 2e-5


@pytest.mark.parametrize("dtype,tol", [("f32", TOL), ("f16", 1e-2)])
def test_cfg3_frame0_full_size_sampled(dtype, tol):
    """2M scene + 150k avatar Gaussians, 4 lights, 512 x 512 x 64 (the timed workload)."""
    U = _util()
    c = synth.cfg3(frames=1)
    g = synth.Gaussians.concat([c["scene"], c["avatar"]])
    spec = c["atlas"]
    T, atlas = U.gpu_build(g, c["lights"], spec, dtype=dtype)
    host = T.float().cpu().numpy()
    for l in range(4):
        light = c["lights"][l]
        i, j = U.sample_texels(g, light, spec.H, spec.W, 16, seed=30 + l)
        ref = od.build_texels(light, g, i, j, spec.K, spec.spacing, spec.r0, spec.r1, H=spec.H, W=spec.W)
        err = np.abs(host[l][:, i, j].T - ref).max()
        _report(f"cfg3 {dtype} light {l} sampled texels", err)
        assert err <= tol
    # the query kernel at all 2.15M centres and 4 lights: FP64 trilinear of the GPU's own table
    qall = U.gpu_query(c["lights"], atlas, T, g.mean)
    for l in range(4):
        own = od.query(host[l].astype(np.float64), c["lights"][l], g.mean, spec.spacing, spec.r0, spec.r1)
        err = np.abs(qall[l] - own).max()
        _report(f"cfg3 {dtype} light {l} query of all {g.n} centres vs FP64 trilinear of the GPU table", err)
        assert err <= 2e-5


# ---------------------------------------------------------------------------
# SH radiance transfer
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kp,q", [(16, 1.0), (9, 1.0), (4, 3.5), (1, 1.0), (16, 8.0)])
def test_sh_transfer_matches_oracle(kp, q):
    _check_sh_transfer(kp, q, 32, 64)


# grids whose columns are padded to 16 (13, 100, 1, 40), whose waves'
# direction ranges cross rows (48 x 100: 7 groups of 16 per row, 42 groups per
# wave) or start inside a row (17 x 40), with fewer direction groups than
# waves (3 x 16, 1 x 1), and with long rows (4 x 2048: 128 groups per row, the
# column angle of each group carried by 63 rotation steps from the wave's
# first group)
@pytest.mark.parametrize("kp,q,n_theta,n_phi", [(9, 1.0, 7, 13), (16, 1.0, 48, 100), (4, 3.5, 3, 16),
                                                 (1, 1.0, 1, 1), (16, 2.0, 17, 40), (16, 1.0, 4, 2048)])
def test_sh_transfer_on_other_grids(kp, q, n_theta, n_phi):
    _check_sh_transfer(kp, q, n_theta, n_phi)


def _check_sh_transfer(kp, q, n_theta, n_phi):
    import paper_2601_01660_amd as P
    c = synth.cfg2(n_scene=10, n_avatar=3000)
    av = c["avatar"]
    rng = np.random.default_rng(40 + kp)
    probe = synth.sh_probe(rng, kp)
    f = c["colour_sh"]
    gs = P.GaussianSet.from_host(av)
    cen_gpu = P.dgsm_alpha_centroid(gs)
    cen = osh.alpha_centroid(av.mean, av.opacity)
    assert np.abs(cen_gpu.cpu().numpy() - cen).max() <= 1e-6
    s, fo, rgb = P.sh_transfer(torch.from_numpy(probe), gs, torch.from_numpy(f), cen_gpu, q=q, n_theta=n_theta,
                               n_phi=n_phi)
    torch.cuda.synchronize()
    s_ref, f_ref, rgb_ref = osh.relight(probe, av, f, centroid=cen_gpu.cpu().numpy().astype(np.float64), q=q,
                                        n_theta=n_theta, n_phi=n_phi)
    s = s.cpu().numpy()
    # normals that sit on the centroid plane may legitimately flip: accept either side there
    n = osh.normals(av.rot, av.scale, av.mean, cen_gpu.cpu().numpy().astype(np.float64))
    side = np.abs(np.einsum("ni,ni->n", n, av.mean - cen_gpu.cpu().numpy()))
    amb = side < 1e-5
    s_flip = osh.transfer_scale(probe, -n[amb], n_theta, n_phi, q=q) if amb.any() else None
    # relative 1e-4, with an absolute floor of 5e-6 where s is near zero (a 2048-term
    # FP32 sum of mixed-sign radiance carries ~1e-7 absolute rounding)
    rel = np.abs(s - s_ref) / np.maximum(np.abs(s_ref), 0.05)
    if amb.any():
        rel_f = np.abs(s[amb] - s_flip) / np.maximum(np.abs(s_flip), 0.05)
        rel[amb] = np.minimum(rel[amb], rel_f)
    print(f"[parity] sh kp={kp} q={q} grid {n_theta}x{n_phi}: max rel = {rel.max():.3e}", flush=True)
    assert rel.max() <= 1e-4
    ok = ~amb
    assert np.abs(fo.cpu().numpy()[ok] - f_ref[ok]).max() <= 1e-4 * max(1.0, np.abs(f_ref).max())
    assert np.abs(rgb.cpu().numpy()[ok] - rgb_ref[ok]).max() <= 1e-4 * max(1.0, np.abs(rgb_ref).max())


def test_domain_check_counts_bad_gaussians():
    import paper_2601_01660_amd as P
    rng = np.random.default_rng(3)
    g = synth.random_gaussians(rng, rng.uniform(-1, 1, (1000, 3)), 0.03)
    assert P.dgsm_check_gaussians(P.GaussianSet.from_host(g)) == 0
    mean, scale, rot, opac = g.mean.copy(), g.scale.copy(), g.rot.copy(), g.opacity.copy()
    mean[5, 1] = np.nan
    scale[17, 2] = 0.0
    rot[300] = 0.0
    opac[999] = 1.0
    opac[640] = -0.1
    scale[640, 0] = np.inf          # two faults on one Gaussian count once
    bad = P.GaussianSet.from_host(synth.Gaussians(mean, scale, rot, opac))
    assert P.dgsm_check_gaussians(bad) == 5


@pytest.mark.parametrize("kind", ["stencil7", "mc16"])
def test_footprint_query_matches_oracle(cfg1, kind):
    import paper_2601_01660_amd as P
    U = _util()
    g = cfg1["gaussians"]
    T, atlas = U.gpu_build(g, cfg1["lights"], cfg1["atlas"])
    if kind == "stencil7":
        z, w = od.footprint_stencil7()
    else:
        z = np.random.default_rng(12).normal(size=(16, 3))
        w = np.full(16, 1 / 16)
    got = P.dgsm_query_footprint(torch.from_numpy(cfg1["lights"]), atlas, T, P.GaussianSet.from_host(g),
                                 torch.from_numpy(z.astype(np.float32)), torch.from_numpy(w.astype(np.float32)))
    torch.cuda.synchronize()
    a = cfg1["atlas"]
    zf = z.astype(np.float32).astype(np.float64)      # the offsets the device saw
    ref = od.query_footprint(cfg1["oracle_T"], cfg1["lights"][0], g, zf, w, a.spacing, a.r0, a.r1)
    err = np.abs(got[0].cpu().numpy() - ref).max()
    _report(f"footprint {kind}", err)
    assert err <= TOL


@pytest.mark.parametrize("beta", ["constant", "density"])
def test_beta_mappings_match_oracle(beta):
    """Ablation B mappings: the build with each opacity-to-absorption mapping
    against the oracle (small Gaussians make the density mapping strong)."""
    U = _util()
    rng = np.random.default_rng(17)
    g = synth.random_gaussians(rng, rng.uniform(0.5, 2.5, (1500, 3)), 0.03)
    spec = synth.AtlasSpec(24, 24, 12, "geometric")
    light = np.zeros((1, 3), np.float32)
    kappa = 0.05 if beta == "density" else 0.5
    T, _ = U.gpu_build(g, light, spec, kappa=kappa, beta=beta)
    ref = od.build(light[0], g, spec.H, spec.W, spec.K, spec.spacing, spec.r0, spec.r1, kappa=kappa, beta=beta)
    err = np.abs(T[0].cpu().numpy().astype(np.float64) - ref).max()
    _report(f"beta {beta} (min T {ref.min():.3f})", err)
    assert ref.min() < 0.9 and err <= TOL


def test_maximum_shell_count():
    """K = 256 (the largest supported): four shell radii per lane of the shell
    table, LDS accumulators of 128 KiB per tile, long erf ramps."""
    U = _util()
    rng = np.random.default_rng(29)
    g = synth.random_gaussians(rng, rng.uniform(-1.5, 1.5, (400, 3)) + [0, 0, 1.0], 0.08)
    lights = np.array([[0.1, 0.0, -0.2]], np.float32)
    spec = synth.AtlasSpec(16, 16, 256, r0=0.05, r1=4.0)
    T, _ = U.gpu_build(g, lights, spec)
    ref = od.build(lights[0], g, spec.H, spec.W, spec.K, spec.spacing, spec.r0, spec.r1)
    err = np.abs(T[0].cpu().numpy() - ref).max()
    _report("K = 256", err)
    assert err <= TOL


def test_maximum_atlas_side_sampled():
    """A 1024 x 1024 atlas (the largest side) with few Gaussians: sampled texels
    against the oracle, and T = 1 far from every Gaussian."""
    U = _util()
    c = synth.cfg1(400)
    spec = synth.AtlasSpec(1024, 1024, 8)
    T, _ = U.gpu_build(c["gaussians"], c["lights"], spec)
    i, j = U.sample_texels(c["gaussians"], c["lights"][0], 1024, 1024, 40, seed=3)
    ref = od.build_texels(c["lights"][0], c["gaussians"], i, j, 8, H=1024, W=1024)
    got = T[0].cpu().numpy()[:, i, j].T.astype(np.float64)
    err = np.abs(got - ref).max()
    _report("1024 x 1024 sampled", err)
    assert err <= TOL
    # directions pointing away from the Gaussians' octant see nothing
    assert torch.all(T[0, :, 1023, 1023] == 1.0) and torch.all(T[0, :, 0, 0] == 1.0)


@pytest.mark.parametrize("Kp,lam,cube", [(16, 0.0, True), (9, 0.05, True), (16, 0.01, False)])
def test_probe_fit_matches_oracle(Kp, lam, cube):
    """Sec. 3.4 weighted ridge fit: cube-map samples (solid-angle weights) or
    scattered directions with random weights, against the FP64 oracle."""
    import paper_2601_01660_amd as P
    rng = np.random.default_rng(40 + Kp)
    if cube:
        D, w = synth.cubemap_directions(48)
    else:
        D = rng.normal(size=(20000, 3))
        D /= np.linalg.norm(D, axis=1, keepdims=True)
        w = rng.uniform(0.2, 1.0, 20000) * (4 * np.pi / 20000)
    Y = rng.uniform(0.0, 2.0, (D.shape[0], 3))
    D32, w32, Y32 = D.astype(np.float32), w.astype(np.float32), Y.astype(np.float32)
    A = P.dgsm_probe_fit(torch.from_numpy(Y32), torch.from_numpy(D32), torch.from_numpy(w32), Kp, lam)
    torch.cuda.synchronize()
    ref = osh.probe_fit(Y32.astype(np.float64), D32.astype(np.float64), w32.astype(np.float64),
                        int(round(math.sqrt(Kp))) - 1, lam)
    err = np.abs(A.cpu().numpy() - ref).max() / np.abs(ref).max()
    _report(f"probe fit Kp={Kp} lam={lam} cube={cube} (relative)", err)
    assert err <= 1e-4


def test_workspace_sized_for_the_set():
    """A workspace holding exactly the list entries a set needs (counted by
    dgsm_count_entries) gives the atlas of the worst-case workspace bit for bit;
    one too small for the set is refused by nothing but leaves every list empty
    (T = 1, no write past its end) and says so through dgsm_list_entries."""
    import paper_2601_01660_amd as P
    c = synth.cfg1(3000)
    g, lights = c["gaussians"], torch.from_numpy(np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 0.5]], np.float32)).cuda()
    atlas = P.Atlas(96, 80, 12)
    gs = P.GaussianSet.from_host(g)
    entries = P.dgsm_count_entries(lights, gs, atlas)
    worst = P.dgsm_build_workspace_size(atlas, g.n, 2)
    exact = P.dgsm_build_workspace_size_entries(atlas, g.n, 2, entries)
    assert 0 < exact < worst
    ws = torch.empty(exact, dtype=torch.uint8, device="cuda")
    T_exact = P.dgsm_build(lights, gs, atlas, workspace=ws)
    T_worst = P.dgsm_build(lights, gs, atlas)
    torch.cuda.synchronize()
    assert torch.equal(T_exact, T_worst)
    for l in range(2):
        need, cap = P.dgsm_list_entries(atlas, g.n, 2, ws, l)
        assert need <= cap and cap >= entries
    small = torch.empty(P.dgsm_build_workspace_size_entries(atlas, g.n, 2, 0), dtype=torch.uint8, device="cuda")
    T_small = P.dgsm_build(lights, gs, atlas, workspace=small)
    torch.cuda.synchronize()
    need, cap = P.dgsm_list_entries(atlas, g.n, 2, small, 0)
    print(f"[parity] workspace for the set: {entries} entries, {exact} vs {worst} bytes; too small: need {need} "
          f"> capacity {cap}", flush=True)
    assert need > cap and need == P.dgsm_list_entries(atlas, g.n, 2, ws, 0)[0]
    assert torch.all(T_small == 1.0)
