"""Shared helpers for the GPU parity tests (HIP path through the C ABI vs the FP64 oracle)."""
import numpy as np
import torch

import paper_2601_01660_amd as P
from oracle import dgsm as od


def gpu_build(g, lights, spec, dtype="f32", cull_eps=1e-8, kappa=1.0, beta="trace"):
    gs = P.GaussianSet.from_host(g)
    atlas = P.Atlas.from_spec(spec, dtype=dtype, cull_eps=cull_eps)
    T = P.dgsm_build(torch.from_numpy(np.ascontiguousarray(lights, dtype=np.float32)), gs, atlas, kappa, beta=beta)
    torch.cuda.synchronize()
    return T, atlas


def gpu_query(lights, atlas, T, points):
    out = P.dgsm_query(torch.from_numpy(np.ascontiguousarray(lights, dtype=np.float32)), atlas, T,
                       torch.from_numpy(np.ascontiguousarray(points, dtype=np.float32)))
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def texels_towards(points, light, H, W):
    """(row, col) of the texel containing the direction from the light to each point."""
    u, v = od.octahedral_encode(np.asarray(points, np.float64) - np.asarray(light, np.float64))
    j = np.clip(np.floor((u + 1) * W / 2).astype(int), 0, W - 1)
    i = np.clip(np.floor((v + 1) * H / 2).astype(int), 0, H - 1)
    return i, j


def sample_texels(g, light, H, W, n, seed):
    """Seeded texels: half aimed at random Gaussian centres (likely shadowed), half uniform."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(g.n, n // 2, replace=False)
    i1, j1 = texels_towards(g.mean[idx], light, H, W)
    i2 = rng.integers(0, H, n - n // 2)
    j2 = rng.integers(0, W, n - n // 2)
    return np.concatenate([i1, i2]), np.concatenate([j1, j2])
