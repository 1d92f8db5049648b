"""Seeded synthetic inputs for the DGSM hot path.

This module only draws random scenes; it holds none of the method's
arithmetic (no precision matrices, no optical depth, no atlas logic).  Both
the FP64 oracle tests and the GPU path read their inputs from here, so the
two sides always see bit-identical FP32 arrays.

The paper evaluates on captured scenes and avatars (ScanNet++, DL3DV,
SuperSplat, AvatarX, ActorsHQ, NeuralDome) that are not available here;
the generators below stand in for them with the sizes and distributions of
the five workload configurations:

* ``cfg1``: 1 light at the origin, 5,000 Gaussians uniform in [0.5, 4.5]^3,
  32x32 atlas x 16 geometric shells (0.05-8 m).
* ``cfg2``: an 8x8x3 m room (floor slab, wall slabs, volume) with 500k
  scene Gaussians plus a 100k avatar in an upright capsule, 256x256x64.
* ``cfg3``: the same room at 2M scene + 150k avatar Gaussians, 4 lights,
  60 frames of rigid avatar translation, 512x512x64 (FP16 storage).
* ``cfg5``: 6M scene Gaussians, 8 lights, 8 avatars x 200k.

Scales are log-normal per axis (median m, sigma_log 0.5), rotations are
normalised N(0, I4) quaternions (uniform on SO(3)), opacities U[0.05, 0.99].
"""
from __future__ import annotations

import dataclasses
import numpy as np

ROOM_LO = np.array([-4.0, -4.0, 0.0])
ROOM_HI = np.array([4.0, 4.0, 3.0])
SHELL_R0 = 0.05
SHELL_R1 = 8.0


@dataclasses.dataclass
class Gaussians:
    """Structure-of-arrays Gaussian set, all float32 and C-contiguous."""

    mean: np.ndarray      # [N, 3] metres
    scale: np.ndarray     # [N, 3] standard deviations in metres (not log)
    rot: np.ndarray       # [N, 4] unit quaternion (w, x, y, z)
    opacity: np.ndarray   # [N]    in [0, 1)

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    def subset(self, idx) -> "Gaussians":
        return Gaussians(np.ascontiguousarray(self.mean[idx]),
                         np.ascontiguousarray(self.scale[idx]),
                         np.ascontiguousarray(self.rot[idx]),
                         np.ascontiguousarray(self.opacity[idx]))

    def translated(self, t) -> "Gaussians":
        """Rigidly translated copy (single FP32 rounding per coordinate)."""
        t = np.asarray(t, dtype=np.float32).reshape(1, 3)
        return Gaussians((self.mean + t).astype(np.float32), self.scale, self.rot,
                         self.opacity)

    @staticmethod
    def concat(parts) -> "Gaussians":
        return Gaussians(*(np.ascontiguousarray(np.concatenate([getattr(p, f) for p in parts]))
                           for f in ("mean", "scale", "rot", "opacity")))

    @staticmethod
    def empty() -> "Gaussians":
        return Gaussians(np.zeros((0, 3), np.float32), np.ones((0, 3), np.float32),
                         np.tile(np.array([[1, 0, 0, 0]], np.float32), (0, 1)),
                         np.zeros((0,), np.float32))


@dataclasses.dataclass
class AtlasSpec:
    H: int
    W: int
    K: int
    spacing: str = "geometric"   # or "uniform"
    r0: float = SHELL_R0
    r1: float = SHELL_R1


def _streams(cfg_id: int, n: int):
    ss = np.random.SeedSequence(1000 + cfg_id)
    return [np.random.default_rng(s) for s in ss.spawn(n)]


def _attributes(rng_s, rng_r, rng_o, n, median):
    scale = median * np.exp(0.5 * rng_s.standard_normal((n, 3)))
    q = rng_r.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q[q[:, 0] < 0] *= -1.0          # canonical hemisphere, same rotation
    opacity = rng_o.uniform(0.05, 0.99, n)
    return scale.astype(np.float32), q.astype(np.float32), opacity.astype(np.float32)


def random_gaussians(rng, centers, median) -> Gaussians:
    """Attach log-normal scales, uniform rotations and opacities to centres."""
    n = centers.shape[0]
    r1, r2, r3 = (np.random.default_rng(rng.integers(1 << 62)) for _ in range(3))
    s, q, o = _attributes(r1, r2, r3, n, median)
    return Gaussians(np.ascontiguousarray(centers, dtype=np.float32), s, q, o)


def room_centres(rng, n: int) -> np.ndarray:
    """Centres of an 8x8x3 m room: 35% floor slab, 35% wall slabs, 30% volume."""
    n_floor = int(round(0.35 * n))
    n_wall = int(round(0.35 * n))
    n_vol = n - n_floor - n_wall
    floor = np.column_stack([rng.uniform(-4, 4, n_floor), rng.uniform(-4, 4, n_floor),
                             rng.uniform(0.0, 0.1, n_floor)])
    # four walls of equal area (8 m x 3 m), each a 0.1 m slab inside the room
    which = rng.integers(0, 4, n_wall)
    along = rng.uniform(-4, 4, n_wall)
    depth = rng.uniform(3.9, 4.0, n_wall)
    z = rng.uniform(0.0, 3.0, n_wall)
    wx = np.where(which == 0, depth, np.where(which == 1, -depth, along))
    wy = np.where(which == 2, depth, np.where(which == 3, -depth, along))
    wall = np.column_stack([wx, wy, z])
    vol = rng.uniform(ROOM_LO, ROOM_HI, (n_vol, 3))
    c = np.concatenate([floor, wall, vol])
    return c[rng.permutation(n)]


def capsule_centres(rng, n: int, feet=(1.0, 0.5, 0.0), semi=(0.25, 0.15), height=1.8):
    """Uniform points in an upright elliptic capsule standing at ``feet``."""
    cap = 0.25                       # z semi-axis of the two end caps
    half_cyl = height / 2 - cap
    out = np.empty((0, 3))
    while out.shape[0] < n:
        m = 2 * (n - out.shape[0]) + 64
        p = rng.uniform([-1, -1, -height / 2], [1, 1, height / 2], (m, 3))
        zc = np.maximum(0.0, np.abs(p[:, 2]) - half_cyl) / cap
        ok = p[:, 0] ** 2 + p[:, 1] ** 2 + zc ** 2 <= 1.0
        out = np.concatenate([out, p[ok]])
    out = out[:n]
    out[:, 0] *= semi[0]
    out[:, 1] *= semi[1]
    out[:, 2] += height / 2
    return out + np.asarray(feet)


def random_walk(rng, frames: int, step=0.05, turn_sigma=0.3, bound=3.5, start=(1.0, 0.5)):
    """Per-frame rigid translations (frames x 3, float32) of a 2-D random walk.

    The heading changes by N(0, turn_sigma) each frame; the walker is reflected
    at |x|, |y| <= bound.  Frame 0 has zero translation.
    """
    pos = np.array(start, dtype=np.float64)
    start = pos.copy()
    heading = rng.uniform(0, 2 * np.pi)
    out = np.zeros((frames, 3))
    for f in range(1, frames):
        heading += rng.normal(0.0, turn_sigma)
        nxt = pos + step * np.array([np.cos(heading), np.sin(heading)])
        for ax in range(2):
            if abs(nxt[ax]) > bound:
                nxt[ax] = np.sign(nxt[ax]) * (2 * bound - abs(nxt[ax]))
                heading = np.pi - heading if ax == 0 else -heading
        pos = nxt
        out[f, :2] = pos - start
    return out.astype(np.float32)


def sh_probe(rng, kp: int) -> np.ndarray:
    """Seeded SH radiance probe [kp, 3]: DC ~ U[0.5, 1.5], higher ~ N(0, 0.3^2)."""
    a = rng.normal(0.0, 0.3, (kp, 3))
    a[0] = rng.uniform(0.5, 1.5, 3)
    return a.astype(np.float32)


def sh_colours(rng, n: int, coeffs: int = 16) -> np.ndarray:
    """Per-Gaussian SH colour coefficients [n, coeffs, 3] ~ N(0, 0.5^2)."""
    return rng.normal(0.0, 0.5, (n, coeffs, 3)).astype(np.float32)


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------

def cfg1(n: int = 5000):
    """1 point light at the origin; n Gaussians uniform in [0.5, 4.5]^3, 3 cm."""
    rs = _streams(1, 4)
    centres = rs[0].uniform(0.5, 4.5, (n, 3))
    s, q, o = _attributes(rs[1], rs[2], rs[3], n, 0.03)
    g = Gaussians(centres.astype(np.float32), s, q, o)
    lights = np.zeros((1, 3), np.float32)
    return dict(gaussians=g, lights=lights, atlas=AtlasSpec(32, 32, 16),
                points=g.mean.copy())


def cfg2(n_scene: int = 500_000, n_avatar: int = 100_000, atlas=None):
    """Room scene + capsule avatar, 1 light at (0, 0, 2.5), 256x256x64."""
    rs = _streams(2, 10)
    scene = Gaussians(room_centres(rs[0], n_scene).astype(np.float32),
                      *_attributes(rs[1], rs[2], rs[3], n_scene, 0.03))
    avatar = Gaussians(capsule_centres(rs[4], n_avatar).astype(np.float32),
                       *_attributes(rs[5], rs[6], rs[7], n_avatar, 0.01))
    g = Gaussians.concat([scene, avatar])
    lights = np.array([[0.0, 0.0, 2.5]], np.float32)
    probe = sh_probe(rs[8], 16)
    colours = sh_colours(rs[9], n_avatar)
    return dict(gaussians=g, scene=scene, avatar=avatar, lights=lights,
                atlas=atlas or AtlasSpec(256, 256, 64), points=g.mean.copy(),
                probe=probe, colour_sh=colours)


CFG3_LIGHTS = np.array([[2.0, 2.0, 2.5], [-2.0, 2.0, 2.5], [-2.0, -2.0, 2.5],
                        [2.0, -2.0, 2.5]], np.float32)


def cfg3(n_scene: int = 2_000_000, n_avatar: int = 150_000, frames: int = 60, atlas=None):
    """Room + moving avatar, 4 lights, ``frames`` rigid translations, 512x512x64."""
    rs = _streams(3, 10)
    scene = Gaussians(room_centres(rs[0], n_scene).astype(np.float32),
                      *_attributes(rs[1], rs[2], rs[3], n_scene, 0.03))
    avatar = Gaussians(capsule_centres(rs[4], n_avatar).astype(np.float32),
                       *_attributes(rs[5], rs[6], rs[7], n_avatar, 0.01))
    traj = random_walk(rs[8], frames)
    return dict(scene=scene, avatar=avatar, lights=CFG3_LIGHTS.copy(), trajectory=traj,
                atlas=atlas or AtlasSpec(512, 512, 64))


def cfg5(n_scene: int = 6_000_000, n_avatars: int = 8, n_per_avatar: int = 200_000,
         frames: int = 60, atlas=None):
    """6M-Gaussian room, 8 lights on a 4x2 grid, 8 avatars on their own walks."""
    rs = _streams(5, 8 + 5 * n_avatars)
    scene = Gaussians(room_centres(rs[0], n_scene).astype(np.float32),
                      *_attributes(rs[1], rs[2], rs[3], n_scene, 0.03))
    lights = np.array([[x, y, 2.5] for y in (-1.5, 1.5) for x in (-3.0, -1.0, 1.0, 3.0)],
                      np.float32)
    avatars, trajs, probes9, probes16 = [], [], [], []
    for a in range(n_avatars):
        r = rs[8 + 5 * a: 13 + 5 * a]
        feet = (r[0].uniform(-3, 3), r[0].uniform(-3, 3), 0.0)
        avatars.append(Gaussians(capsule_centres(r[1], n_per_avatar, feet=feet).astype(np.float32),
                                 *_attributes(r[2], r[3], r[4], n_per_avatar, 0.01)))
        trajs.append(random_walk(r[0], frames, start=feet[:2]))
        probes9.append(sh_probe(r[0], 9))
        probes16.append(sh_probe(r[0], 16))
    return dict(scene=scene, avatars=avatars, lights=lights, trajectories=trajs,
                probes9=probes9, probes16=probes16,
                atlas=atlas or AtlasSpec(1024, 1024, 128))


# --------------------------------------------------------------------------
# initial parameters of the learned per-light field (a seeded input)
# --------------------------------------------------------------------------

MLP_HIDDEN = 128
MLP_LAYERS = 4
MLP_LIVE_FEATURES = 99


def mlp_init_params(seed: int) -> np.ndarray:
    """Flat float32 initial parameters: per layer W_l [128][128] (He-uniform over
    the live inputs; padded input columns of layer 0 zero) then b_l = 0, then
    w4 ~ U(+-sqrt(3/128)) and b4 = -2."""
    rng = np.random.default_rng(seed)
    H = MLP_HIDDEN
    parts = []
    for l in range(MLP_LAYERS):
        fan_in = MLP_LIVE_FEATURES if l == 0 else H
        lim = np.sqrt(6.0 / fan_in)
        W = rng.uniform(-lim, lim, (H, H))
        if l == 0:
            W[:, MLP_LIVE_FEATURES:] = 0.0
        parts += [W.ravel(), np.zeros(H)]
    parts += [rng.uniform(-np.sqrt(3.0 / H), np.sqrt(3.0 / H), H), np.array([-2.0])]
    return np.concatenate(parts).astype(np.float32)


# faces: (major axis, u axis, v axis); a pixel's direction is major + a u + b v
CUBE_FACES = np.array([
    [[1, 0, 0], [0, 0, -1], [0, -1, 0]],
    [[-1, 0, 0], [0, 0, 1], [0, -1, 0]],
    [[0, 1, 0], [1, 0, 0], [0, 0, 1]],
    [[0, -1, 0], [1, 0, 0], [0, 0, -1]],
    [[0, 0, 1], [1, 0, 0], [0, -1, 0]],
    [[0, 0, -1], [-1, 0, 0], [0, -1, 0]],
], dtype=np.float64)


def cubemap_directions(res):
    """Sample directions of a six-face 90-degree cube-map render (the probe
    fit's input): pixel-centre unit directions D [6 res^2, 3] and the solid
    angle w of every pixel.  The solid angle of the face-plane
    rectangle [x0, x1] x [y0, y1] at unit distance is
    F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0), F(x, y) = atan2(x y, sqrt(1 + x^2 + y^2))."""
    edges = -1.0 + 2.0 * np.arange(res + 1) / res
    cent = 0.5 * (edges[:-1] + edges[1:])
    a, b = np.meshgrid(cent, cent, indexing="ij")

    def F(x, y):
        return np.arctan2(x * y, np.sqrt(1.0 + x * x + y * y))

    x0, y0 = np.meshgrid(edges[:-1], edges[:-1], indexing="ij")
    x1, y1 = np.meshgrid(edges[1:], edges[1:], indexing="ij")
    omega = (F(x1, y1) - F(x0, y1) - F(x1, y0) + F(x0, y0)).reshape(-1)
    dirs, weights = [], []
    for n, u, v in CUBE_FACES:
        d = n[None, :] + a.reshape(-1, 1) * u[None, :] + b.reshape(-1, 1) * v[None, :]
        dirs.append(d / np.linalg.norm(d, axis=1, keepdims=True))
        weights.append(omega)
    return np.concatenate(dirs), np.concatenate(weights)
