"""FP64 oracle: SH probe evaluation and per-Gaussian radiance transfer.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.4 fits SH coefficients A [K, 3] (K = (d+1)^2) of the environment and
evaluates L(w) = B(w) A.  Sec. 3.5 samples a latitude-longitude grid {w_j}
with weights w_j proportional to sin(theta_j), aggregates incident light with
a cosine lobe S(w, n) = max(0, <w, n>)^q and forms the per-channel scale

    s_c(n) = clip_[0, t_max]( sum_j w_j L_c(w_j) S_j / (sum_j w_j S_j + eps) ),

then the relit colour c' = max(0, gamma c (.) s(n)).

Readings where the paper is silent:
* real SH, orthonormal on the sphere, index k = l^2 + l + m, WITHOUT the
  Condon-Shortley phase, so Y_1,-1 ~ +y, Y_1,0 ~ +z, Y_1,1 ~ +x;
* grid cell centres theta_a = (a + 1/2) pi / n_theta, phi_b = (b + 1/2) 2 pi / n_phi,
  w = (sin theta cos phi, sin theta sin phi, cos theta), weight sin(theta);
* the normal n is the rotation column of the smallest scale (ties: lowest
  axis), signed so that n . (mu - centroid) >= 0 with the alpha-weighted
  centroid of the avatar Gaussians;
* colour SH coefficients f [16, 3] are scaled per channel by gamma s_c with
  no clamp; the clamp max(0, .) applies to the DC colour c = 0.5 + C0 f_0
  (C0 = 1 / (2 sqrt(pi))), which is the RGB output.
"""
from __future__ import annotations

import math
import numpy as np

from .dgsm import quaternion_to_matrix

C0 = 0.5 / math.sqrt(math.pi)


def _assoc_legendre(l, m, x):
    """P_l^m(x), m >= 0, without the Condon-Shortley phase (upward recurrence)."""
    pmm = np.ones_like(x)
    somx2 = np.sqrt(np.maximum(0.0, 1 - x * x))
    fact = 1.0
    for _ in range(m):
        pmm = pmm * fact * somx2
        fact += 2.0
    if l == m:
        return pmm
    pmmp1 = x * (2 * m + 1) * pmm
    if l == m + 1:
        return pmmp1
    pll = pmmp1
    for ll in range(m + 2, l + 1):
        pll = ((2 * ll - 1) * x * pmmp1 - (ll + m - 1) * pmm) / (ll - m)
        pmm, pmmp1 = pmmp1, pll
    return pll


def real_sh(l_max, dirs):
    """Real orthonormal SH basis B [M, (l_max+1)^2] at unit directions [M, 3]."""
    dirs = np.asarray(dirs, dtype=np.float64)
    x, y, z = dirs[:, 0], dirs[:, 1], dirs[:, 2]
    phi = np.arctan2(y, x)
    ct = np.clip(z, -1.0, 1.0)
    out = np.zeros((dirs.shape[0], (l_max + 1) ** 2))
    for l in range(l_max + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            K = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            P = _assoc_legendre(l, am, ct)
            if m > 0:
                val = math.sqrt(2) * K * np.cos(am * phi) * P
            elif m < 0:
                val = math.sqrt(2) * K * np.sin(am * phi) * P
            else:
                val = K * P
            out[:, l * l + l + m] = val
    return out


def latlong_grid(n_theta, n_phi):
    """Directions [M, 3] and weights w_j = sin(theta_j) of the lat-long grid."""
    th = (np.arange(n_theta) + 0.5) * math.pi / n_theta
    ph = (np.arange(n_phi) + 0.5) * 2 * math.pi / n_phi
    T, P = np.meshgrid(th, ph, indexing="ij")
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    return dirs, np.sin(T).reshape(-1)


def probe_radiance(probe, dirs):
    """L(w) = B(w) A for probe A [Kp, 3]; returns [M, 3] (Sec. 3.4)."""
    probe = np.asarray(probe, dtype=np.float64)
    l_max = int(round(math.sqrt(probe.shape[0]))) - 1
    return real_sh(l_max, dirs) @ probe


def alpha_centroid(mean, opacity):
    mean = np.asarray(mean, dtype=np.float64)
    a = np.asarray(opacity, dtype=np.float64)
    return (a[:, None] * mean).sum(0) / a.sum()


def normals(rot, scale, mean, centroid):
    """Smallest-scale rotation column, oriented away from the centroid."""
    R = quaternion_to_matrix(rot)
    axis = np.argmin(np.asarray(scale, dtype=np.float64), axis=1)
    n = R[np.arange(R.shape[0]), :, axis]
    side = np.einsum("ni,ni->n", n, np.asarray(mean, dtype=np.float64) - centroid)
    return np.where(side[:, None] >= 0, n, -n)


def transfer_scale(probe, n, n_theta=32, n_phi=64, q=1.0, clip_max=4.0, eps=1e-6, chunk=4096):
    """Per-channel lighting scale s_c(n) [N, 3] (Sec. 3.5)."""
    dirs, w = latlong_grid(n_theta, n_phi)
    L = probe_radiance(probe, dirs)
    n = np.asarray(n, dtype=np.float64)
    out = np.empty((n.shape[0], 3))
    for s in range(0, n.shape[0], chunk):
        cos = n[s:s + chunk] @ dirs.T
        S = np.maximum(0.0, cos) ** q
        num = (S * w) @ L
        den = (S * w).sum(1, keepdims=True) + eps
        out[s:s + chunk] = np.clip(num / den, 0.0, clip_max)
    return out


def relight(probe, gaussians, colour_sh, centroid=None, n_theta=32, n_phi=64, q=1.0,
            clip_max=4.0, eps=1e-6, gamma=1.0):
    """Scales s [N,3], relit SH coefficients [N,16,3] and clamped RGB [N,3]."""
    if centroid is None:
        centroid = alpha_centroid(gaussians.mean, gaussians.opacity)
    n = normals(gaussians.rot, gaussians.scale, gaussians.mean, centroid)
    s = transfer_scale(probe, n, n_theta, n_phi, q, clip_max, eps)
    f = np.asarray(colour_sh, dtype=np.float64)
    f_out = gamma * s[:, None, :] * f
    rgb = np.maximum(0.0, gamma * (0.5 + C0 * f[:, 0, :]) * s)
    return s, f_out, rgb


# ---------------------------------------------------------------------------
# Approximate HDRI probe (Sec. 3.4): weighted ridge least squares of the SH
# coefficients from radiance samples Y at directions D with weights w (the
# renderer's output; synth.cubemap_directions makes cube-face samples).
# ---------------------------------------------------------------------------

def probe_fit(Y, D, w, l_max, lam):
    """A [K, 3], K = (l_max + 1)^2, minimising ||W^(1/2) (B A - Y)||_F^2 + lam ||A||_F^2
    with B = real_sh(l_max, D) and W = diag(w): (B^T W B + lam I) A = B^T W Y."""
    B = real_sh(l_max, D)
    w = np.asarray(w, dtype=np.float64)
    G = B.T @ (w[:, None] * B) + lam * np.eye(B.shape[1])
    R = B.T @ (w[:, None] * np.asarray(Y, dtype=np.float64))
    return np.linalg.solve(G, R)
