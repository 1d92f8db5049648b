"""FP64 oracle: learned per-light transmittance field (forward, backward, Adam).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component; this is the surrogate that the build's
batched extension trains on its own atlases.  Definition (all FP64 here):

  input   a point x seen from light o_L: (u, v) = octahedral code of x - o_L
          (Sec. 3.2 encoding), rho in [-1, 1] the radius coordinate
          (geometric shells: 2 ln(r/r0)/ln(r1/r0) - 1; uniform: 2 r/r1 - 1),
          clamped to [-1, 1]
  features phi[128]: u, v, rho, then for i = 0..15 with f_i = pi F^(i/15)
          (F = W/4 for a W-wide atlas): sin(f_i u), cos(f_i u), sin(f_i v),
          cos(f_i v), sin(f_i rho), cos(f_i rho); zeros from index 99 on
  network h1 = relu(W0 phi + b0), h_{l+1} = relu(W_l h_l + b_l) for l = 1..3,
          z = w4 . h4 + b4, predicted T = sigmoid(-z) (log T = -softplus(z))
  loss    mean over the batch of (T - T*)^2

With ``bf16=True`` the forward/backward round exactly where the MFMA path
feeds its matrix units (BF16, round to nearest even of the FP32 value):
weights W0..W3, the features phi, the hidden activations h1..h3 entering the
next layer, and the back-propagated pre-activation gradients entering the
weight and data-gradient products.  Accumulation stays exact (FP64), so a GPU
result differs from this one only by FP32 accumulation order.
"""
from __future__ import annotations

import math

import numpy as np

NF = 16                 # Fourier frequencies per input
D_IN = 3 + 6 * NF       # 99 live features
D_PAD = 128             # padded feature width
H = 128                 # hidden width
N_HIDDEN = 4
N_PARAMS = N_HIDDEN * (H * H + H) + H + 1   # 66177


def bf16(x):
    """Round to BF16 (RNE) via FP32, returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def frequencies(W):
    """f_i = pi (W/4)^(i/15), i = 0..15."""
    F = W / 4.0
    return math.pi * F ** (np.arange(NF) / (NF - 1.0))


def unpack(flat):
    """Flat FP32/FP64 parameter vector -> dict (layout of the device buffer)."""
    flat = np.asarray(flat, dtype=np.float64)
    p, o = {}, 0
    for l in range(N_HIDDEN):
        p[f"W{l}"] = flat[o:o + H * H].reshape(H, H); o += H * H
        p[f"b{l}"] = flat[o:o + H]; o += H
    p["w4"] = flat[o:o + H]; o += H
    p["b4"] = flat[o]
    return p


def pack(p):
    parts = []
    for l in range(N_HIDDEN):
        parts += [np.ravel(p[f"W{l}"]), np.ravel(p[f"b{l}"])]
    parts += [np.ravel(p["w4"]), np.atleast_1d(p["b4"])]
    return np.concatenate(parts).astype(np.float64)


def encode_points(points, light, r0, r1, spacing="geometric"):
    """(u, v, rho) of world points for one light."""
    d = np.asarray(points, np.float64) - np.asarray(light, np.float64)
    r = np.linalg.norm(d, axis=1)
    l1 = np.abs(d).sum(1)
    q = np.where(l1[:, None] > 0, d / np.where(l1 > 0, l1, 1.0)[:, None], np.array([0.0, 0.0, 1.0]))
    up = q[:, 2] >= 0
    sx = np.where(q[:, 0] >= 0, 1.0, -1.0)
    sy = np.where(q[:, 1] >= 0, 1.0, -1.0)
    u = np.where(up, q[:, 0], sx * (1 - np.abs(q[:, 1])))
    v = np.where(up, q[:, 1], sy * (1 - np.abs(q[:, 0])))
    if spacing == "geometric":
        with np.errstate(divide="ignore"):
            rho = 2 * np.log(np.maximum(r, 1e-300) / r0) / math.log(r1 / r0) - 1
    else:
        rho = 2 * r / r1 - 1
    return u, v, np.clip(rho, -1.0, 1.0)


def features(u, v, rho, W):
    """phi [B, 128] (Fourier encoding of (u, v, rho))."""
    f = frequencies(W)
    B = np.shape(u)[0]
    phi = np.zeros((B, D_PAD))
    phi[:, 0], phi[:, 1], phi[:, 2] = u, v, rho
    for i in range(NF):
        for c, x in enumerate((u, v, rho)):
            phi[:, 3 + 6 * i + 2 * c] = np.sin(f[i] * x)
            phi[:, 3 + 6 * i + 2 * c + 1] = np.cos(f[i] * x)
    return phi


def forward(flat, phi, bf16_emulation=True):
    """Returns (T_pred [B], cache) for the backward pass."""
    p = unpack(flat)
    rnd = bf16 if bf16_emulation else (lambda x: np.asarray(x, np.float64))
    x = rnd(phi)
    cache = {"x0": x}
    h = None
    for l in range(N_HIDDEN):
        a = x @ rnd(p[f"W{l}"]).T + p[f"b{l}"]
        h = np.maximum(a, 0.0)
        cache[f"a{l}"] = a
        x = rnd(h) if l < N_HIDDEN - 1 else h
        cache[f"x{l + 1}"] = x
    z = h @ p["w4"] + p["b4"]
    T = 1.0 / (1.0 + np.exp(z))
    cache["z"], cache["T"] = z, T
    return T, cache


def loss(T, target):
    return float(np.mean((T - target) ** 2))


def backward(flat, cache, target, bf16_emulation=True):
    """Gradient of the mean squared T error, as a flat vector in the parameter layout."""
    p = unpack(flat)
    rnd = bf16 if bf16_emulation else (lambda x: np.asarray(x, np.float64))
    T = cache["T"]
    B = T.shape[0]
    gz = 2.0 * (T - target) / B * (-T * (1.0 - T))     # dL/dz
    g = {"w4": cache[f"x{N_HIDDEN}"].T @ gz, "b4": gz.sum()}
    dh = np.outer(gz, p["w4"])                          # dL/dh4
    for l in range(N_HIDDEN - 1, -1, -1):
        da = dh * (cache[f"a{l}"] > 0)
        dar = rnd(da)
        g[f"W{l}"] = dar.T @ cache[f"x{l}"]
        g[f"b{l}"] = da.sum(0)
        if l > 0:
            dh = dar @ rnd(p[f"W{l}"])
    return pack(g)


def adam(flat, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t >= 1); returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
