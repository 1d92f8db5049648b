"""Pins for the FP64 MLP oracle: finite differences, closed forms, library rounding."""
import math

import numpy as np
import pytest
import torch

from oracle import dgsm as od
import synth
from oracle import mlp as om


def _batch(seed=0, B=24):
    rng = np.random.default_rng(seed)
    u, v, rho = rng.uniform(-1, 1, (3, B))
    return om.features(u, v, rho, 64), rng.uniform(0, 1, B)


def test_parameter_count_and_pack_roundtrip():
    flat = synth.mlp_init_params(3)
    assert flat.shape == (om.N_PARAMS,) == (66177,)
    assert np.array_equal(om.pack(om.unpack(flat)), flat.astype(np.float64))
    assert np.all(om.unpack(flat)["W0"][:, om.D_IN:] == 0)


def test_backward_matches_central_differences():
    phi, t = _batch(1)
    flat = synth.mlp_init_params(4).astype(np.float64)
    flat += np.random.default_rng(5).normal(0, 0.05, flat.shape)      # non-trivial biases
    T, cache = om.forward(flat, phi, bf16_emulation=False)
    g = om.backward(flat, cache, t, bf16_emulation=False)
    rng = np.random.default_rng(6)
    p = om.unpack(np.arange(om.N_PARAMS, dtype=np.float64))           # index map
    idx = np.concatenate([rng.choice(p["W0"][:, :om.D_IN].ravel().astype(int), 6),
                          rng.choice(p["W2"].ravel().astype(int), 6), rng.choice(p["b1"].astype(int), 4),
                          rng.choice(p["b3"].astype(int), 4), rng.choice(p["w4"].astype(int), 4),
                          [int(p["b4"])]])
    h = 1e-6
    for i in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        num = (om.loss(om.forward(fp, phi, False)[0], t) - om.loss(om.forward(fm, phi, False)[0], t)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1e-4, abs(g[i])) + 1e-11, (i, num, g[i])


def test_zero_network_closed_form():
    phi, t = _batch(2)
    p = om.unpack(np.zeros(om.N_PARAMS))
    p["b4"] = 0.7
    flat = om.pack(p)
    T, cache = om.forward(flat, phi)
    ref = 1.0 / (1.0 + math.exp(0.7))
    assert np.allclose(T, ref, rtol=0, atol=1e-15)
    g = om.unpack(om.backward(flat, cache, t))
    assert abs(g["b4"] - np.mean(2 * (ref - t) * (-ref * (1 - ref)))) < 1e-15
    assert np.all(g["W0"] == 0) and np.all(g["w4"] == 0)


def test_bf16_rounding_matches_torch():
    x = np.random.default_rng(7).normal(0, 3, 10000).astype(np.float32)
    x = np.concatenate([x, np.float32([1 + 2 ** -8, 1 + 3 * 2 ** -9, -1 - 2 ** -8, 0.0, 65504.0])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(om.bf16(x), ref)
    assert om.bf16(np.float32(1 + 2 ** -8)) == 1.0          # tie to even


def test_features_special_values():
    phi = om.features(np.zeros(1), np.zeros(1), np.zeros(1), 512)
    assert np.all(phi[0, 3:om.D_IN:2] == 0) and np.all(phi[0, 4:om.D_IN:2] == 1)
    assert np.all(phi[0, om.D_IN:] == 0)
    f = om.frequencies(512)
    assert abs(f[0] - math.pi) < 1e-15 and abs(f[-1] - math.pi * 128) < 1e-9
    phi = om.features(np.ones(1), -np.ones(1), np.zeros(1), 512)
    assert abs(phi[0, 3]) < 1e-15 and abs(phi[0, 4] + 1) < 1e-15      # sin(pi), cos(pi)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(8)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    p1, m, v = om.adam(p0, g, np.zeros(50), np.zeros(50), 1, lr=1e-2, eps=0.0)
    assert np.allclose(p1, p0 - 1e-2 * np.sign(g), rtol=0, atol=1e-15)


def test_point_encoding_matches_octahedral_map():
    rng = np.random.default_rng(9)
    pts = rng.uniform(-5, 5, (500, 3))
    light = np.array([0.3, -0.2, 1.0])
    u, v, rho = om.encode_points(pts, light, 0.05, 8.0)
    uu, vv = od.octahedral_encode(pts - light)
    assert np.allclose(u, uu, atol=1e-15) and np.allclose(v, vv, atol=1e-15)
    r = np.linalg.norm(pts - light, axis=1)
    inside = (r > 0.05) & (r < 8.0)
    k = od.query_coords(light, pts, 8, 8, 33)[2]       # fractional shell of 33 geometric shells
    assert np.allclose(rho[inside], 2 * k[inside] / 32 - 1, atol=1e-12)


def test_adam_constant_gradient_steps_are_lr_sign_at_every_t():
    """With a constant gradient g the moments are m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected step is lr sign(g) at every t
    (eps = 0); a wrong power in a bias correction moves steps 2 and 3."""
    rng = np.random.default_rng(11)
    p = rng.normal(size=64)
    g = rng.normal(size=64)
    m = np.zeros(64)
    v = np.zeros(64)
    p0 = p.copy()
    for t in (1, 2, 3):
        p, m, v = om.adam(p, g, m, v, t, lr=1e-2, eps=0.0)
        assert np.allclose(p, p0 - t * 1e-2 * np.sign(g), rtol=0, atol=1e-14)
        assert np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-13, atol=0)
        assert np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12, atol=0)


def test_adam_second_step_closed_form_with_changing_gradient():
    """Two steps with gradients g1 then g2: m_hat = (b1 g1 + g2)/(1 + b1),
    v_hat = (b2 g1^2 + g2^2)/(1 + b2), and the second update is
    lr m_hat / (sqrt(v_hat) + eps)."""
    rng = np.random.default_rng(12)
    p0 = rng.normal(size=40)
    g1, g2 = rng.normal(size=40), rng.normal(size=40)
    b1, b2, lr, eps = 0.8, 0.95, 3e-3, 1e-7
    p1, m, v = om.adam(p0, g1, np.zeros(40), np.zeros(40), 1, lr=lr, beta1=b1, beta2=b2, eps=eps)
    p2, m, v = om.adam(p1, g2, m, v, 2, lr=lr, beta1=b1, beta2=b2, eps=eps)
    mh = (b1 * g1 + g2) / (1 + b1)
    vh = (b2 * g1 * g1 + g2 * g2) / (1 + b2)
    assert np.allclose(p2, p1 - lr * mh / (np.sqrt(vh) + eps), rtol=0, atol=1e-15)
