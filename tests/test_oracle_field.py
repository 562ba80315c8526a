"""Pins of the neural-field oracle (no GPU)."""
import math

import numpy as np

from oracle import field as fo


def test_parameter_count():
    assert fo.N_PARAMS == 96 * 64 + 64 + 3 * (64 * 64 + 64) + 64 + 1 == 18753


def test_feature_closed_forms():
    lo = np.zeros(3); ext = 2.0
    x = np.array([[0.0, 0.0, 0.0], [0.5, 1.0, 1.5]])
    phi = fo.features(x, lo, ext, bf=False)
    # origin: every sine 0, every cosine 1
    assert np.allclose(phi[0, 0::2], 0.0) and np.allclose(phi[0, 1::2], 1.0)
    # band 0 (frequency 1): x~ = (0.25, 0.5, 0.75) -> sin(2 pi x~) = (1, 0, -1)
    assert np.allclose(phi[1, [0, 2, 4]], [1.0, 0.0, -1.0], atol=1e-15)
    assert np.allclose(phi[1, [1, 3, 5]], [0.0, -1.0, 0.0], atol=1e-15)
    # geometric ladder from 1 to max_cycles: with 32, band 3 has frequency 32^(1/5) = 2
    assert math.isclose(fo.freqs()[3], 2.0, rel_tol=1e-6) and math.isclose(fo.freqs()[15], 32.0)
    assert math.isclose(fo.freqs(2.0 ** 15)[5], 32.0, rel_tol=1e-6)
    assert np.allclose(phi[:, 0::2] ** 2 + phi[:, 1::2] ** 2, 1.0)


def test_bf16_rounding():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 3.14159265, -2.5e-3])
    r = fo.bf16(v)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # tie to even
    assert r[2] == 1.0 + 4 * 2 ** -8         # tie to even (odd below)
    assert abs(r[3] - 3.140625) < 1e-12
    assert np.all(np.abs(r - v) <= np.abs(v) * 2 ** -8)


def test_softplus_and_gradient_closed_form():
    """A network whose only non-zero parameter is b5: y = softplus(b5) everywhere, the
    loss gradient is 2 (y - t) sigmoid(b5) averaged, every other gradient is 0."""
    flat = np.zeros(fo.N_PARAMS); flat[-1] = 0.3
    x = np.random.default_rng(0).uniform(0, 1, (7, 3))
    t = np.linspace(0, 1, 7)
    loss, g, y = fo.loss_and_grad(flat, x, t, np.zeros(3), 1.0, bf=False)
    sp = math.log1p(math.exp(0.3)); sg = 1 / (1 + math.exp(-0.3))
    assert np.allclose(y, sp)
    assert math.isclose(loss, np.mean((sp - t) ** 2))
    assert math.isclose(g[-1], np.mean(2 * (sp - t)) * sg, rel_tol=1e-12)
    assert np.all(g[:-1] == 0)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    flat = fo.init_params(3) + rng.normal(scale=0.01, size=fo.N_PARAMS)
    x = rng.uniform(-1, 1, (40, 3))
    t = rng.uniform(0, 1, 40)
    lo, ext = np.full(3, -1.0), 2.0
    loss, g, _ = fo.loss_and_grad(flat, x, t, lo, ext, bf=False)
    idx = rng.choice(fo.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [fo.N_PARAMS - 1, fo.N_PARAMS - 2, 96 * 64 + 3]])
    for i in idx:
        h = 1e-6 * max(1.0, abs(flat[i]))
        fp = flat.copy(); fp[i] += h
        fm = flat.copy(); fm[i] -= h
        num = (fo.loss_and_grad(fp, x, t, lo, ext, bf=False)[0] - fo.loss_and_grad(fm, x, t, lo, ext, bf=False)[0]) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, num, g[i])


def test_adam_first_step_is_signed_learning_rate():
    """After one step from zero moments the bias-corrected update is lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p, m, v = fo.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, 1, lr=0.01, eps=1e-8)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_network_is_close_to_fp64_network():
    rng = np.random.default_rng(2)
    flat = fo.init_params(4)
    x = rng.uniform(0, 1, (200, 3))
    y64, _ = fo.forward(flat, x, np.zeros(3), 1.0, bf=False)
    y16, _ = fo.forward(flat, x, np.zeros(3), 1.0, bf=True)
    assert np.max(np.abs(y16 - y64)) < 0.1 * np.max(np.abs(y64)) + 1e-3
