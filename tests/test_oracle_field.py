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


def test_adam_constant_gradient_moves_by_signed_learning_rate_every_step():
    """With a constant gradient g, the bias-corrected moments equal g and g^2 after every
    step n (m_n = (1 - b1^n) g, v_n = (1 - b2^n) g^2), so each update is lr g / (|g| + eps)
    and n updates move the parameters by n lr g / (|g| + eps).  Moments dropped between
    steps, or a bias correction taken at the wrong step, break it from step 2 on."""
    g = np.array([0.5, -2.0, 3e-4, -7.0])
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    p, m, v = np.full(4, 0.25), np.zeros(4), np.zeros(4)
    for n in range(1, 11):
        p, m, v = fo.adam_step(p, m, v, g, n, lr=lr, b1=b1, b2=b2, eps=eps)
        assert np.allclose(m, (1 - b1 ** n) * g, rtol=1e-12)
        assert np.allclose(v, (1 - b2 ** n) * g * g, rtol=1e-12)
        assert np.allclose(p, 0.25 - n * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-15)


def test_adam_two_steps_with_changing_gradients_by_hand():
    """Two updates with gradients g1 then g2, worked out by hand: the first moves by
    lr g1 / (|g1| + eps); the second uses m^ = (b1 g1 + g2) / (1 + b1) and
    v^ = (b2 g1^2 + g2^2) / (1 + b2) (the moments carried over, corrected with step 2)."""
    lr, b1, b2, eps = 0.05, 0.8, 0.95, 1e-6
    g1 = np.array([1.0, -0.5, 2.0, 0.0])
    g2 = np.array([-3.0, -0.5, 0.25, 1.0])
    p0 = np.array([0.1, -0.2, 0.3, 0.4])
    p1, m1, v1 = fo.adam_step(p0, np.zeros(4), np.zeros(4), g1, 1, lr=lr, b1=b1, b2=b2, eps=eps)
    p2, m2, v2 = fo.adam_step(p1, m1, v1, g2, 2, lr=lr, b1=b1, b2=b2, eps=eps)
    e1 = p0 - lr * g1 / (np.abs(g1) + eps)
    mh = (b1 * g1 + g2) / (1 + b1)
    vh = (b2 * g1 ** 2 + g2 ** 2) / (1 + b2)
    e2 = e1 - lr * mh / (np.sqrt(vh) + eps)
    assert np.allclose(p1, e1, rtol=1e-13, atol=1e-16)
    assert np.allclose(p2, e2, rtol=1e-13, atol=1e-16)
    # the second component: equal gradients, so the second step is the first one again
    assert np.isclose(p2[1] - p1[1], p1[1] - p0[1], rtol=1e-12)


def test_bf16_network_is_close_to_fp64_network():
    rng = np.random.default_rng(2)
    flat = fo.init_params(4)
    x = rng.uniform(0, 1, (200, 3))
    y64, _ = fo.forward(flat, x, np.zeros(3), 1.0, bf=False)
    y16, _ = fo.forward(flat, x, np.zeros(3), 1.0, bf=True)
    assert np.max(np.abs(y16 - y64)) < 0.1 * np.max(np.abs(y64)) + 1e-3
