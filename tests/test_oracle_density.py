"""Pins for the oracle's angular kernel and density (Sec. 3.2.1-3.2.3, Appendix A)."""
import math

import numpy as np
import pytest

import oracle

SQ2PI = math.sqrt(2.0 * math.pi)


def plane_samples(half, n):
    xs = (np.arange(n) + 0.5) / n * 2 * half - half
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    return np.stack([X, Y, np.zeros_like(X)], -1).reshape(-1, 3)


def dens(pos, eye, gaze, dur, theta):
    d = oracle.density(None, np.asarray(pos, np.float32), None, None, np.asarray(eye, np.float32),
                       np.asarray(gaze, np.float32), np.asarray(dur, np.float32), theta, mode=oracle.OCC_NONE)
    return d.rho


@pytest.mark.parametrize("theta", [0.5, 1.0, 2.0])
def test_plane_closed_form(theta):
    """Eye at height h over the plane z = 0 looking straight down: the footprint is an
    isotropic Gaussian of standard deviation h*sigma, cut at radius 4*sigma*h."""
    h, t = 1.25, 0.75
    sigma = math.tan(math.radians(theta))
    rng = np.random.default_rng(0)
    rad = rng.uniform(0, 5 * sigma * h, 2000)
    ang = rng.uniform(0, 2 * np.pi, 2000)
    pos = np.stack([rad * np.cos(ang), rad * np.sin(ang), np.zeros_like(rad)], -1).astype(np.float32)
    rho = dens(pos, [[0, 0, h]], [[0, 0, -2.5]], [t], theta)     # |r| != 1 on purpose
    p64 = pos.astype(np.float64)
    r2 = p64[:, 0] ** 2 + p64[:, 1] ** 2
    want = t / (sigma * SQ2PI) * np.exp(-r2 / (2 * h * h * sigma * sigma))
    inside = np.sqrt(r2) <= 4 * sigma * h * (1 - 1e-9)
    outside = np.sqrt(r2) >= 4 * sigma * h * (1 + 1e-9)
    assert np.all(np.abs(rho[inside] - want[inside]) <= 1e-12 * want[inside])
    assert np.all(rho[outside] == 0.0)
    assert inside.sum() > 1000 and outside.sum() > 100


def test_four_sigma_mass():
    """Integral of the footprint over the plane = t h^2 sigma sqrt(2 pi) (1 - e^-8):
    the 4-sigma cone keeps all but e^-8 of the Gaussian mass (Sec. 3.3.2)."""
    h, t, theta = 2.0, 0.4, 1.0
    sigma = math.tan(math.radians(theta))
    R = 4 * sigma * h
    n = 801
    pos = plane_samples(R * 1.01, n)
    rho = dens(pos, [[0, 0, h]], [[0, 0, -1]], [t], theta)
    cell = (2 * R * 1.01 / n) ** 2
    want = t * h * h * sigma * SQ2PI * (1 - math.exp(-8))
    assert abs(rho.sum() * cell - want) < 2e-4 * want


def test_back_cone_and_side_give_nothing():
    pos = np.array([[0, 0, 5.0], [1.0, 0, 1.0], [0, 0, -3.0]], np.float32)
    rho = dens(pos, [[0, 0, 1.0]], [[0, 0, -1]], [1.0], 1.0)
    assert rho[0] == 0.0         # behind the eye, on the gaze axis
    assert rho[1] == 0.0         # 90 degrees off axis (d = 0)
    assert rho[2] > 0.0


def _quat_rotate(v, axis, ang):
    """Rotation of v by ang about the unit axis with a quaternion q v q^-1 (Appendix A)."""
    w = math.cos(ang / 2); s = math.sin(ang / 2)
    q = np.array([w, *(s * np.asarray(axis))])

    def mul(a, b):
        return np.array([a[0] * b[0] - a[1:] @ b[1:], *(a[0] * b[1:] + b[0] * a[1:] + np.cross(a[1:], b[1:]))])
    qc = q * np.array([1, -1, -1, -1])
    return mul(mul(q, np.array([0.0, *v])), qc)[1:]


def test_oblique_footprint_matches_appendix_construction():
    """Appendix A: rotating the gaze ray by +-phi = atan(4 sigma) about u1 = r x i and
    u2 = r x u1 gives the four points A0, A1, B0, B1 where the 4-sigma cone meets the
    near plane z = -n.  The oracle's gate must switch exactly there."""
    theta, n = 1.0, 2.0
    sigma = math.tan(math.radians(theta))
    phi = math.atan(4 * sigma)
    r = np.array([0.3, 0.1, -1.0]); r /= np.linalg.norm(r)
    i_fwd = np.array([0.0, 0.0, -1.0])
    u1 = np.cross(r, i_fwd); u1 /= np.linalg.norm(u1)
    u2 = np.cross(r, u1); u2 /= np.linalg.norm(u2)

    def on_plane(v):
        return v * (-n / v[2])
    A0 = on_plane(_quat_rotate(r, u1, -phi)); A1 = on_plane(_quat_rotate(r, u1, phi))
    B0 = on_plane(_quat_rotate(r, u2, -phi)); B1 = on_plane(_quat_rotate(r, u2, phi))
    E = on_plane(r)
    pts = []
    for lam in (1e-5, 1 - 1e-5, -1e-5, 1 + 1e-5):
        pts.append(A0 + lam * (A1 - A0))
    for B in (B0, B1):
        pts.append(E + (1 - 1e-5) * (B - E))
        pts.append(E + (1 + 1e-5) * (B - E))
    pts = np.array(pts)
    d = oracle.density(None, pts.astype(np.float32), None, None, np.zeros((1, 3), np.float32),
                       r[None].astype(np.float32), np.ones(1, np.float32), theta, mode=oracle.OCC_NONE)
    got = d.rho > 0
    assert list(got) == [True, True, False, False, True, False, True, False]


def test_linearity_duration_and_gaze_length():
    rng = np.random.default_rng(4)
    pos = rng.uniform(-0.3, 0.3, (500, 3)); pos[:, 2] = 0
    eye = np.stack([rng.uniform(-0.2, 0.2, 40), rng.uniform(-0.2, 0.2, 40), rng.uniform(1, 2, 40)], -1)
    tgt = rng.uniform(-0.2, 0.2, (40, 3)); tgt[:, 2] = 0
    gaze = tgt - eye
    dur = rng.uniform(0.1, 0.5, 40)
    th = 2.0
    full = dens(pos, eye, gaze, dur, th)
    a = dens(pos, eye[:17], gaze[:17], dur[:17], th)
    b = dens(pos, eye[17:], gaze[17:], dur[17:], th)
    assert np.allclose(full, a + b, rtol=1e-12, atol=0)
    assert np.allclose(dens(pos, eye, gaze, 2 * dur.astype(np.float32), th), 2 * full, rtol=1e-12, atol=0)
    assert np.allclose(dens(pos, eye, 4 * gaze.astype(np.float32), dur, th), full, rtol=1e-12, atol=0)
    assert full.max() > 0


def test_rigid_motion_invariance():
    """Axis permutation with sign flips is exact in FP32, so the density is unchanged;
    a translation changes the FP32 inputs by rounding only."""
    rng = np.random.default_rng(5)
    pos = rng.uniform(-0.3, 0.3, (400, 3)).astype(np.float32)
    eye = (rng.uniform(-0.2, 0.2, (30, 3)) + [0, 0, 1.5]).astype(np.float32)
    gaze = (pos[rng.integers(0, 400, 30)] - eye).astype(np.float32)
    dur = np.ones(30, np.float32)
    base = dens(pos, eye, gaze, dur, 2.0)
    P = np.array([[0, 0, -1], [1, 0, 0], [0, -1, 0]], np.float32)
    rot = dens(pos @ P.T, eye @ P.T, gaze @ P.T, dur, 2.0)
    assert np.allclose(rot, base, rtol=1e-12, atol=1e-300)
    sh = np.array([0.375, -1.25, 0.5], np.float32)
    mov = dens(pos + sh, eye + sh, gaze, dur, 2.0)
    ok = np.abs(mov - base) <= 1e-4 * base + 1e-3 * base.max()
    assert ok.mean() > 0.995


def test_hand_computed_single_pair():
    """One sample, one fixation, values worked out in the paper's notation."""
    theta, t = 1.5, 0.3
    e = np.array([0.1, -0.2, 2.0]); x = np.array([0.12, -0.19, 0.0])
    r = np.array([0.0, 0.0, -1.0])
    p = x - e
    d1 = p @ r
    d2 = math.sqrt(p @ p - d1 * d1)
    sig = math.tan(math.radians(theta))
    sig_k = d2 / (d1 * sig) * sig
    g = t / (sig * SQ2PI) * math.exp(-sig_k ** 2 / (2 * sig ** 2))
    inside, gv, _ = oracle.pair_value(x, e, r, t, theta)
    assert inside and abs(gv - g) <= 1e-13 * g
    rho = dens(x[None], e[None], r[None], [t], theta)
    xf = np.float32(x); ef = np.float32(e)
    p = xf.astype(np.float64) - ef.astype(np.float64)
    d2 = math.hypot(p[0], p[1]); d1 = -p[2]
    g32 = t / (sig * SQ2PI) * math.exp(-(d2 / d1) ** 2 / (2 * sig ** 2))
    assert abs(rho[0] - float(np.float32(t)) / t * g32) <= 1e-12 * g32


def test_normalization():
    rho = np.array([0.0, 2.0, 8.0, 4.0])
    out, mx = oracle.normalize(rho)
    assert mx == 8.0 and list(out) == [0.0, 0.25, 1.0, 0.5]
    out, mx = oracle.normalize(np.zeros(5))
    assert mx == 0.0 and np.all(out == 0)
