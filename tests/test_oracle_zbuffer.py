"""Pins for the oracle of the paper's own visibility approximation: the crop of the camera
to the 4-sigma cone (Sec. 3.3.2, Appendix A) and the per-fixation z-buffer test with its
depth tolerance (Sec. 3.2.2)."""
import math

import numpy as np

import oracle
import workloads


def _qmul(a, b):
    return np.array([a[0] * b[0] - a[1:] @ b[1:], *(a[0] * b[1:] + b[0] * a[1:] + np.cross(a[1:], b[1:]))])


def _rotate(v, axis, ang):
    """q v q^-1 written out with quaternion products (independent of the oracle's form)."""
    q = np.array([math.cos(ang / 2), *(math.sin(ang / 2) * np.asarray(axis))])
    qc = q * np.array([1, -1, -1, -1])
    return _qmul(_qmul(q, np.array([0.0, *v])), qc)[1:]


def test_centred_gaze_gives_the_square_around_the_cone():
    for theta in (0.5, 1.0, 3.0):
        for n in (0.01, 0.05, 1.0):
            h = n * 4 * math.tan(math.radians(theta))   # tan(atan(4 sigma)) = 4 sigma
            l, r, b, t = oracle.crop_bounds([0, 0, -1], theta, n)
            assert np.allclose([l, r, b, t], [-h, h, -h, h], rtol=1e-13, atol=0)


def test_oblique_gaze_bounds_follow_the_appendix():
    """Appendix A with the quaternion products written out here: the rectangle is centred
    on E (the gaze's hit) with half-widths sqrt(a^2 cos^2 a + b^2 sin^2 a) and
    sqrt(a^2 sin^2 a + b^2 cos^2 a); it holds B0, B1 and the A point nearer to E.  For
    an oblique gaze E is not the true centre of the cone's ellipse, so the farther A
    point can lie beyond the rectangle (it does for a tilt along one axis): the paper's
    crop cuts a sliver of the cone there (what the comparison with the exact test
    measures)."""
    theta, n = 2.0, 0.1
    phi = math.atan(4 * math.tan(math.radians(theta)))
    for g in ([0.3, 0.1, -1.0], [-0.2, 0.35, -1.0], [0.0, -0.4, -1.0]):
        r = np.array(g) / np.linalg.norm(g)
        l, rr, b, t = oracle.crop_bounds(r, theta, n)
        u1 = np.cross(r, [0, 0, -1.0]); u1 /= np.linalg.norm(u1)
        u2 = np.cross(r, u1); u2 /= np.linalg.norm(u2)
        hit = lambda v: -n / v[2] * v[:2]
        A = [hit(_rotate(r, u1, s * phi)) for s in (-1, 1)]
        B = [hit(_rotate(r, u2, s * phi)) for s in (-1, 1)]
        for axis in (u1, u2):
            assert math.isclose(math.acos(_rotate(r, axis, phi) @ r), phi, rel_tol=1e-10)   # on the cone
        E = hit(r)
        a = np.linalg.norm(A[1] - A[0]) / 2; bb = np.linalg.norm(B[1] - B[0]) / 2
        al = math.acos(E[0] / np.linalg.norm(E))
        hx = math.sqrt(a * a * math.cos(al) ** 2 + bb * bb * math.sin(al) ** 2)
        hy = math.sqrt(a * a * math.sin(al) ** 2 + bb * bb * math.cos(al) ** 2)
        assert np.allclose([l, rr, b, t], [E[0] - hx, E[0] + hx, E[1] - hy, E[1] + hy], rtol=1e-12, atol=1e-18)
        inside = lambda P: l - 1e-15 <= P[0] <= rr + 1e-15 and b - 1e-15 <= P[1] <= t + 1e-15
        assert all(inside(P) for P in B)
        near, far = sorted(A, key=lambda P: np.linalg.norm(P - E))
        assert inside(near)
        if g[0] == 0.0:   # tilt along one axis: no slack from the box's corners
            assert not inside(far) and np.linalg.norm(far - E) > a
        # mirror the gaze in x: the bounds mirror
        l2, r2, b2, t2 = oracle.crop_bounds(r * np.array([-1, 1, 1]), theta, n)
        assert np.allclose([l2, r2, b2, t2], [-rr, -l, b, t], rtol=1e-12, atol=1e-18)


def test_camera_basis_is_right_handed_and_level():
    for h in ([0.3, -0.2, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]):
        x, y, f = oracle.camera_basis(h)
        M = np.stack([x, y, f])
        assert np.allclose(M @ M.T, np.eye(3), atol=1e-15)
        assert np.allclose(np.cross(x, y), -f, atol=1e-15)   # looking along -z of (x, y, z)
        if abs(f[1]) < 0.99:
            assert abs(x[1]) < 1e-15                          # the right vector stays level


def _quad(c, u, v):
    c, u, v = (np.asarray(a, np.float64) for a in (c, u, v))
    V = np.array([c - u - v, c + u - v, c + u + v, c - u + v], np.float32)
    return V, np.array([[0, 1, 2], [0, 2, 3]], np.int32)


def test_zbuffer_of_planes_in_closed_form():
    """A wall facing the eye at distance 3 fills every pixel with depth 3; a tilted wall
    n . p = c gives t = (c - n . e) / (n . d) through each pixel centre."""
    V, I = _quad([0, 0, 3.0], [5, 0, 0], [0, 5, 0])
    sc = oracle.Scene([(V, I)])
    eye = np.zeros((1, 3), np.float32); gaze = np.array([[0, 0, 1.0]], np.float32)
    z = oracle.density_zbuffer(sc, np.zeros((0, 3), np.float32), eye, gaze, np.ones(1, np.float32), 2.0,
                               resolution=16).zbuf[0]
    assert np.allclose(z, 3.0, rtol=1e-13, atol=0)
    nrm = np.array([0.0, 0.6, 0.8])
    V2, I2 = _quad([0, 0, 3.0], [5, 0, 0], 5 * np.array([0.0, 0.8, -0.6]))
    sc2 = oracle.Scene([(V2, I2)])
    out = oracle.density_zbuffer(sc2, np.zeros((0, 3), np.float32), eye, gaze, np.ones(1, np.float32), 2.0,
                                 resolution=8)
    cam = out.cams[0]
    c = nrm @ np.array([0, 0, 3.0])
    sx = 2 * 0.05 / (cam[10] - cam[9]); ox = (cam[10] + cam[9]) / (cam[10] - cam[9])
    sy = 2 * 0.05 / (cam[12] - cam[11]); oy = (cam[12] + cam[11]) / (cam[12] - cam[11])
    for j in range(8):
        for i in range(8):
            nx, ny = -1 + (2 * i + 1) / 8, -1 + (2 * j + 1) / 8
            d = (nx + ox) / sx * cam[:3] + (ny + oy) / sy * cam[3:6] + cam[6:9]
            assert math.isclose(out.zbuf[0, j, i], c / (nrm @ d), rel_tol=1e-12)


def test_occluder_shadow_and_depth_tolerance():
    """A back wall at depth 2 behind a small square at depth 1: samples on the wall behind
    the square fail the depth test, the others pass; eps decides for points set behind
    the surface by a known fraction of their depth."""
    back = _quad([0, 0, 2.0], [3, 0, 0], [0, 3, 0])
    front = _quad([0, 0, 1.0], [0.01, 0, 0], [0, 0.01, 0])
    sc = oracle.Scene([back, front])
    eye = np.zeros((1, 3), np.float32); gaze = np.array([[0, 0, 1.0]], np.float32)
    theta = 1.0
    half = 2.0 * 4 * math.tan(math.radians(theta))      # the frustum's half-width on the wall
    xs = np.linspace(-0.9, 0.9, 13) * half
    pts = np.array([[x, y, 2.0] for x in xs for y in xs], np.float32)
    out = oracle.density_zbuffer(sc, pts, eye, gaze, np.ones(1, np.float32), theta, resolution=64)
    shadow = (np.abs(pts[:, 0]) < 0.02 - 0.002) & (np.abs(pts[:, 1]) < 0.02 - 0.002)
    lit = (np.abs(pts[:, 0]) > 0.02 + 0.002) | (np.abs(pts[:, 1]) > 0.02 + 0.002)
    assert shadow.any() and lit.any()
    assert np.all(out.rho[shadow] == 0) and np.all(out.rho[lit] > 0)
    assert np.all(out.stats[:, 0] == 1)                   # every point lies in the frustum
    # points 0.5 % and 2 % of their depth behind a lit wall point: visible only within eps
    p = np.array([[0.05, 0.05, 2.0 * 1.005], [0.05, 0.05, 2.0 * 1.02]], np.float32)
    solo = oracle.Scene([back])
    r = oracle.density_zbuffer(solo, p, eye, gaze, np.ones(1, np.float32), theta, resolution=64, eps_depth=1e-2)
    assert r.rho[0] > 0 and r.rho[1] == 0


def test_fine_zbuffer_agrees_with_the_exact_test_away_from_the_silhouette():
    """On the tiny scene (a convex sphere of radius 0.5), with a fine z-buffer and a small
    depth tolerance: for fixations whose gaze meets the sphere at an incidence cosine above
    0.5 the z-buffer map equals the exact one within 1 %; where the cone reaches the
    silhouette, grazing surfaces make the depth at a pixel centre differ from the sample's
    by more than eps (or the front surface masks the back one within eps), and the two
    maps part (by up to half of the map here): the approximation this comparison
    measures."""
    w = workloads.tiny_icosphere_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    s = oracle.sample_scene(meshes, w.k, w.seed)
    sc = oracle.Scene(meshes)
    eye = w.fix.eye.astype(np.float64); g = w.fix.gaze.astype(np.float64)
    g /= np.linalg.norm(g, axis=1, keepdims=True)
    b = np.einsum("ij,ij->i", eye, g); c = np.einsum("ij,ij->i", eye, eye) - 0.25
    disc = b * b - c
    t = -b - np.sqrt(np.maximum(disc, 0))
    hit = eye + t[:, None] * g
    cos_inc = np.where(disc > 0, -np.einsum("ij,ij->i", hit / 0.5, g), -1)
    front = np.nonzero(cos_inc > 0.5)[0][:12]
    grazing = np.nonzero((cos_inc > -1) & (cos_inc < 0.4))[0][:6]
    assert len(front) >= 8 and len(grazing) >= 3
    errs = {}
    for name, sel in (("front", front), ("grazing", grazing)):
        ex = oracle.density(sc, s.pos32, s.tri, s.mesh, w.fix.eye[sel], w.fix.gaze[sel], w.fix.dur[sel], w.theta_deg,
                            mode=oracle.OCC_FULL)
        zb = oracle.density_zbuffer(sc, s.pos32, w.fix.eye[sel], w.fix.gaze[sel], w.fix.dur[sel], w.theta_deg,
                                    resolution=256, eps_depth=2e-3)
        errs[name] = np.linalg.norm(zb.rho - ex.rho) / np.linalg.norm(ex.rho)
    assert errs["front"] < 0.01, errs
    assert errs["grazing"] > 5 * errs["front"], errs


def test_crop_refusals_in_closed_form():
    """The two refusals of the crop (a builder rule, not a passage of Appendix A), pinned
    where they have closed forms.  A gaze along the view axis gets the square of half-width
    n 4 sigma, whose corners lie atan(4 sigma sqrt 2) off the gaze: refused from 80 degrees
    on, i.e. from theta = atan(tan 80 / (4 sqrt 2)) = 45.07 deg.  A gaze psi off the view
    axis has a cone edge psi + phi (phi = atan(4 sigma)) off it, which reaches behind the
    camera (no crop at all) once psi + phi >= 90 degrees."""
    cut = math.degrees(math.atan(math.tan(math.radians(80.0)) / (4.0 * math.sqrt(2.0))))
    assert 45.07 < cut < 45.08
    for theta, expect in ((10.0, True), (45.0, True), (45.15, False), (60.0, False)):
        _, ok = oracle.crop_cameras([[0.0, 0.0, -1.0]], None, theta, 0.05)
        assert bool(ok[0]) is expect, theta
    psi = math.radians(60.0)
    gaze = [[math.sin(psi), 0.0, -math.cos(psi)]]
    head = [[0.0, 0.0, -1.0]]
    for phi_deg, behind in ((29.5, False), (30.5, True)):
        theta = math.degrees(math.atan(math.tan(math.radians(phi_deg)) / 4.0))
        rc = [math.sin(psi), 0.0, -math.cos(psi)]   # the gaze in camera coordinates (right = x)
        assert (oracle.crop_bounds(rc, theta, 0.05) is None) is behind, phi_deg
        if behind:
            _, ok = oracle.crop_cameras(gaze, head, theta, 0.05)
            assert not ok[0]
