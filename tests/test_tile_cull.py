"""The density kernel skips, for a whole tile, every fixation whose gate cone cannot reach
the tile's bounding sphere.  This checks that test on the CPU, in FP32 as the kernel
evaluates it, against brute force in FP64: every point of the sphere that lies inside the
gate cone (angle to the gaze below psi_g, cos^2 psi_g = kappa / |r|^2) must belong to a
kept (tile, fixation) pair.  Cones and spheres are drawn near the boundary on purpose."""
import numpy as np


def tile_keeps(o, rad2, e, r, kappa):
    """The kernel's staging test in float32: o tile origin, rad2 largest squared distance
    of a tile sample to o, e eye, r gaze, kappa gate constant."""
    f = np.float32
    rad_t = f(np.sqrt(f(rad2))) * f(1.001) + f(1e-6)
    ex, ey, ez = (f(e[i]) - f(o[i]) for i in range(3))
    e2 = ex * ex + (ey * ey + ez * ez)
    rx, ry, rz = (f(v) for v in r)
    c0 = -(rx * ex + (ry * ey + rz * ez))
    near2 = f(4.0) * f(rad2) + f(1e-12)
    if e2 <= near2:
        return True
    rr = rx * rx + (ry * ry + rz * rz)
    cg2 = min(f(kappa) / rr, f(1.0))
    cg, sg = np.sqrt(cg2), np.sqrt(f(1.0) - cg2)
    sd = min(rad_t / np.sqrt(e2), f(1.0))
    cd = np.sqrt(max(f(1.0) - sd * sd, f(0.0)))
    cA, sA = cg * cd - sg * sd, sg * cd + cg * sd
    cT = f(-1e-4) * sA + cA
    return (not cT > 0) or (c0 > 0 and c0 * c0 > cT * cT * rr * e2)


def test_tile_cull_keeps_every_reachable_fixation():
    rng = np.random.default_rng(11)
    sigma = np.tan(np.radians(1.0))
    kscale = 1.0 / (1.0 + 16 * sigma * sigma) * (1 - 1e-6)
    kept_cases = skipped_cases = 0
    for _ in range(3000):
        o = rng.uniform(-2, 2, 3)
        R = 10 ** rng.uniform(-3, -0.5)
        dist = 10 ** rng.uniform(-0.5, 1.0)
        u = rng.normal(size=3); u /= np.linalg.norm(u)
        e = o - dist * u                       # eye at dist from the tile, looking roughly at it
        psi = np.arccos(np.sqrt(kscale))
        delta = np.arcsin(min(1.0, R / dist))
        # gaze at an angle near psi + delta from the eye-to-origin direction
        ang = psi + delta + rng.uniform(-3e-3, 3e-3)
        w = np.cross(u, rng.normal(size=3)); w /= np.linalg.norm(w)
        r = np.cos(ang) * u + np.sin(ang) * w
        r *= 10 ** rng.uniform(-0.5, 0.5)
        kappa = float(np.dot(r, r) * kscale)
        keep = tile_keeps(o, R * R, e, r, kappa)
        # brute force: points of the sphere closest in angle to the gaze
        pts = o + R * np.sqrt(rng.uniform(0, 1, (4000, 1))) ** (1 / 3) * (
            lambda v: v / np.linalg.norm(v, axis=1, keepdims=True))(rng.normal(size=(4000, 3)))
        toward = o - R * w * np.sign(np.dot(r, w) + 1e-30)  # the sphere's point towards the gaze
        pts = np.vstack([pts, toward, o + R * (r / np.linalg.norm(r))])
        pts = o + (pts - o) * np.minimum(1.0, R / np.maximum(np.linalg.norm(pts - o, axis=1, keepdims=True), 1e-300))
        v = pts - e
        rv = v @ r
        inside = (rv > 0) & (rv * rv > kappa * np.einsum("ij,ij->i", v, v))
        if inside.any():
            assert keep, (o, R, e, r)
        # and in FP64 geometry: the smallest angle between the gaze and a ray from the eye
        # into the ball is angle(r, o - e) - asin(R / |o - e|)
        c = o - e
        phi_c = np.arccos(np.clip(np.dot(r, c) / (np.linalg.norm(r) * np.linalg.norm(c)), -1, 1))
        if phi_c - np.arcsin(min(1.0, R / np.linalg.norm(c))) < psi:
            assert keep, (o, R, e, r)
        kept_cases += keep
        skipped_cases += not keep
    assert kept_cases > 300 and skipped_cases > 300   # both outcomes occur near the boundary
