"""Pins for the oracle's visibility test (Sec. 3.2.2) and its BVH."""
import numpy as np

import oracle
import workloads


def quad(x0, x1, y0, y1, z):
    V = np.array([[x0, y0, z], [x1, y0, z], [x1, y1, z], [x0, y1, z]], np.float32)
    I = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    return V, I


def test_hand_placed_occluder_and_modes():
    floor = quad(-2, 2, -2, 2, 0.0)
    blocker = quad(-0.25, 0.25, -0.25, 0.25, 1.0)
    sc = oracle.Scene([floor, blocker])
    e = np.array([0.0, 0.0, 2.0])
    # directly below the blocker: hidden; far to the side: visible
    assert sc.visible(e, [0.1, 0.1, 0.0], own_tri=0, own_mesh=0, mode=oracle.OCC_FULL)[0] is False
    assert sc.visible(e, [1.5, 1.5, 0.0], own_tri=0, own_mesh=0, mode=oracle.OCC_FULL)[0] is True
    # blocker belongs to another mesh: ignored in self mode and with no occlusion
    assert sc.visible(e, [0.1, 0.1, 0.0], own_tri=0, own_mesh=0, mode=oracle.OCC_SELF)[0] is True
    assert sc.visible(e, [0.1, 0.1, 0.0], own_tri=0, own_mesh=0, mode=oracle.OCC_NONE)[0] is True
    # a point on the blocker is not hidden by its own triangle
    assert sc.visible(e, [0.1, 0.0, 1.0], own_tri=3, own_mesh=1, mode=oracle.OCC_FULL)[0] is True


def test_segment_end_tolerance():
    """An occluder between 1-eps and the sample does not hide it; one before 1-eps does."""
    eps = 1e-4
    target = quad(-1, 1, -1, 1, 0.0)
    e = np.array([0.0, 0.0, 1.0])
    near = quad(-0.5, 0.5, -0.5, 0.5, 0.5 * eps)       # tau = 1 - eps/2
    far = quad(-0.5, 0.5, -0.5, 0.5, 2.0 * eps)        # tau = 1 - 2 eps
    assert oracle.Scene([target, near]).visible(e, [0.01, 0.02, 0.0], 0, 0, oracle.OCC_FULL, eps)[0] is True
    assert oracle.Scene([target, far]).visible(e, [0.01, 0.02, 0.0], 0, 0, oracle.OCC_FULL, eps)[0] is False


def test_bvh_equals_brute_force_random_soup():
    rng = np.random.default_rng(6)
    centers = rng.uniform(-1, 1, (600, 3))
    V = (centers[:, None, :] + rng.normal(scale=0.12, size=(600, 3, 3))).reshape(-1, 3).astype(np.float32)
    I = np.arange(len(V), dtype=np.int32).reshape(-1, 3)
    sc = oracle.Scene([(V[:900], I[:300]), (V[900:], I[300:] - 900)])
    for _ in range(3000):
        e = rng.uniform(-2, 2, 3)
        x = rng.uniform(-1, 1, 3)
        m = int(rng.integers(0, 2))
        for mode in (oracle.OCC_SELF, oracle.OCC_FULL):
            a = sc.visible(e, x, -1, m, mode, brute=False)
            b = sc.visible(e, x, -1, m, mode, brute=True)
            assert a == b


def test_convex_sphere_visibility_is_front_facing():
    """On a convex polyhedron a surface point is visible from an outside eye exactly when
    the eye lies on the outer side of its face plane (a textbook special case)."""
    w = workloads.tiny_icosphere_scene()
    m = w.meshes[0]
    s = oracle.sample_scene([(m.V, m.I)], w.k, 0)
    sc = oracle.Scene([(m.V, m.I)])
    rng = np.random.default_rng(8)
    ps = rng.integers(0, len(s.tri), 4000)
    pf = rng.integers(0, len(w.fix.eye), 4000)
    vis, frag = sc.pair_visibility(s.pos32, s.tri, s.mesh, w.fix.eye, ps, pf, mode=oracle.OCC_SELF)
    visb, fragb = sc.pair_visibility(s.pos32, s.tri, s.mesh, w.fix.eye, ps, pf, mode=oracle.OCC_SELF, brute=True)
    assert np.array_equal(vis, visb) and np.array_equal(frag, fragb)
    V = m.V.astype(np.float64)
    T = m.I[s.tri[ps]]
    n = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    front = np.einsum("ij,ij->i", w.fix.eye[pf].astype(np.float64) - V[T[:, 0]], n) > 0
    assert np.all(front[~frag] == vis[~frag])
    assert frag.mean() < 0.01
    assert 0.2 < vis.mean() < 0.8


def test_density_bvh_equals_brute_on_tiny_scene():
    w = workloads.tiny_icosphere_scene()
    m = w.meshes[0]
    s = oracle.sample_scene([(m.V, m.I)], w.k, 0)
    sc = oracle.Scene([(m.V, m.I)])
    a = oracle.density(sc, s.pos32, s.tri, s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg, oracle.OCC_SELF)
    b = oracle.density(sc, s.pos32, s.tri, s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg, oracle.OCC_SELF,
                       brute=True)
    assert np.array_equal(a.rho, b.rho) and np.array_equal(a.stats, b.stats)
    # occlusion only ever removes contributions
    c = oracle.density(sc, s.pos32, s.tri, s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg, oracle.OCC_NONE)
    assert np.all(c.rho >= a.rho) and c.rho.sum() > a.rho.sum()
