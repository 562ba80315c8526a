"""Pins for the oracle of moving objects (posed_density): the map of a recording where
every mesh has a pose per fixation is the sum over fixations of the static map of the
scene as it stood at that fixation, with values bound to each object's own frame."""
import math

import numpy as np

import oracle
import workloads


def _small_scene():
    sph = workloads.sphere_mesh(level=2, radius=0.4)
    plate = workloads.plate_mesh(0.8, 4)
    return [(sph.V, sph.I), (plate.V, plate.I)]


def _samples(meshes, k=3000.0):
    return oracle.sample_scene(meshes, k, 5)


def _identity(F, M):
    P = np.zeros((F, M, 12), np.float32)
    P[:, :, 0] = P[:, :, 5] = P[:, :, 10] = 1.0
    return P


def _fixations(F, seed=0, y=-2.0):
    rng = np.random.default_rng(seed)
    eye = np.stack([rng.uniform(-0.5, 0.5, F), np.full(F, y), rng.uniform(-0.5, 0.5, F)], 1)
    tgt = np.stack([rng.uniform(-0.3, 0.3, F), np.zeros(F), rng.uniform(-0.3, 0.3, F)], 1)
    return eye.astype(np.float32), (tgt - eye).astype(np.float32), rng.uniform(0.1, 0.5, F).astype(np.float32)


def test_identity_poses_give_the_static_map():
    meshes = _small_scene()
    # the plate stands between the eyes and the sphere: lift it into the x-z plane
    V, I = meshes[1]
    meshes[1] = (np.ascontiguousarray(V[:, [0, 2, 1]] + np.array([0, -0.6, 0], np.float32)), I)
    s = _samples(meshes)
    eye, gaze, dur = _fixations(12)
    sc = oracle.Scene(meshes)
    for mode in (oracle.OCC_NONE, oracle.OCC_SELF, oracle.OCC_FULL):
        a = oracle.posed_density(meshes, s.pos32, s.tri, s.mesh, eye, gaze, dur, _identity(12, 2), 1.0, mode)
        b = oracle.density(sc, s.pos32, s.tri, s.mesh, eye, gaze, dur, 1.0, mode=mode)
        assert np.array_equal(a.rho, b.rho) and np.array_equal(a.budget, b.budget)
        assert np.array_equal(a.stats, b.stats)
    assert b.stats[:, 1].sum() < b.stats[:, 0].sum()   # the plate occludes in mode full


def test_quarter_turn_of_everything_changes_nothing():
    """Rotate every mesh by a quarter turn about z and the fixations with it (exact in
    FP32): the fixation seen from each mesh is bit-for-bit the unrotated one."""
    meshes = _small_scene()
    s = _samples(meshes)
    eye, gaze, dur = _fixations(10, seed=3)
    F = len(eye)
    P = np.zeros((F, 2, 12), np.float32)
    P[:, :, 1] = -1.0; P[:, :, 4] = 1.0; P[:, :, 10] = 1.0     # (x, y, z) -> (-y, x, z)
    rot = lambda v: np.stack([-v[:, 1], v[:, 0], v[:, 2]], 1).astype(np.float32)
    a = oracle.posed_density(meshes, s.pos32, s.tri, s.mesh, rot(eye), rot(gaze), dur, P, 1.0, oracle.OCC_SELF)
    b = oracle.density(oracle.Scene(meshes), s.pos32, s.tri, s.mesh, eye, gaze, dur, 1.0, mode=oracle.OCC_SELF)
    assert np.array_equal(a.rho, b.rho)
    for k in range(F):
        el, rl, ok = oracle.local_fixation(P[k, 0], rot(eye)[k:k + 1][0], rot(gaze)[k:k + 1][0])
        assert ok and np.array_equal(el, eye[k]) and np.array_equal(rl, gaze[k])
    # with inter-object occlusion the world test runs on rotated coordinates: equal up to
    # the fragile pairs that both sides count in their budgets
    a = oracle.posed_density(meshes, s.pos32, s.tri, s.mesh, rot(eye), rot(gaze), dur, P, 1.0, oracle.OCC_FULL)
    b = oracle.density(oracle.Scene(meshes), s.pos32, s.tri, s.mesh, eye, gaze, dur, 1.0, mode=oracle.OCC_FULL)
    assert np.all(np.abs(a.rho - b.rho) <= a.budget + b.budget + 1e-12 * b.rho)


def test_mesh_carried_with_its_eye_repeats_one_fixation():
    """A sphere translated by (0.25 f, 0, 0) at fixation f, watched from an eye carried
    along with it: every fixation sees the same thing, so rho = F x the map of one."""
    sph = workloads.sphere_mesh(level=2, radius=0.4)
    meshes = [(sph.V, sph.I)]
    s = _samples(meshes, 4000.0)
    F = 8
    e0 = np.array([0.5, -2.0, 0.25], np.float32); r0 = np.array([-0.5, 2.0, -0.25], np.float32)
    P = _identity(F, 1)
    P[:, 0, 3] = 0.25 * np.arange(F)
    eye = np.stack([e0 + np.array([0.25 * f, 0, 0], np.float32) for f in range(F)]).astype(np.float32)
    gaze = np.tile(r0, (F, 1)); dur = np.ones(F, np.float32)
    a = oracle.posed_density(meshes, s.pos32, s.tri, s.mesh, eye, gaze, dur, P, 1.0, oracle.OCC_SELF)
    one = oracle.density(oracle.Scene(meshes), s.pos32, s.tri, s.mesh, e0[None], r0[None], dur[:1], 1.0,
                         mode=oracle.OCC_SELF)
    assert one.rho.max() > 0
    assert np.max(np.abs(a.rho - F * one.rho)) <= 1e-12 * F * one.rho.max()
    # a static scene would have smeared the same fixations over the sphere
    static = oracle.density(oracle.Scene(meshes), s.pos32, s.tri, s.mesh, eye, gaze, dur, 1.0, mode=oracle.OCC_SELF)
    assert np.abs(static.rho - a.rho).max() > 0.1 * a.rho.max()


def test_moving_occluder_is_the_sum_of_static_instants():
    """A plate slides in front of a sphere and away again: the posed map equals the sum
    over fixations of the static map of the scene as it stood at that fixation (the
    points placed in the world, within the FP32 rounding of the placed points)."""
    meshes = _small_scene()
    s = _samples(meshes)
    F = 6
    eye = np.tile(np.array([[0.0, -2.0, 0.05]], np.float32), (F, 1))
    gaze = np.tile(np.array([[0.0, 1.0, 0.0]], np.float32), (F, 1))
    dur = np.full(F, 0.25, np.float32)
    P = _identity(F, 2)
    # plate: local x-y plane turned to face -y, at y = -0.75, x offsets from 0 to 2.5 m
    for f in range(F):
        P[f, 1] = [1, 0, 0, 0.5 * f, 0, 0, -1, -0.75, 0, 1, 0, 0]
    a = oracle.posed_density(meshes, s.pos32, s.tri, s.mesh, eye, gaze, dur, P, 1.0, oracle.OCC_FULL)
    total = np.zeros(len(s.pos32)); bud = np.zeros(len(s.pos32))
    for f in range(F):
        world = [(oracle.posed_world(V, P[f, m]), I) for m, (V, I) in enumerate(meshes)]
        xw = np.zeros_like(s.pos32)
        for m in range(2):
            sel = s.mesh == m
            xw[sel] = oracle.posed_world(s.pos32[sel], P[f, m])
        r = oracle.density(oracle.Scene(world), xw, s.tri, s.mesh, eye[f:f + 1], gaze[f:f + 1], dur[f:f + 1], 1.0,
                           mode=oracle.OCC_FULL)
        total += r.rho; bud += r.budget
    assert np.all(np.abs(a.rho - total) <= 1e-4 * total + a.budget + bud + 1e-12)
    sphere = s.mesh == 0
    blocked = oracle.posed_density(meshes, s.pos32, s.tri, s.mesh, eye[:1], gaze[:1], dur[:1], P[:1], 1.0,
                                   oracle.OCC_FULL).rho[sphere].sum()
    clear = oracle.posed_density(meshes, s.pos32, s.tri, s.mesh, eye[-1:], gaze[-1:], dur[-1:], P[-1:], 1.0,
                                 oracle.OCC_FULL).rho[sphere].sum()
    assert blocked == 0.0 and clear > 0.0


def test_shears_and_invalid_fixations_are_refused():
    P = np.array([1, 0.01, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)   # shear
    assert not oracle.local_fixation(P, [0, 0, 0], [0, 0, 1])[2]
    c, s_ = math.cos(0.3), math.sin(0.3)
    R = np.array([2 * c, -2 * s_, 0, 1, 2 * s_, 2 * c, 0, 2, 0, 0, 2, 3], np.float32)  # rotation x 2 + move
    el, rl, ok = oracle.local_fixation(R, [1, 2, 5], [0, 0, 1])
    assert ok and np.allclose(el, [0, 0, 1], atol=1e-6) and np.allclose(rl, [0, 0, 0.5], atol=1e-7)
    meshes = _small_scene()
    s = _samples(meshes)
    eye, gaze, dur = _fixations(3)
    pose = _identity(3, 2)
    pose[1, 1, 1] = 0.2   # fixation 1: a shear on the plate
    a = oracle.posed_density(meshes, s.pos32, s.tri, s.mesh, eye, gaze, dur, pose, 1.0, oracle.OCC_SELF)
    keep = np.array([True, False, True])
    b = oracle.density(oracle.Scene(meshes), s.pos32, s.tri, s.mesh, eye[keep], gaze[keep], dur[keep], 1.0,
                       mode=oracle.OCC_SELF)
    assert np.max(np.abs(a.rho - b.rho)) <= 1e-12 * max(1e-300, b.rho.max())
