"""Pins for the oracle's time-window selection (the analysis interval of Sec. 3.3.4):
density over a window is the Sec. 3.2.1 sum over the fixations that start inside it."""
import numpy as np

import oracle
import workloads


def _tiny():
    w = workloads.tiny_icosphere_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    s = oracle.sample_scene(meshes, w.k, w.seed)
    return w, meshes, s


def test_back_to_back_windows_partition_the_recording():
    """rho is linear in the fixations, so windows [a, b) and [b, c) add up to [a, c).  One
    fixation starts exactly at b: a closed window on both ends would count it twice, an
    open one not at all."""
    w, meshes, s = _tiny()
    sc = oracle.Scene(meshes)
    t = workloads.start_times(w.fix.dur)
    b = float(t[40])
    args = (sc, s.pos32, s.tri, s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur, t)
    lo = oracle.density_window(*args, (0.0, b), w.theta_deg, mode=oracle.OCC_SELF).rho
    hi = oracle.density_window(*args, (b, np.inf), w.theta_deg, mode=oracle.OCC_SELF).rho
    full = oracle.density(sc, s.pos32, s.tri, s.mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                          mode=oracle.OCC_SELF).rho
    assert np.max(np.abs(lo + hi - full)) <= 1e-12 * np.max(full)
    # the fixation at t = b belongs to the upper window only
    only_b = oracle.density(sc, s.pos32, s.tri, s.mesh, w.fix.eye[40:41], w.fix.gaze[40:41], w.fix.dur[40:41],
                            w.theta_deg, mode=oracle.OCC_SELF).rho
    assert only_b.max() > 0
    first = oracle.density_window(*args, (0.0, float(t[41])), w.theta_deg, mode=oracle.OCC_SELF).rho
    assert np.max(np.abs(first - lo - only_b)) <= 1e-12 * np.max(full)
    assert oracle.in_window(t, 0.0, b).sum() == 40


def test_window_edges_and_nan():
    t = np.array([0.0, 1.0, 2.0, np.nan, 3.0])
    assert list(oracle.in_window(t, 1.0, 3.0)) == [False, True, True, False, False]
    assert not oracle.in_window(t, -np.inf, np.inf)[3]
    assert oracle.in_window(t, 2.0, 2.0).sum() == 0


def test_empty_window_is_zero_and_full_window_is_everything():
    w, meshes, s = _tiny()
    t = workloads.start_times(w.fix.dur)
    r = oracle.density_window(None, s.pos32, None, None, w.fix.eye, w.fix.gaze, w.fix.dur, t, (1e9, 2e9),
                              w.theta_deg, mode=oracle.OCC_NONE)
    assert not r.rho.any()
    a = oracle.density_window(None, s.pos32, None, None, w.fix.eye, w.fix.gaze, w.fix.dur, t, (-np.inf, np.inf),
                              w.theta_deg, mode=oracle.OCC_NONE).rho
    b = oracle.density(None, s.pos32, None, None, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg,
                       mode=oracle.OCC_NONE).rho
    assert np.array_equal(a, b)


def test_start_times_follow_the_recording():
    d = np.array([0.2, 0.3, 0.1], np.float32)
    t = workloads.start_times(d, gap=0.05)
    assert np.allclose(t, [0.0, 0.25, 0.6])
