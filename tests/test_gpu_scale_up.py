"""Scale-up workload (25 displaced geodesic spheres on a 5 x 5 grid, 5M triangles, 20M
samples, 50,000 fixations from 10 head trajectories, theta 1 deg, full occlusion) in the
launch configuration of the benchmark: per-mesh sample counts against the oracle's exact
integer rule, and the density of sampled points (plus the densest ones) against the FP64
oracle recomputing them one by one."""
import time

import numpy as np
import pytest

import oracle
import parity_util
import workloads

pytestmark = pytest.mark.gpu


def test_scale_up_sampled_parity():
    import torch
    import paper_2601_07571_amd as gm
    gm.load_library()
    w = workloads.scale_up_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    scene = gm.Scene(meshes)
    counts = scene.count_samples(w.k)
    for m, (V, I) in enumerate(meshes[:3]):
        A = oracle.triangle_areas(V, I)
        _, _, S, Wm = oracle.mesh_weights(A)
        assert counts[m] == oracle.sample_count(Wm, S, w.k)
    s = scene.build_samples(w.k, w.seed)
    N = int(s.pos.shape[0])
    assert abs(N - 20_000_000) < 0.02 * 20_000_000   # k comes from the nominal sphere area
    fix = gm.Fixations(w.fix.eye, w.fix.gaze, w.fix.dur)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = scene.accumulate(s.pos, fix, w.theta_deg, occlusion="full", tri=s.tri, mesh=s.mesh)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = scene.density_stats()
    print(f"scale-up map: {dt * 1e3:.0f} ms, {N * len(w.fix.eye) / dt:.3e} pairs/s, "
          f"{st['in_cone'] / dt:.3e} rays/s, in-cone {st['in_cone']}, visible {st['visible']}")
    d = out.density.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(7)
    # plus the three samples that an FP32 segment test from the eye once saw edge-on the
    # wrong way (golden/grazing_pairs.json)
    grazing = [11090699, 12686781, 18763059]
    pick = np.unique(np.concatenate([rng.choice(N, 6000, replace=False), np.argsort(d)[-10:], grazing]))
    pos = s.pos.cpu().numpy()[pick]; tri = s.tri.cpu().numpy()[pick]; mesh = s.mesh.cpu().numpy()[pick]
    sc = oracle.Scene(meshes)
    ref = oracle.density(sc, pos, tri, mesh, w.fix.eye, w.fix.gaze, w.fix.dur, w.theta_deg, mode=oracle.OCC_FULL)
    flips, in_cone, explained = parity_util.check(gm, scene, meshes, pos, tri, mesh, w.fix.eye, w.fix.gaze,
                                                  w.fix.dur, w.theta_deg, oracle.OCC_FULL, d[pick], ref)
    print(f"checked {len(pick)} samples, {in_cone} in-cone pairs, {flips} visibility flips, "
          f"{explained} samples explained by them")
    firm, fragile, pairs = parity_util.count_flips(scene, meshes, pos, tri, mesh, w.fix.eye, w.fix.gaze, w.fix.dur,
                                                   w.theta_deg, oracle.OCC_FULL)
    print(f"visibility of all {pairs} in-cone pairs: {firm} disagreements outside the oracle's fragile set, "
          f"{fragile} inside it")
    assert firm == 0
    assert (ref.rho > 0).mean() > 0.05
    assert out.density_norm.cpu().numpy().max() == 1.0
