"""Writes grazing_pairs.json: three (sample, fixation) pairs of the scale-up workload
(25 displaced geodesic spheres, 50,000 fixations) whose eye sees the sample almost
edge-on, with the triangles within 2 cm of the sample and the oracle's verdict on the
whole scene.  Every value comes from workloads/ (inputs) and oracle/ (samples,
visibility); run from the repository root: python tests/golden/make_grazing_pairs.py"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

PAIRS = [(11090699, 27464), (12686781, 29551), (18763059, 35618)]
RADIUS = 0.02


def f32hex(a):
    return [format(int(v), "08x") for v in np.asarray(a, np.float32).reshape(-1).view(np.uint32)]


def main():
    w = workloads.scale_up_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    sc = oracle.Scene(meshes)
    cases = []
    for s, f in PAIRS:
        x, tri, mesh = oracle.sample_at(meshes, w.k, w.seed, s)
        e, r = w.fix.eye[f], w.fix.gaze[f]
        vis, frag = sc.pair_visibility(x[None], np.array([tri]), np.array([mesh]), e[None], np.array([0]),
                                       np.array([0]), mode=oracle.OCC_FULL)
        # the patch: triangles with a vertex within RADIUS of the sample
        V = sc.V[sc.I]                                             # [T][3][3]
        near = np.where((np.linalg.norm(V - x[None, None], axis=2) < RADIUS).any(1))[0]
        assert tri in near
        cases.append({"sample": s, "fixation": f, "eye": f32hex(e), "gaze": f32hex(r), "point": f32hex(x),
                      "own": int(np.where(near == tri)[0][0]), "mesh_of_own": int(mesh),
                      "triangles": [f32hex(V[t]) for t in near], "tri_mesh": [int(sc.tri_mesh[t]) for t in near],
                      "scene_triangle": [int(t) for t in near],
                      "oracle_visible": bool(vis[0]), "oracle_fragile": bool(frag[0])})
    out = {"workload": w.name, "theta_deg": w.theta_deg, "eps_v": oracle.EPS_V, "cases": cases}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "grazing_pairs.json"), "w") as fp:
        json.dump(out, fp, indent=1)


if __name__ == "__main__":
    main()
