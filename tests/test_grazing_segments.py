"""Segments that graze the triangles next to their sample point (no GPU).

Three pairs of the scale-up workload, kept in golden/grazing_pairs.json with the
triangles within 2 cm of the sample (written by golden/make_grazing_pairs.py from the
workload generator and the oracle), see their sample almost edge-on (incidence cosines
of 1e-5 to 1e-4): the segment runs within a fraction of a millimetre of the surface and
crosses, or just misses, a neighbouring triangle 1-3 mm from the point, at incidence
cosines of 2e-4 to 8e-3.  An FP32 watertight test with vertices taken relative to the
eye (2.5-8.6 m away) carries ~1e-7 of that distance in every sheared coordinate, which
the grazing incidence turns into errors of order one in the edge functions: it gives
the other answer on all three.  Taken relative to the sample point, the vertices keep
the precision of their millimetre offsets and the same FP32 test agrees with the
oracle.  The density kernel takes its segments from the point for this reason.

The FP32 model below follows the kernel's segment test operation by operation (shear
axis from the gaze, FMA where the kernel fuses, FP64 re-evaluation of zero edge
functions); the GPU check of the same pairs is in test_gpu_density.py."""
import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
F32 = np.float32


def load_cases():
    d = json.load(open(os.path.join(HERE, "golden", "grazing_pairs.json")))
    out = []
    for c in d["cases"]:
        h = lambda v: np.array([int(x, 16) for x in v], np.uint32).view(np.float32)  # noqa: E731
        out.append(dict(c, eye=h(c["eye"]), gaze=h(c["gaze"]), point=h(c["point"]),
                        tris=np.stack([h(t).reshape(3, 3) for t in c["triangles"]])))
    return d, out


def fma(a, b, c):
    return F32(np.float64(a) * np.float64(b) + np.float64(c))


def shear_axes(gaze, d):
    g = np.abs(gaze)
    gz = (0 if g[0] > g[2] else 2) if g[0] > g[1] else (1 if g[1] > g[2] else 2)
    dk = d[gz]
    if not (F32(dk * dk) >= F32(F32(0.16) * F32(F32(F32(d[0] * d[0]) + F32(d[1] * d[1])) + F32(d[2] * d[2])))):
        a = np.abs(d)
        gz = (0 if a[0] > a[2] else 2) if a[0] > a[1] else (1 if a[1] > a[2] else 2)
    kx = 0 if gz == 2 else gz + 1
    ky = 0 if kx == 2 else kx + 1
    return kx, ky, gz


def segment_hits(start, end, tri, gaze, t_lo, t_hi):
    """FP32 model of the kernel's watertight test of the segment start + t (end - start)
    against one triangle: hit iff t_lo < t < t_hi."""
    start = start.astype(F32); end = end.astype(F32)
    d = (end - start).astype(F32)
    kx, ky, kz = shear_axes(gaze, d)
    sx = F32(d[kx] / d[kz]); sy = F32(d[ky] / d[kz]); tz = d[kz]
    A, B, C = ((v.astype(F32) - start).astype(F32) for v in tri)
    Ax, Ay = fma(-sx, A[kz], A[kx]), fma(-sy, A[kz], A[ky])
    Bx, By = fma(-sx, B[kz], B[kx]), fma(-sy, B[kz], B[ky])
    Cx, Cy = fma(-sx, C[kz], C[kx]), fma(-sy, C[kz], C[ky])
    U = F32(F32(Cx * By) - F32(Cy * Bx))
    V = F32(F32(Ax * Cy) - F32(Ay * Cx))
    W = F32(F32(Bx * Ay) - F32(By * Ax))
    if min(abs(U), abs(V), abs(W)) == 0:
        f = np.float64
        U = F32(f(Cx) * f(By) - f(Cy) * f(Bx)); V = F32(f(Ax) * f(Cy) - f(Ay) * f(Cx))
        W = F32(f(Bx) * f(Ay) - f(By) * f(Ax))
    if min(U, V, W) < 0 and max(U, V, W) > 0:
        return False
    det = F32(F32(U + V) + W)
    if det == 0:
        return False
    T = fma(W, C[kz], fma(V, B[kz], F32(U * A[kz])))
    Ts = -T if (det < 0) != (tz < 0) else T
    lim = F32(abs(tz) * abs(det))
    return bool(Ts > F32(F32(t_lo) * lim) and Ts < F32(F32(t_hi) * lim))


def occluded(c, from_point, eps):
    hits = 0
    for j, tri in enumerate(c["tris"]):
        if j == c["own"]:
            continue
        if from_point:   # the kernel: point (t = 0) to eye (t = 1), occluders at eps < t < 1
            hits += segment_hits(c["point"], c["eye"], tri, c["gaze"], F32(eps), F32(1.0))
        else:            # eye (tau = 0) to point (tau = 1), occluders at 0 < tau < 1 - eps
            hits += segment_hits(c["eye"], c["point"], tri, c["gaze"], F32(0.0), F32(1.0 - eps))
    return hits > 0


def test_patch_keeps_the_whole_scene_verdict():
    """The oracle on the 2 cm patch alone gives the verdict it gave on the whole scene
    (the deciding triangles are near the point), and none of the three is fragile."""
    d, cases = load_cases()
    for c in cases:
        V = c["tris"].reshape(-1, 3)
        I = np.arange(len(V), dtype=np.int32).reshape(-1, 3)
        sc = oracle.Scene([(V, I)])
        vis, frag = sc.visible(c["eye"], c["point"], own_tri=c["own"], own_mesh=0, mode=oracle.OCC_FULL)
        assert vis == c["oracle_visible"] and not frag and not c["oracle_fragile"], c["sample"]
    assert [c["oracle_visible"] for c in cases] == [False, True, True]


def test_fp32_from_the_eye_flips_and_from_the_point_agrees():
    d, cases = load_cases()
    eps = d["eps_v"]
    for c in cases:
        truth = not c["oracle_visible"]
        assert occluded(c, from_point=False, eps=eps) != truth, c["sample"]
        assert occluded(c, from_point=True, eps=eps) == truth, c["sample"]


def test_the_segments_are_edge_on():
    """Incidence cosine of the segment on the sample's own triangle below 1e-4."""
    _, cases = load_cases()
    for c in cases:
        a, b, cc = c["tris"][c["own"]].astype(np.float64)
        n = np.cross(b - a, cc - a)
        dv = c["point"].astype(np.float64) - c["eye"].astype(np.float64)
        cos = abs(n @ dv) / (np.linalg.norm(n) * np.linalg.norm(dv))
        assert cos < 1e-4, (c["sample"], cos)
