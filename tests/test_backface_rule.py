"""The back-face rule checked against the oracle on the CPU (no GPU).

The rule: a point x on a triangle of a closed mesh (one that bounds a solid), seen from
an eye e outside that mesh's bounding box, with the eye behind the triangle's plane, is
occluded when no triangle of the mesh other than x's own can cross the segment's last
stretch, x to x + 1e-4 (e - x): such a crossing exists (the winding number is 0 at e and
1 just behind the triangle) and then lies at tau < 1 - 1e-4, where the oracle counts it.
x is the FP32 rounding of a point of the triangle, off its plane by up to eta = 2^-24
(|x| + |y| + |z|): the segment meets the plane within eta / c of x (c: cosine to the
inward normal), still inside the triangle while c D >= 4 eta (D: x's distance to the
triangle's edges), which the rule requires (without it a grazing segment near an edge
can pass beside the triangle and never enter the solid).  Triangles that can cross that stretch lie
within 1e-4 |e - x| of x; the kernel lists those within rmax = 1e-4 x (twice the scene's
diagonal + 4 m) (segments longer than rmax / 1e-4 go to the BVH walk).  Here the same rule,
written in FP64 with a k-d tree for the neighbour lists, is applied to every in-cone pair
of seeded samples of the paper-shaped and the scale-up workloads; wherever it says
occluded, the oracle must agree or call the pair fragile.  The closed-mesh flags come
from the library's host-side topology check (gm_mesh_closed)."""
import ctypes
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2601_07571_amd", "libgazemap.so")
EPS = 1e-4
K_CAND = 8


def _closed(lib, V, I):
    V = np.ascontiguousarray(V, np.float32); I = np.ascontiguousarray(I, np.int32)
    return lib.gm_mesh_closed(V.ctypes.data_as(ctypes.c_void_p), len(V), I.ctypes.data_as(ctypes.c_void_p), len(I))


def stretch_may_cross(x, U, tri):
    """Whether x + t u, t in [0, EPS], may touch the triangle, for each row u of U: a
    Moller-Trumbore test in FP64 whose margins keep every doubtful case as 'may'."""
    v0, v1, v2 = tri
    e1, e2 = v1 - v0, v2 - v0
    pv = np.cross(U, e2)
    det = pv @ e1
    scale = np.linalg.norm(e1) * np.linalg.norm(e2) * np.linalg.norm(U, axis=1)
    flat = np.abs(det) <= 1e-9 * scale
    det = np.where(flat, 1.0, det)
    tv = x - v0
    b1 = (pv @ tv) / det
    qv = np.cross(tv, e1)
    b2 = (U @ qv) / det
    t = (e2 @ qv) / det
    tol = 1e-6
    inside = (b1 >= -tol) & (b2 >= -tol) & (b1 + b2 <= 1 + tol) & (t >= -1e-3 * EPS) & (t <= EPS * (1 + 1e-3))
    return flat | inside


class Rule:
    def __init__(self, meshes, closed):
        self.V = [np.asarray(V, np.float64) for V, _ in meshes]
        self.I = [np.asarray(I, np.int64) for _, I in meshes]
        self.closed = closed
        lo = np.min([V.min(0) for V in self.V], 0); hi = np.max([V.max(0) for V in self.V], 0)
        self.rmax = EPS * (2.0 * float(np.linalg.norm(hi.astype(np.float32).astype(np.float64) -
                                                      lo.astype(np.float32).astype(np.float64))) + 4.0)
        self.lmax = self.rmax / EPS * (1 - 1e-3)
        self.box = [(V.min(0), V.max(0)) for V in self.V]
        self.tree, self.tlo, self.thi, self.rad = [], [], [], []
        for V, I in zip(self.V, self.I):
            T = V[I]
            c = T.mean(1)
            self.tree.append(cKDTree(c))
            self.tlo.append(T.min(1)); self.thi.append(T.max(1))
            self.rad.append(float(np.max(np.linalg.norm(T - c[:, None], axis=2))))
        self.base = np.cumsum([0] + [len(I) for I in self.I])

    def point(self, x, tri, mesh):
        """(unit normal, distance to the triangle's edges, neighbour list) or None when the
        rule cannot apply to the point."""
        if not self.closed[mesh]:
            return None
        lt = tri - self.base[mesh]
        a, b, c = self.V[mesh][self.I[mesh][lt]]
        n = np.cross(b - a, c - a)
        nn = np.linalg.norm(n)
        bar = [np.cross(c - b, x - b) @ n, np.cross(a - c, x - c) @ n, np.cross(b - a, x - a) @ n]
        D = min(max(bi, 0.0) / np.linalg.norm(e) for bi, e in zip(bar, (c - b, a - c, b - a))) / nn
        n /= nn
        cand = []
        for j in self.tree[mesh].query_ball_point(x, self.rmax + self.rad[mesh]):
            if j == lt:
                continue
            d = np.maximum(np.maximum(self.tlo[mesh][j] - x, x - self.thi[mesh][j]), 0.0)
            if d @ d <= self.rmax ** 2 * 1.001:
                cand.append(j)
        if len(cand) > K_CAND or not D > 0:
            return None
        return n, D, [self.V[mesh][self.I[mesh][j]] for j in cand]

    def occluded(self, pt, x, E, mesh):
        """The rule for point x and each eye (row of E): True where it says occluded."""
        out = np.zeros(len(E), bool)
        if pt is None:
            return out
        n, D, cand = pt
        U = E - x
        L = np.linalg.norm(U, axis=1)
        lo, hi = self.box[mesh]
        inside = np.all((E >= lo) & (E <= hi), axis=1)
        eta = 2.0 ** -24 * np.abs(x).sum()
        ok = (-(U @ n) / L * D >= 4 * eta) & (L <= self.lmax) & ~inside
        for t in cand:
            ok &= ~stretch_may_cross(x, U, t)
        return ok


def _check(w, meshes, pos, tri, mesh, pick):
    lib = ctypes.CDLL(LIB)
    closed = [bool(_closed(lib, V, I)) for V, I in meshes]
    rule = Rule(meshes, closed)
    eye = w.fix.eye.astype(np.float64); gaze = w.fix.gaze.astype(np.float64)
    sig = np.tan(np.radians(w.theta_deg))
    ps, pf, said, back = [], [], [], []
    for s in pick:
        x = pos[s].astype(np.float64)
        p = x - eye
        d1 = np.einsum("ij,ij->i", p, gaze)
        c = np.cross(p, gaze)
        f = np.nonzero((d1 > 0) & (np.einsum("ij,ij->i", c, c) <= 16 * sig * sig * d1 * d1 * (1 + 1e-6)))[0]
        pt = rule.point(x, int(tri[s]), int(mesh[s]))
        ps.append(np.full(len(f), s)); pf.append(f)
        said.append(rule.occluded(pt, x, eye[f], int(mesh[s])))
        back.append(np.zeros(len(f), bool) if pt is None else (eye[f] - x) @ pt[0] < 0)
    ps = np.concatenate(ps); pf = np.concatenate(pf); said = np.concatenate(said); back = np.concatenate(back)
    sub = np.nonzero(said)[0]
    vis, frag = oracle.Scene(meshes).pair_visibility(pos, tri, mesh, w.fix.eye, ps[sub], pf[sub],
                                                     mode=oracle.OCC_FULL)
    return {"in_cone": len(ps), "back_facing_closed": int(back.sum()), "settled": int(said.sum()),
            "fragile_among_settled": int(frag.sum()), "wrong": int((vis & ~frag).sum())}


@pytest.fixture(scope="module")
def lib_built():
    if not os.path.exists(LIB):
        pytest.skip("library not built")


def test_closed_flags(lib_built):
    lib = ctypes.CDLL(LIB)
    flags = [_closed(lib, m.V, m.I) for m in workloads.paper_shaped_meshes()]
    assert flags == [1, 1, 1, 0]                       # the heightfield has a border
    cube = workloads.cube_mesh(0.5)
    assert _closed(lib, cube.V, cube.I) == 1
    assert _closed(lib, cube.V, cube.I[:, [0, 2, 1]]) == 0          # inside out: negative volume
    bad = cube.I.copy(); bad[3] = bad[3][[0, 2, 1]]
    assert _closed(lib, cube.V, bad) == 0                            # one triangle wound the other way
    assert _closed(lib, cube.V, cube.I[:-1]) == 0                    # a hole
    # faces with vertices of their own: merged by position, still closed
    V = cube.V[cube.I.reshape(-1)]
    assert _closed(lib, V, np.arange(len(V), dtype=np.int32).reshape(-1, 3)) == 1
    assert _closed(lib, cube.V, np.array([[0, 1, 9]], np.int32)) == -1


def test_rule_agrees_with_the_oracle_paper_shaped(lib_built):
    w = workloads.paper_shaped_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    s = oracle.sample_scene(meshes, 204240.0, w.seed)
    pick = np.random.default_rng(21).choice(len(s.tri), 1500, replace=False)
    r = _check(w, meshes, s.pos32, s.tri, s.mesh, pick)
    print("paper-shaped:", r)
    assert r["wrong"] == 0
    assert r["settled"] > 0.5 * r["back_facing_closed"] > 0


def test_rule_agrees_with_the_oracle_scale_up(lib_built):
    w = workloads.scale_up_scene()
    meshes = [(m.V, m.I) for m in w.meshes]
    s = oracle.sample_scene(meshes, 10000.0, w.seed)
    pick = np.random.default_rng(22).choice(len(s.tri), 250, replace=False)
    r = _check(w, meshes, s.pos32, s.tri, s.mesh, pick)
    print("scale-up:", r)
    assert r["wrong"] == 0
    assert r["settled"] > 0.5 * r["back_facing_closed"] > 0
