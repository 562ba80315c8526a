"""FP64 CPU oracle for surface-based fixation density maps (arXiv 2601.07571).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``.  The product library never imports
it, and it imports nothing from the product library.

The arithmetic lives in ``gm_oracle.c`` (plain C, FP64, ``-ffp-contract=off``),
loaded here through ctypes; this module adds the per-scene orchestration and a
second, pure-Python Philox4x32-10 used to pin the C one.

Parity status of each function (what pins it is in ``tests/test_oracle_*.py``):
  philox4x32_10 / philox_py ... pinned (published known answers, two codes)
  triangle_areas .............. pinned (Heron in Kahan's ordering, closed forms)
  mesh_weights / sample_count . pinned (exact integer brute force, k*area)
  sample_scene / sample_at .... pinned (chi-square, KS, brute force, invariants;
                                 sample_at equals sample_scene's entries)
  lattice_* ................... pinned (loop enumeration of Eq. (2), the lattice
                                 set, Eq. (1) and (4) closed forms and bounds)
  pair_value / density ........ pinned (plane closed form, 4-sigma mass,
                                 linearity, rigid motion, hand-computed cases)
  visibility .................. pinned (brute force == BVH, convex sphere ==
                                 front-facing, hand-placed occluders)
  normalize ................... pinned (max == 1, range)
  local_fixation / posed_density  pinned (identity poses give the static map,
                                 exact quarter turns give the static map, a mesh
                                 carried along with its eye repeats one fixation,
                                 a moving occluder equals the static maps of each
                                 instant, shears are refused)
  camera_basis / crop_bounds /
  density_zbuffer ............. pinned (centred gaze: the square of half-width
                                 n tan(phi); oblique gaze: A0, A1, B0, B1 on the
                                 cone and inside the bounds, mirror symmetry;
                                 z-buffer depths of planes and spheres in closed
                                 form, an occluder's shadow, eps widening;
                                 a fine z-buffer agrees with the exact test
                                 away from silhouettes).  A crop that reaches
                                 behind the camera, or with a corner 80 degrees
                                 or more off the gaze, refuses its fixation: the
                                 builder's reading (Appendix A gives the crop,
                                 not what to do where it degenerates), shared
                                 by both sides, not pinned by the paper
  in_window / density_window .. pinned (partition of a recording into back-to-back
                                 windows sums to the whole, boundary and NaN
                                 times, empty window)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile gm_oracle.c into liboracle.so (gcc, FP64, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.POINTER
    c_f, c_d, c_i32, c_i64, c_u32, c_u64, c_u8 = (
        ctypes.c_float, ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
        ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint8)
    lib.or_philox4x32_10.argtypes = [P(c_u32), P(c_u32), P(c_u32)]
    lib.or_philox_stream.argtypes = [c_u64, c_i64, c_u32, c_u32, c_u64, P(c_u32)]
    lib.or_triangle_areas.argtypes = [P(c_f), P(c_i32), c_i64, P(c_d)]
    lib.or_mesh_weights.argtypes = [P(c_d), c_i64, P(c_u64), P(c_u64), P(c_i32)]
    lib.or_mesh_weights.restype = c_u64
    lib.or_sample_count.argtypes = [c_u64, c_i32, c_d]
    lib.or_sample_count.restype = c_i64
    lib.or_sample_mesh.argtypes = [P(c_f), P(c_i32), P(c_u64), c_i64, c_u32, c_u64, c_i64, c_i64,
                                   P(c_i32), P(c_d), P(c_d), P(c_f), P(c_f)]
    lib.or_lattice_points.argtypes = [c_i64]
    lib.or_lattice_points.restype = c_i64
    lib.or_lattice_resolution.argtypes = [c_d, c_d]
    lib.or_lattice_resolution.restype = c_i64
    lib.or_lattice_row_col.argtypes = [c_i64, P(c_i64), P(c_i64)]
    lib.or_lattice_counts.argtypes = [P(c_f), P(c_i32), c_i64, c_d, P(c_i64), P(c_i64)]
    lib.or_lattice_counts.restype = c_i64
    lib.or_lattice_mesh.argtypes = [P(c_f), P(c_i32), c_i64, c_d, c_i64, P(c_i32), P(c_d), P(c_f), P(c_f)]
    lib.or_lattice_mesh.restype = c_i64
    lib.or_scene_create.argtypes = [P(c_f), P(c_i32), P(c_i32), c_i64]
    lib.or_scene_create.restype = ctypes.c_void_p
    lib.or_scene_destroy.argtypes = [ctypes.c_void_p]
    lib.or_visible.argtypes = [ctypes.c_void_p, P(c_d), P(c_d), c_i32, c_i32, ctypes.c_int, c_d,
                               ctypes.c_int, P(ctypes.c_int)]
    lib.or_visible.restype = ctypes.c_int
    lib.or_pair_value.argtypes = [P(c_d), P(c_d), P(c_d), c_d, c_d, P(c_d), P(c_d)]
    lib.or_pair_value.restype = ctypes.c_int
    lib.or_density.argtypes = [ctypes.c_void_p, P(c_f), P(c_i32), P(c_i32), c_i64, P(c_f), P(c_f),
                               P(c_f), c_i64, c_d, ctypes.c_int, c_d, ctypes.c_int, ctypes.c_int,
                               P(c_d), P(c_d), P(c_i64)]
    lib.or_closest.argtypes = [ctypes.c_void_p, P(c_d), P(c_d), c_d, c_d, P(ctypes.c_int)]
    lib.or_closest.restype = c_d
    lib.or_zbuffer.argtypes = [ctypes.c_void_p, P(c_d), P(c_d), c_d, c_d, ctypes.c_int, P(c_d), P(c_u8)]
    lib.or_density_zbuffer.argtypes = [ctypes.c_void_p, P(c_f), c_i64, P(c_f), P(c_f), P(c_f), P(c_d), c_i64,
                                       c_d, ctypes.c_int, c_d, c_d, c_d, ctypes.c_int, P(c_d), P(c_u8), P(c_d),
                                       P(c_d), P(c_i64)]
    lib.or_pair_visibility.argtypes = [ctypes.c_void_p, P(c_f), P(c_i32), P(c_i32), P(c_f),
                                       P(c_i64), P(c_i64), c_i64, ctypes.c_int, c_d, ctypes.c_int,
                                       P(c_u8), P(c_u8)]
    lib.or_pair_values.argtypes = [P(c_f), P(c_f), P(c_f), P(c_f), P(c_i64), P(c_i64), c_i64, c_d,
                                   P(c_d), P(c_d), P(c_u8)]
    lib.or_normalize.argtypes = [P(c_d), c_i64, P(c_d)]
    lib.or_normalize.restype = c_d
    _lib = lib
    return lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


# ----------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al., SC'11)
# ----------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    """C oracle: one block for counter (4 x u32) and key (2 x u32)."""
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.or_philox4x32_10(_ptr(c, ctypes.c_uint32), _ptr(k, ctypes.c_uint32), _ptr(out, ctypes.c_uint32))
    return out


def philox_stream(first: int, n: int, w2: int, w3: int, seed: int):
    """C oracle: blocks for counters (first+i as 64 bits, w2, w3), key = seed."""
    lib = _load()
    out = np.zeros((n, 4), dtype=np.uint32)
    lib.or_philox_stream(first, n, w2, w3, seed, _ptr(out, ctypes.c_uint32))
    return out


def philox_py(ctr, key):
    """Second, independent Philox4x32-10 in Python integers (pins the C one)."""
    m = (0xD2511F53, 0xCD9E8D57)
    weyl = (0x9E3779B9, 0xBB67AE85)
    mask = 0xFFFFFFFF
    c = [int(v) & mask for v in ctr]
    k = [int(v) & mask for v in key]
    for _ in range(10):
        a = m[0] * c[0]
        b = m[1] * c[2]
        c = [((b >> 32) ^ c[1] ^ k[0]) & mask, b & mask,
             ((a >> 32) ^ c[3] ^ k[1]) & mask, a & mask]
        k = [(k[0] + weyl[0]) & mask, (k[1] + weyl[1]) & mask]
    return c


# ----------------------------------------------------------------------------
# Areas, weights, counts, sampling (Sec. 3.1)
# ----------------------------------------------------------------------------

def triangle_areas(V, I):
    lib = _load()
    V = np.ascontiguousarray(V, dtype=np.float32)
    I = np.ascontiguousarray(I, dtype=np.int32)
    A = np.zeros(len(I), dtype=np.float64)
    lib.or_triangle_areas(_ptr(V, ctypes.c_float), _ptr(I, ctypes.c_int32), len(I), _ptr(A, ctypes.c_double))
    return A


def mesh_weights(A):
    """(W uint64[T], C inclusive uint64[T], S, total)."""
    lib = _load()
    A = np.ascontiguousarray(A, dtype=np.float64)
    W = np.zeros(len(A), dtype=np.uint64)
    C = np.zeros(len(A), dtype=np.uint64)
    S = ctypes.c_int32(0)
    tot = lib.or_mesh_weights(_ptr(A, ctypes.c_double), len(A), _ptr(W, ctypes.c_uint64),
                              _ptr(C, ctypes.c_uint64), ctypes.byref(S))
    return W, C, int(S.value), int(tot)


def sample_count(Wm: int, S: int, k: float) -> int:
    return int(_load().or_sample_count(Wm, S, k))


@dataclass
class OracleSamples:
    tri_local: np.ndarray    # int32 [N], mesh-local triangle index
    tri: np.ndarray          # int32 [N], scene-global triangle index
    mesh: np.ndarray         # int32 [N]
    bary64: np.ndarray       # float64 [N][2]  (b1, b2)
    pos64: np.ndarray        # float64 [N][3]
    bary32: np.ndarray       # float32 [N][2]
    pos32: np.ndarray        # float32 [N][3]
    counts: np.ndarray       # int64 [M]
    S: np.ndarray            # int32 [M]
    Wm: np.ndarray           # uint64 [M]


def sample_scene(meshes, k: float, seed: int) -> OracleSamples:
    """Samples of every mesh, mesh order then Philox counter order."""
    lib = _load()
    parts = []
    counts, Ss, Wms = [], [], []
    tri_base = 0
    for m, (V, I) in enumerate(meshes):
        V = np.ascontiguousarray(V, dtype=np.float32)
        I = np.ascontiguousarray(I, dtype=np.int32)
        A = triangle_areas(V, I)
        W, C, S, Wm = mesh_weights(A)
        n = sample_count(Wm, S, k) if Wm > 0 else 0
        counts.append(n); Ss.append(S); Wms.append(Wm)
        tri = np.zeros(n, np.int32)
        b64 = np.zeros((n, 2)); p64 = np.zeros((n, 3))
        b32 = np.zeros((n, 2), np.float32); p32 = np.zeros((n, 3), np.float32)
        if n > 0:
            lib.or_sample_mesh(_ptr(V, ctypes.c_float), _ptr(I, ctypes.c_int32), _ptr(C, ctypes.c_uint64),
                               len(I), m, seed, 0, n, _ptr(tri, ctypes.c_int32), _ptr(b64, ctypes.c_double),
                               _ptr(p64, ctypes.c_double), _ptr(b32, ctypes.c_float), _ptr(p32, ctypes.c_float))
        parts.append((tri, tri + tri_base, np.full(n, m, np.int32), b64, p64, b32, p32))
        tri_base += len(I)
    cat = [np.concatenate([p[i] for p in parts]) if parts else None for i in range(7)]
    return OracleSamples(cat[0].astype(np.int32), cat[1].astype(np.int32), cat[2].astype(np.int32),
                         cat[3], cat[4], cat[5].astype(np.float32), cat[6].astype(np.float32),
                         np.array(counts, np.int64), np.array(Ss, np.int32), np.array(Wms, np.uint64))


def sample_at(meshes, k: float, seed: int, index: int):
    """One sample of sample_scene's output, by its global index (mesh order, then
    Philox counter order), without drawing the others: (pos32 [3], global triangle,
    mesh)."""
    lib = _load()
    tri_base = 0
    for m, (V, I) in enumerate(meshes):
        V = np.ascontiguousarray(V, dtype=np.float32)
        I = np.ascontiguousarray(I, dtype=np.int32)
        _, C, S, Wm = mesh_weights(triangle_areas(V, I))
        n = sample_count(Wm, S, k) if Wm > 0 else 0
        if index < n:
            tri = np.zeros(1, np.int32)
            b64 = np.zeros((1, 2)); p64 = np.zeros((1, 3))
            b32 = np.zeros((1, 2), np.float32); p32 = np.zeros((1, 3), np.float32)
            lib.or_sample_mesh(_ptr(V, ctypes.c_float), _ptr(I, ctypes.c_int32), _ptr(C, ctypes.c_uint64),
                               len(I), m, seed, int(index), 1, _ptr(tri, ctypes.c_int32), _ptr(b64, ctypes.c_double),
                               _ptr(p64, ctypes.c_double), _ptr(b32, ctypes.c_float), _ptr(p32, ctypes.c_float))
            return p32[0], int(tri[0]) + tri_base, m
        index -= n
        tri_base += len(I)
    raise IndexError("sample index beyond the scene's samples")


# ----------------------------------------------------------------------------
# The paper's lattice sampler (Sec. 3.1.1, 3.1.2)
# ----------------------------------------------------------------------------

def lattice_points(r: int) -> int:
    """Eq. (1)."""
    return int(_load().or_lattice_points(int(r)))


def lattice_resolution(k: float, A: float) -> int:
    """Eq. (4), truncated to a whole resolution, at least 1."""
    return int(_load().or_lattice_resolution(float(k), float(A)))


def lattice_row_col(idx: int):
    """Eq. (2) with the integer correction."""
    row, col = ctypes.c_int64(), ctypes.c_int64()
    _load().or_lattice_row_col(int(idx), ctypes.byref(row), ctypes.byref(col))
    return row.value, col.value


def lattice_counts(V, I, k: float):
    """Per-triangle (resolution, point count) of one mesh."""
    V = np.ascontiguousarray(V, dtype=np.float32)
    I = np.ascontiguousarray(I, dtype=np.int32)
    r = np.zeros(len(I), np.int64); c = np.zeros(len(I), np.int64)
    _load().or_lattice_counts(_ptr(V, ctypes.c_float), _ptr(I, ctypes.c_int32), len(I), float(k),
                              _ptr(r, ctypes.c_int64), _ptr(c, ctypes.c_int64))
    return r, c


@dataclass
class OracleLattice:
    tri_local: np.ndarray    # int32 [N], mesh-local triangle index
    tri: np.ndarray          # int32 [N], scene-global triangle index
    mesh: np.ndarray         # int32 [N]
    pos64: np.ndarray        # float64 [N][3]
    bary32: np.ndarray       # float32 [N][2]  (w2, w3): weights of v1, v2
    pos32: np.ndarray        # float32 [N][3]
    counts: np.ndarray       # int64 [M]


def lattice_scene(meshes, k: float) -> OracleLattice:
    """Every lattice point of every mesh: mesh order, triangle order, then idx."""
    lib = _load()
    parts, counts = [], []
    tri_base = 0
    for m, (V, I) in enumerate(meshes):
        V = np.ascontiguousarray(V, dtype=np.float32)
        I = np.ascontiguousarray(I, dtype=np.int32)
        n = int(lib.or_lattice_counts(_ptr(V, ctypes.c_float), _ptr(I, ctypes.c_int32), len(I), float(k),
                                      None, None))
        tri = np.zeros(n, np.int32); p64 = np.zeros((n, 3))
        b32 = np.zeros((n, 2), np.float32); p32 = np.zeros((n, 3), np.float32)
        lib.or_lattice_mesh(_ptr(V, ctypes.c_float), _ptr(I, ctypes.c_int32), len(I), float(k), n,
                            _ptr(tri, ctypes.c_int32), _ptr(p64, ctypes.c_double), _ptr(b32, ctypes.c_float),
                            _ptr(p32, ctypes.c_float))
        counts.append(n)
        parts.append((tri, tri + tri_base, np.full(n, m, np.int32), p64, b32, p32))
        tri_base += len(I)
    cat = [np.concatenate([p[i] for p in parts]) for i in range(6)]
    return OracleLattice(cat[0].astype(np.int32), cat[1].astype(np.int32), cat[2].astype(np.int32), cat[3],
                         cat[4].astype(np.float32), cat[5].astype(np.float32), np.array(counts, np.int64))


# ----------------------------------------------------------------------------
# Density (Sec. 3.2)
# ----------------------------------------------------------------------------

OCC_NONE, OCC_SELF, OCC_FULL = 0, 1, 2
EPS_V = 1e-4


class Scene:
    """Triangle soup of all meshes with the oracle's own median-split BVH."""

    def __init__(self, meshes):
        lib = _load()
        Vs, Is, Ms = [], [], []
        vbase = 0
        for m, (V, I) in enumerate(meshes):
            V = np.asarray(V, np.float32); I = np.asarray(I, np.int32)
            Vs.append(V); Is.append(I + vbase); Ms.append(np.full(len(I), m, np.int32))
            vbase += len(V)
        self.V = np.ascontiguousarray(np.concatenate(Vs) if Vs else np.zeros((0, 3), np.float32))
        self.I = np.ascontiguousarray(np.concatenate(Is) if Is else np.zeros((0, 3), np.int32))
        self.tri_mesh = np.ascontiguousarray(np.concatenate(Ms) if Ms else np.zeros(0, np.int32))
        self._h = lib.or_scene_create(_ptr(self.V, ctypes.c_float), _ptr(self.I, ctypes.c_int32),
                                      _ptr(self.tri_mesh, ctypes.c_int32), len(self.I))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.or_scene_destroy(self._h)
            self._h = None

    def visible(self, e, x, own_tri=-1, own_mesh=-1, mode=OCC_FULL, eps=EPS_V, brute=False):
        e = np.ascontiguousarray(e, np.float64); x = np.ascontiguousarray(x, np.float64)
        fr = ctypes.c_int(0)
        v = _lib.or_visible(self._h, _ptr(e, ctypes.c_double), _ptr(x, ctypes.c_double), own_tri, own_mesh,
                            mode, eps, int(brute), ctypes.byref(fr))
        return bool(v), bool(fr.value)

    def pair_visibility(self, pos, tri, mesh, eye, pair_s, pair_f, mode=OCC_FULL, eps=EPS_V, brute=False):
        pos = np.ascontiguousarray(pos, np.float32); eye = np.ascontiguousarray(eye, np.float32)
        tri = None if tri is None else np.ascontiguousarray(tri, np.int32)
        mesh = None if mesh is None else np.ascontiguousarray(mesh, np.int32)
        ps = np.ascontiguousarray(pair_s, np.int64); pf = np.ascontiguousarray(pair_f, np.int64)
        vis = np.zeros(len(ps), np.uint8); frag = np.zeros(len(ps), np.uint8)
        _lib.or_pair_visibility(self._h, _ptr(pos, ctypes.c_float), _ptr(tri, ctypes.c_int32),
                                _ptr(mesh, ctypes.c_int32), _ptr(eye, ctypes.c_float),
                                _ptr(ps, ctypes.c_int64), _ptr(pf, ctypes.c_int64), len(ps), mode, eps,
                                int(brute), _ptr(vis, ctypes.c_uint8), _ptr(frag, ctypes.c_uint8))
        return vis.astype(bool), frag.astype(bool)


def pair_value(x, e, r, t, theta_deg):
    """(in_cone, g, margin) of one pair in FP64."""
    lib = _load()
    x = np.ascontiguousarray(x, np.float64); e = np.ascontiguousarray(e, np.float64)
    r = np.ascontiguousarray(r, np.float64)
    g = ctypes.c_double(0.0); mg = ctypes.c_double(0.0)
    sigma = math.tan(math.radians(theta_deg))
    inside = lib.or_pair_value(_ptr(x, ctypes.c_double), _ptr(e, ctypes.c_double), _ptr(r, ctypes.c_double),
                               float(t), sigma, ctypes.byref(g), ctypes.byref(mg))
    return bool(inside), g.value, mg.value


def pair_values(pos, eye, gaze, dur, pair_s, pair_f, theta_deg):
    """(g, margin, in_cone) for explicit pairs, FP64, no visibility; g = 0 outside the cone."""
    lib = _load()
    pos = np.ascontiguousarray(pos, np.float32); eye = np.ascontiguousarray(eye, np.float32)
    gaze = np.ascontiguousarray(gaze, np.float32); dur = np.ascontiguousarray(dur, np.float32)
    ps = np.ascontiguousarray(pair_s, np.int64); pf = np.ascontiguousarray(pair_f, np.int64)
    g = np.zeros(len(ps)); mg = np.zeros(len(ps)); inc = np.zeros(len(ps), np.uint8)
    lib.or_pair_values(_ptr(pos, ctypes.c_float), _ptr(eye, ctypes.c_float), _ptr(gaze, ctypes.c_float),
                       _ptr(dur, ctypes.c_float), _ptr(ps, ctypes.c_int64), _ptr(pf, ctypes.c_int64), len(ps),
                       float(theta_deg), _ptr(g, ctypes.c_double), _ptr(mg, ctypes.c_double),
                       _ptr(inc, ctypes.c_uint8))
    return g, mg, inc.astype(bool)


@dataclass
class OracleDensity:
    rho: np.ndarray      # float64 [n], raw density
    budget: np.ndarray   # float64 [n], sum of g over boundary-ambiguous / fragile pairs
    stats: np.ndarray    # int64 [n][4]: in-cone, visible, ambiguous, fragile


def density(scene: Scene | None, pos, tri, mesh, eye, gaze, dur, theta_deg, mode=OCC_FULL,
            eps=EPS_V, brute=False, nthreads=None) -> OracleDensity:
    lib = _load()
    pos = np.ascontiguousarray(pos, np.float32).reshape(-1, 3)
    n = len(pos)
    tri = None if tri is None else np.ascontiguousarray(tri, np.int32)
    mesh = None if mesh is None else np.ascontiguousarray(mesh, np.int32)
    eye = np.ascontiguousarray(eye, np.float32).reshape(-1, 3)
    gaze = np.ascontiguousarray(gaze, np.float32).reshape(-1, 3)
    dur = np.ascontiguousarray(dur, np.float32).reshape(-1)
    F = len(eye)
    rho = np.zeros(n); budget = np.zeros(n); stats = np.zeros((n, 4), np.int64)
    if scene is None:
        scene = Scene([])
        mode = OCC_NONE
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    lib.or_density(scene._h, _ptr(pos, ctypes.c_float), _ptr(tri, ctypes.c_int32), _ptr(mesh, ctypes.c_int32),
                   n, _ptr(eye, ctypes.c_float), _ptr(gaze, ctypes.c_float), _ptr(dur, ctypes.c_float), F,
                   float(theta_deg), mode, eps, int(brute), int(nthreads), _ptr(rho, ctypes.c_double),
                   _ptr(budget, ctypes.c_double), _ptr(stats, ctypes.c_int64))
    return OracleDensity(rho, budget, stats)


def in_window(time, t_begin, t_end):
    """Fixations whose start time lies in the analysis interval [t_begin, t_end)
    (the time interval among the generation parameters, Sec. 3.3.4): half open, so
    back-to-back windows split a recording without counting a fixation twice; a NaN
    time is in no window."""
    t = np.asarray(time, np.float64).reshape(-1)
    return (t >= t_begin) & (t < t_end)


def density_window(scene: Scene | None, pos, tri, mesh, eye, gaze, dur, time, window, theta_deg, mode=OCC_FULL,
                   **kw) -> OracleDensity:
    """rho of Sec. 3.2 over the fixations in the window only: the per-fixation sum of
    Sec. 3.2.1 restricted to that subset."""
    sel = in_window(time, window[0], window[1])
    eye = np.asarray(eye, np.float32).reshape(-1, 3)[sel]
    gaze = np.asarray(gaze, np.float32).reshape(-1, 3)[sel]
    dur = np.asarray(dur, np.float32).reshape(-1)[sel]
    return density(scene, pos, tri, mesh, eye, gaze, dur, theta_deg, mode, **kw)


SIMILARITY_TOL = 1e-5


def local_fixation(pose, e, r):
    """A fixation seen from a mesh placed in the world by `pose` (3x4 row-major, mesh frame
    -> world): eye A^-1 (e - b) and gaze A^-1 r with A^-1 = A^T / s2, s2 = trace(A^T A) / 3,
    each in FP64 as ((A_0i v_0 + A_1i v_1) + A_2i v_2) / s2 and rounded to FP32 (the
    fixation's inputs in that frame; the paper likewise expresses p and r in a local
    space, Sec. 3.2.1).  Returns (eye, gaze, ok); ok is False unless A is a similarity
    (every entry of A^T A - s2 I within 1e-5 s2), the only maps that keep angles."""
    P = np.asarray(pose, np.float32).reshape(12).astype(np.float64)
    A = [[P[0], P[1], P[2]], [P[4], P[5], P[6]], [P[8], P[9], P[10]]]
    b = [P[3], P[7], P[11]]
    G = [[(A[0][i] * A[0][j] + A[1][i] * A[1][j]) + A[2][i] * A[2][j] for j in range(3)] for i in range(3)]
    s2 = ((G[0][0] + G[1][1]) + G[2][2]) / 3.0
    ok = bool(np.all(np.isfinite(P))) and s2 > 0.0 and math.isfinite(s2)
    if ok:
        ok = all(abs(G[i][j] - (s2 if i == j else 0.0)) <= SIMILARITY_TOL * s2 for i in range(3) for j in range(3))
    e = np.asarray(e, np.float32).astype(np.float64); r = np.asarray(r, np.float32).astype(np.float64)
    d = [e[0] - b[0], e[1] - b[1], e[2] - b[2]]

    def frame(v):
        return np.array([((A[0][i] * v[0] + A[1][i] * v[1]) + A[2][i] * v[2]) / s2 if s2 > 0 else 0.0
                         for i in range(3)], np.float32)

    return frame(d), frame(r), ok


def posed_world(V, pose):
    """Vertices of a mesh placed by `pose` (3x4, FP64 arithmetic, rounded to FP32)."""
    P = np.asarray(pose, np.float32).astype(np.float64).reshape(3, 4)
    V = np.asarray(V, np.float32).astype(np.float64)
    W = np.stack([((P[k, 0] * V[:, 0] + P[k, 1] * V[:, 1]) + P[k, 2] * V[:, 2]) + P[k, 3] for k in range(3)], 1)
    return W.astype(np.float32)


def posed_density(meshes, pos, tri, mesh, eye, gaze, dur, pose, theta_deg, mode=OCC_FULL,
                  eps=EPS_V) -> OracleDensity:
    """rho of Sec. 3.2 when the meshes move: at fixation f mesh m stands where pose[f, m]
    (3x4, mesh frame -> world) puts it and the points move with their mesh (values
    bound to objects, Sec. 2.2, Sec. 3.3.3).  The pair value is taken in the point's
    mesh frame from local_fixation's FP32 eye and gaze; visibility is taken in the world
    at the fixation's time: with mode self against the point's own mesh (in its own
    frame, the same thing), with mode full against every mesh as posed, the point moved
    to the world in FP64.  A fixation whose duration, eye or gaze is invalid or whose
    any pose is not a similarity contributes nothing.  Same bookkeeping (budget, stats)
    as density()."""
    pos = np.asarray(pos, np.float32).reshape(-1, 3)
    tri = np.asarray(tri, np.int32); mesh = np.asarray(mesh, np.int32)
    eye = np.asarray(eye, np.float32).reshape(-1, 3); gaze = np.asarray(gaze, np.float32).reshape(-1, 3)
    dur = np.asarray(dur, np.float32).reshape(-1)
    pose = np.asarray(pose, np.float32).reshape(len(eye), len(meshes), 12)
    n = len(pos); M = len(meshes)
    rho = np.zeros(n); budget = np.zeros(n); stats = np.zeros((n, 4), np.int64)
    own = Scene(meshes)
    groups = [np.nonzero(mesh == m)[0] for m in range(M)]
    for f in range(len(eye)):
        t = float(dur[f])
        if not (np.all(np.isfinite(eye[f])) and np.all(np.isfinite(gaze[f])) and np.dot(gaze[f].astype(np.float64),
                gaze[f].astype(np.float64)) > 0 and math.isfinite(t) and 0.0 <= t <= 1e6):
            continue
        loc = [local_fixation(pose[f, m], eye[f], gaze[f]) for m in range(M)]
        if not all(ok for _, _, ok in loc):
            continue
        world = Scene([(posed_world(V, pose[f, m]), I) for m, (V, I) in enumerate(meshes)]) \
            if mode == OCC_FULL else None
        for m in range(M):
            idx = groups[m]
            if len(idx) == 0:
                continue
            el, rl, _ = loc[m]
            g, mg, inc = pair_values(pos[idx], el[None], rl[None], dur[f:f + 1], np.arange(len(idx)),
                                     np.zeros(len(idx), np.int64), theta_deg)
            amb = np.abs(mg) < 1e-5
            P = pose[f, m].astype(np.float64).reshape(3, 4)
            for j in np.nonzero(inc | amb)[0]:
                s = idx[j]
                if mode == OCC_NONE:
                    vis, frag = True, False
                elif mode == OCC_SELF:
                    vis, frag = own.visible(el.astype(np.float64), pos[s].astype(np.float64), int(tri[s]), m,
                                            OCC_SELF, eps)
                else:
                    x = pos[s].astype(np.float64)
                    xw = np.array([((P[k, 0] * x[0] + P[k, 1] * x[1]) + P[k, 2] * x[2]) + P[k, 3]
                                   for k in range(3)])
                    vis, frag = world.visible(eye[f].astype(np.float64), xw, int(tri[s]), m, OCC_FULL, eps)
                if inc[j]:
                    stats[s, 0] += 1
                    if vis:
                        stats[s, 1] += 1
                        rho[s] += g[j]
                if amb[j]:
                    stats[s, 2] += 1
                if frag and inc[j]:
                    stats[s, 3] += 1
                if amb[j] or (frag and inc[j]):
                    budget[s] += g[j]
    return OracleDensity(rho, budget, stats)


WORLD_UP = np.array([0.0, 1.0, 0.0])


def camera_basis(head):
    """Camera frame of a fixation, FP64: forward f = head / |head| (the head's view direction;
    without head tracking the gaze itself), right = f x up / |f x up| with the world's up
    (0, 1, 0), or (0, 0, 1) when the view is within 1e-6 of vertical; up' = right x f."""
    f = np.asarray(head, np.float32).astype(np.float64)
    f = f / math.sqrt(f @ f)
    up = WORLD_UP if abs(f @ WORLD_UP) < 1 - 1e-6 else np.array([0.0, 0.0, 1.0])
    x = np.cross(f, up); x /= math.sqrt(x @ x)
    y = np.cross(x, f)
    return x, y, f


def _quat_rotate(v, axis, ang):
    # q v q^-1 with q = cos(ang/2) + axis sin(ang/2), axis a unit vector (Appendix A)
    w, s_ = math.cos(ang / 2), math.sin(ang / 2)
    qv = s_ * np.asarray(axis, np.float64)
    t = 2.0 * np.cross(qv, v)
    return v + w * t + np.cross(qv, t)


def crop_bounds(r_cam, theta_deg, near):
    """Appendix A: the bounds l', r', b', t' on the near plane z = -n (camera coordinates:
    right x, up y, looking along -z) of the ellipse where the 4-sigma cone around the gaze
    r_cam meets that plane.  phi = atan(4 sigma); a0, a1 = r rotated by -+phi about
    u1 = r x i (i the camera's forward (0, 0, -1)), b0, b1 about u2 = r x u1; their hits
    A0, A1, B0, B1 with the plane give a = |A1 - A0| / 2, b = |B1 - B0| / 2; E = the gaze's
    hit, alpha = acos(j . ME / |ME|) (j the right vector, M the plane's centre); l', r' =
    E_x -+ sqrt(a^2 cos^2 alpha + b^2 sin^2 alpha), b', t' = E_y -+ sqrt(a^2 sin^2 alpha +
    b^2 cos^2 alpha).  When the gaze runs along i, u1 is taken along r x j instead (the
    ellipse is then a circle and alpha does not matter).  None when the cone reaches
    behind the camera (the crop is undefined)."""
    r = np.asarray(r_cam, np.float64); r = r / math.sqrt(r @ r)
    sigma = math.tan(math.radians(theta_deg))
    phi = math.atan(4.0 * sigma)
    i_fwd = np.array([0.0, 0.0, -1.0]); j_right = np.array([1.0, 0.0, 0.0])
    u1 = np.cross(r, i_fwd)
    if math.sqrt(u1 @ u1) < 1e-12:
        u1 = np.cross(r, j_right)
    u1 /= math.sqrt(u1 @ u1)
    u2 = np.cross(r, u1); u2 /= math.sqrt(u2 @ u2)

    def hit(v):
        return -near / v[2] * v[:2]
    rays = [_quat_rotate(r, u1, -phi), _quat_rotate(r, u1, phi), _quat_rotate(r, u2, -phi), _quat_rotate(r, u2, phi)]
    if r[2] >= 0 or any(v[2] >= 0 for v in rays):
        return None   # the cone reaches behind the camera: no crop
    A0, A1, B0, B1 = (hit(v) for v in rays)
    E = hit(r)
    a = math.sqrt((A1 - A0) @ (A1 - A0)) / 2.0
    b = math.sqrt((B1 - B0) @ (B1 - B0)) / 2.0
    me = math.sqrt(E @ E)
    alpha = math.acos(max(-1.0, min(1.0, E[0] / me))) if me > 0 else 0.0
    hx = math.sqrt(a * a * math.cos(alpha) ** 2 + b * b * math.sin(alpha) ** 2)
    hy = math.sqrt(a * a * math.sin(alpha) ** 2 + b * b * math.cos(alpha) ** 2)
    return E[0] - hx, E[0] + hx, E[1] - hy, E[1] + hy


def crop_cameras(gaze, head, theta_deg, near):
    """Per fixation [F][13]: right, up, forward (FP64) and l', r', b', t' of its crop; and
    whether the fixation is usable: a defined crop whose four corners lie less than 80
    degrees off the gaze (wider crops are refused rather than cut)."""
    gaze = np.asarray(gaze, np.float32).reshape(-1, 3)
    head = gaze if head is None else np.asarray(head, np.float32).reshape(-1, 3)
    out = np.zeros((len(gaze), 13)); out[:, 10] = out[:, 12] = 1.0
    ok = np.zeros(len(gaze), bool)
    for k in range(len(gaze)):
        x, y, f = camera_basis(head[k])
        g = gaze[k].astype(np.float64)
        rc = np.array([g @ x, g @ y, -(g @ f)])
        out[k, :3], out[k, 3:6], out[k, 6:9] = x, y, f
        cb = crop_bounds(rc, theta_deg, near)
        if cb is None:
            continue
        out[k, 9:] = cb
        rn = rc / math.sqrt(rc @ rc)
        corners = [np.array([cx, cy, -near]) for cx in cb[:2] for cy in cb[2:]]
        ok[k] = min(c @ rn / math.sqrt(c @ c) for c in corners) > math.cos(math.radians(80.0))
    return out, ok


@dataclass
class OracleZDensity:
    rho: np.ndarray      # float64 [n]
    budget: np.ndarray   # float64 [n]
    stats: np.ndarray    # int64 [n][4]: in the frustum, visible, ambiguous, 0
    zbuf: np.ndarray     # float64 [F][R][R] depth of the nearest surface per pixel (inf: none)
    zamb: np.ndarray     # bool [F][R][R] pixels a rasteriser could fill from another triangle
    cams: np.ndarray     # [F][13]
    ok: np.ndarray       # bool [F] fixations with a usable crop


def density_zbuffer(scene: Scene, pos, eye, gaze, dur, theta_deg, resolution=128, eps_depth=1e-2, near=0.05,
                    far=1000.0, head=None, nthreads=None) -> OracleZDensity:
    """The paper's own approximation (Sec. 3.2.2, 3.3.2, Appendix A): per fixation a camera
    at the eye looking along the head direction (the gaze without head tracking), cropped to
    the 4-sigma cone's bounds on the near plane (crop_bounds), a resolution x resolution
    z-buffer of the whole scene (depth of the nearest surface through each pixel centre,
    depths in [near, far]); a sample inside the cropped frustum (the NDC cube) gets the
    angular Gaussian of Sec. 3.2.1 (not cut at 4 sigma) when its depth D satisfies
    D - zbuf(pixel) <= eps_depth D.  Sums in FP64."""
    lib = _load()
    pos = np.ascontiguousarray(pos, np.float32).reshape(-1, 3)
    eye = np.ascontiguousarray(eye, np.float32).reshape(-1, 3)
    gaze = np.ascontiguousarray(gaze, np.float32).reshape(-1, 3)
    dur = np.ascontiguousarray(dur, np.float32).reshape(-1)
    F, n, R = len(eye), len(pos), int(resolution)
    cams, ok = crop_cameras(gaze, head, theta_deg, near)
    cams = np.ascontiguousarray(cams)
    dur = np.ascontiguousarray(np.where(ok, dur, np.float32(0)).astype(np.float32))   # refused: nothing
    zbuf = np.zeros((F, R, R)); zamb = np.zeros((F, R, R), np.uint8)
    rho = np.zeros(n); budget = np.zeros(n); stats = np.zeros((n, 4), np.int64)
    lib.or_density_zbuffer(scene._h, _ptr(pos, ctypes.c_float), n, _ptr(eye, ctypes.c_float),
                           _ptr(gaze, ctypes.c_float), _ptr(dur, ctypes.c_float), _ptr(cams, ctypes.c_double), F,
                           float(theta_deg), R, float(eps_depth), float(near), float(far),
                           int(nthreads or os.cpu_count() or 1), _ptr(zbuf, ctypes.c_double),
                           _ptr(zamb, ctypes.c_uint8), _ptr(rho, ctypes.c_double), _ptr(budget, ctypes.c_double),
                           _ptr(stats, ctypes.c_int64))
    zbuf[~ok] = np.inf
    return OracleZDensity(rho, budget, stats, zbuf, zamb.astype(bool), cams, ok)


def normalize(rho):
    lib = _load()
    rho = np.ascontiguousarray(rho, np.float64)
    out = np.zeros_like(rho)
    mx = lib.or_normalize(_ptr(rho, ctypes.c_double), len(rho), _ptr(out, ctypes.c_double))
    return out, mx
