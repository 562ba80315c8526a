"""Python binding of the gfx950 density-map library (include/gazemap.h).

Argument marshalling only: every step runs in the HIP kernels of libgazemap.so.
Torch is used for device memory and the current HIP stream.  The library must
be built first (``__graft_entry__.build()`` or ``python -m
paper_2601_07571_amd.build``); importing this module fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgazemap.so")

GM_OK = 0
STATUS = {0: "GM_OK", -1: "GM_ERR_INVALID_ARGUMENT", -2: "GM_ERR_OUT_OF_MEMORY", -3: "GM_ERR_DEVICE",
          -4: "GM_ERR_CAPACITY", -5: "GM_ERR_NOT_READY", -99: "GM_ERR_INTERNAL"}
OCC = {"none": 0, "self": 1, "full": 2}
GM_ERR_CAPACITY = -4
# limits of accumulate_density_noalloc (include/gazemap.h)
NOALLOC_MAX_POINTS = 524288
NOALLOC_MAX_FIXATIONS = 65536

# exported symbols of include/gazemap.h
SYMBOLS = ("gm_last_error", "gm_version", "gm_scene_create", "gm_scene_destroy", "gm_scene_info",
           "gm_count_surface_samples", "build_surface_samples", "gm_count_lattice_samples",
           "build_lattice_samples", "accumulate_density",
           "gm_debug_pair_values", "gm_debug_pair_visibility", "gm_debug_sqrt_f64", "gm_profile_enable", "gm_profile_read",
           "gm_density_stats", "gm_field_create", "gm_field_destroy", "gm_field_set_params",
           "gm_field_get_params", "gm_field_train", "gm_field_info", "gm_field_gradient", "gm_field_predict", "query_density",
           "gm_batch_create", "gm_batch_run", "gm_batch_info", "gm_batch_destroy",
           "gm_map_create", "gm_map_add", "gm_map_add_posed", "gm_map_read", "gm_map_reset", "gm_map_info",
           "gm_map_destroy", "gm_export_samples", "gm_render_zbuffers", "accumulate_density_zbuffer",
           "gm_density_counters", "gm_debug_adam_step", "gm_scene_mesh_closed", "gm_scene_set_mesh_closed",
           "gm_mesh_closed", "accumulate_density_noalloc")
GM_MAP_POSED = 4

# one exported sample (gm_export_record), 48 bytes
EXPORT_DTYPE = np.dtype([("value", "<f4"), ("value_norm", "<f4"), ("mesh", "<i4"), ("triangle", "<i4"),
                         ("bary", "<f4", (2,)), ("local", "<f4", (3,)), ("world", "<f4", (3,))])


class GazemapError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Mesh(ctypes.Structure):
    _fields_ = [("vertices", ctypes.c_void_p), ("indices", ctypes.c_void_p),
                ("n_vertices", ctypes.c_int32), ("n_triangles", ctypes.c_int32)]


class _Fix(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_void_p), ("gaze", ctypes.c_void_p), ("duration", ctypes.c_void_p),
                ("n", ctypes.c_int32)]


class _TrainParams(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("lr_final", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("holdout", ctypes.c_float), ("max_rel_l2", ctypes.c_float),
                ("target_max", ctypes.c_float), ("seed", ctypes.c_uint64)]


class _ZParams(ctypes.Structure):
    _fields_ = [("resolution", ctypes.c_int32), ("depth_eps", ctypes.c_float), ("near_plane", ctypes.c_float),
                ("far_plane", ctypes.c_float), ("head", ctypes.c_void_p)]


class _Session(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("pos", ctypes.c_void_p), ("tri", ctypes.c_void_p),
                ("mesh", ctypes.c_void_p), ("n", ctypes.c_int64), ("fix", _Fix), ("theta_deg", ctypes.c_double),
                ("flags", ctypes.c_uint32), ("density", ctypes.c_void_p), ("density_norm", ctypes.c_void_p),
                ("max_out", ctypes.c_void_p)]


FIELD_PARAMS = 18753

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgazemap.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2601_07571_amd.build`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32, u64, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_double)
    lib.gm_last_error.restype = ctypes.c_char_p
    lib.gm_version.restype = i32
    lib.gm_scene_create.argtypes = [ctypes.POINTER(_Mesh), i32, ctypes.POINTER(vp)]
    lib.gm_scene_destroy.argtypes = [vp]
    lib.gm_scene_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i64),
                                  ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    lib.gm_count_surface_samples.argtypes = [vp, dbl, ctypes.POINTER(i64), vp]
    lib.build_surface_samples.argtypes = [vp, dbl, u64, vp, vp, vp, vp, i64, ctypes.POINTER(i64), vp]
    lib.gm_count_lattice_samples.argtypes = [vp, dbl, ctypes.POINTER(i64), vp]
    lib.build_lattice_samples.argtypes = [vp, dbl, vp, vp, vp, vp, i64, ctypes.POINTER(i64), vp]
    lib.accumulate_density.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(_Fix), dbl, u32, vp, vp, vp, vp]
    lib.gm_debug_pair_values.argtypes = [vp, i64, ctypes.POINTER(_Fix), dbl, vp, vp, i64, vp, vp]
    lib.gm_debug_sqrt_f64.argtypes = [vp, vp, i64, vp]
    lib.gm_debug_pair_visibility.argtypes = [vp, vp, vp, vp, i64, vp, vp, i32, vp, vp, i64, u32, vp, vp]
    lib.gm_profile_enable.argtypes = [vp, i32]
    lib.gm_density_stats.argtypes = [vp, ctypes.POINTER(i64)]
    lib.gm_density_counters.argtypes = [vp, ctypes.POINTER(i64), i32]
    lib.gm_scene_mesh_closed.argtypes = [vp, ctypes.POINTER(ctypes.c_uint8)]
    lib.gm_scene_set_mesh_closed.argtypes = [vp, i32, i32]
    lib.gm_mesh_closed.argtypes = [vp, i32, vp, i32]
    f32p = ctypes.POINTER(ctypes.c_float)
    lib.gm_field_create.argtypes = [vp, u64, dbl, ctypes.POINTER(vp)]
    lib.gm_field_destroy.argtypes = [vp]
    lib.gm_field_set_params.argtypes = [vp, f32p]
    lib.gm_field_get_params.argtypes = [vp, f32p]
    lib.gm_field_train.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(_TrainParams), vp]
    lib.gm_field_info.argtypes = [vp, f32p, ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(dbl),
                                  ctypes.POINTER(i64)]
    lib.gm_field_gradient.argtypes = [vp, i32, vp, vp, i64, f32p, ctypes.POINTER(dbl)]
    lib.gm_field_predict.argtypes = [vp, vp, vp, i64, vp, vp]
    f32 = ctypes.c_float
    lib.accumulate_density_noalloc.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(_Fix), dbl, u32, vp, vp, vp,
                                               vp]
    lib.gm_noalloc_scratch_bytes.restype = i64
    lib.gm_noalloc_scratch_bytes.argtypes = []
    lib.gm_debug_adam_step.argtypes = [vp, vp, vp, vp, i64, i32, f32, f32, f32, f32, vp]
    lib.gm_batch_create.argtypes = [ctypes.POINTER(_Session), i32, ctypes.c_char_p, i32, ctypes.POINTER(vp), vp]
    lib.gm_batch_run.argtypes = [vp, vp]
    lib.gm_batch_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.POINTER(i32)]
    lib.gm_batch_destroy.argtypes = [vp]
    lib.query_density.argtypes = [vp, vp, ctypes.POINTER(_Fix), dbl, u32, vp, vp, vp, i64, dbl, vp, vp, vp]
    lib.gm_profile_read.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.gm_map_create.argtypes = [vp, vp, vp, vp, i64, dbl, u32, dbl, ctypes.POINTER(vp), vp]
    lib.gm_map_add.argtypes = [vp, ctypes.POINTER(_Fix), vp, dbl, dbl, vp]
    lib.gm_map_add_posed.argtypes = [vp, ctypes.POINTER(_Fix), vp, vp, dbl, dbl, vp]
    lib.gm_map_read.argtypes = [vp, vp, vp, vp, vp]
    lib.gm_export_samples.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i64, vp, vp]
    lib.gm_render_zbuffers.argtypes = [vp, ctypes.POINTER(_Fix), dbl, ctypes.POINTER(_ZParams), vp, vp]
    lib.accumulate_density_zbuffer.argtypes = [vp, vp, i64, ctypes.POINTER(_Fix), dbl, ctypes.POINTER(_ZParams),
                                               vp, vp, vp, vp]
    lib.gm_map_reset.argtypes = [vp, vp]
    lib.gm_map_info.argtypes = [vp, ctypes.POINTER(i64)]
    lib.gm_map_destroy.argtypes = [vp]
    for name in SYMBOLS[2:]:
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(status):
    if status != GM_OK:
        raise GazemapError(status, _lib.gm_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: this library runs on MI355X (gfx950) only")
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, dtype, shape_last=None):
    torch = _torch()
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t))
    t = t.to(device="cuda", dtype=dtype).contiguous()
    if shape_last is not None:
        t = t.reshape(-1, shape_last)
    return t


@dataclass
class Samples:
    tri: object    # int32 [N] scene-global triangle
    mesh: object   # int32 [N]
    bary: object   # float32 [N][2]
    pos: object    # float32 [N][3]


@dataclass
class Density:
    density: object       # float32 [n], raw rho
    density_norm: object  # float32 [n], rho / max
    max: object           # float32 [1] (device)


class Fixations:
    """Device copies of eye [F][3], gaze [F][3], duration [F]."""

    def __init__(self, eye, gaze, duration):
        torch = _torch()
        self.eye = _dev(eye, torch.float32, 3)
        self.gaze = _dev(gaze, torch.float32, 3)
        self.duration = _dev(duration, torch.float32).reshape(-1)
        self.n = int(self.eye.shape[0])
        self._c = _Fix(self.eye.data_ptr(), self.gaze.data_ptr(), self.duration.data_ptr(), self.n)

    def subset(self, begin, end):
        return Fixations(self.eye[begin:end], self.gaze[begin:end], self.duration[begin:end])


class Scene:
    """A set of triangle meshes on the current device with its occlusion BVH."""

    def __init__(self, meshes):
        lib = load_library()
        _torch()
        self._keep = []
        arr = (_Mesh * len(meshes))()
        self.n_triangles_per_mesh = []
        for i, (V, I) in enumerate(meshes):
            V = np.ascontiguousarray(V, np.float32)
            I = np.ascontiguousarray(I, np.int32)
            self._keep += [V, I]
            arr[i] = _Mesh(V.ctypes.data, I.ctypes.data, len(V), len(I))
            self.n_triangles_per_mesh.append(len(I))
        h = ctypes.c_void_p()
        _check(lib.gm_scene_create(arr, len(meshes), ctypes.byref(h)))
        self._h = h
        self._keep = []
        self.n_meshes = len(meshes)

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gm_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def info(self):
        T = ctypes.c_int64(); M = ctypes.c_int32(); nodes = ctypes.c_int64(); depth = ctypes.c_int32()
        bbox = (ctypes.c_float * 6)()
        _check(_lib.gm_scene_info(self._h, ctypes.byref(T), ctypes.byref(M), ctypes.byref(nodes),
                                  ctypes.byref(depth), bbox))
        return {"n_triangles": T.value, "n_meshes": M.value, "bvh_nodes": nodes.value,
                "bvh_depth": depth.value, "bbox": list(bbox)}

    def density_stats(self):
        """Counters of the last accumulate call: in-cone pairs, visible pairs, traversals,
        node visits, triangle tests (wave level), pairs settled by the back-face rule,
        (work item, fixation) pairs that passed the tile cone test."""
        out = (ctypes.c_int64 * 7)()
        _check(_lib.gm_density_counters(self._h, out, 7))
        return dict(zip(("in_cone", "visible", "traversals", "node_visits", "triangle_tests", "backface",
                         "gate_fixations"), out[:]))

    def mesh_closed(self):
        """Per mesh: whether the visibility test treats it as bounding a solid."""
        out = (ctypes.c_uint8 * self.info()["n_meshes"])()
        _check(_lib.gm_scene_mesh_closed(self._h, out))
        return np.array(out[:], dtype=bool)

    def set_mesh_closed(self, mesh, closed):
        _check(_lib.gm_scene_set_mesh_closed(self._h, int(mesh), 1 if closed else 0))

    def profile(self, on=True):
        _check(_lib.gm_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, stage):
        """(total milliseconds, launches) of a stage since profiling was enabled."""
        ms = ctypes.c_double(0.0); n = ctypes.c_int64(0)
        _check(_lib.gm_profile_read(self._h, stage.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def count_samples(self, samples_per_m2):
        out = (ctypes.c_int64 * self.n_meshes)()
        _check(_lib.gm_count_surface_samples(self._h, float(samples_per_m2), out, _stream()))
        return np.array(out[:], np.int64)

    def build_samples(self, samples_per_m2, seed=0, capacity=None, out: Samples | None = None):
        torch = _torch()
        if out is not None:
            tri, mesh, bary, pos = out.tri, out.mesh, out.bary, out.pos
            capacity = int(pos.shape[0])
        else:
            if capacity is None:
                capacity = int(self.count_samples(samples_per_m2).sum())
            tri = torch.empty(capacity, dtype=torch.int32, device="cuda")
            mesh = torch.empty(capacity, dtype=torch.int32, device="cuda")
            bary = torch.empty((capacity, 2), dtype=torch.float32, device="cuda")
            pos = torch.empty((capacity, 3), dtype=torch.float32, device="cuda")
        n = ctypes.c_int64(0)
        _check(_lib.build_surface_samples(self._h, float(samples_per_m2), int(seed) & (2 ** 64 - 1), _ptr(tri),
                                          _ptr(mesh), _ptr(bary), _ptr(pos), capacity, ctypes.byref(n),
                                          _stream()))
        N = n.value
        return Samples(tri[:N], mesh[:N], bary[:N], pos[:N])

    def count_lattice(self, samples_per_m2):
        """Per-mesh point counts of the paper's lattice sampler (host int64 array)."""
        out = (ctypes.c_int64 * self.n_meshes)()
        _check(_lib.gm_count_lattice_samples(self._h, float(samples_per_m2), out, _stream()))
        return np.array(out[:], np.int64)

    def build_lattice(self, samples_per_m2, capacity=None, out: Samples | None = None):
        """Every lattice point of the scene (mesh, triangle, then index order)."""
        torch = _torch()
        if out is not None:
            tri, mesh, bary, pos = out.tri, out.mesh, out.bary, out.pos
            capacity = int(pos.shape[0])
        else:
            if capacity is None:
                capacity = int(self.count_lattice(samples_per_m2).sum())
            tri = torch.empty(capacity, dtype=torch.int32, device="cuda")
            mesh = torch.empty(capacity, dtype=torch.int32, device="cuda")
            bary = torch.empty((capacity, 2), dtype=torch.float32, device="cuda")
            pos = torch.empty((capacity, 3), dtype=torch.float32, device="cuda")
        n = ctypes.c_int64(0)
        _check(_lib.build_lattice_samples(self._h, float(samples_per_m2), _ptr(tri), _ptr(mesh), _ptr(bary),
                                          _ptr(pos), capacity, ctypes.byref(n), _stream()))
        N = n.value
        return Samples(tri[:N], mesh[:N], bary[:N], pos[:N])

    def accumulate(self, pos, fix: Fixations, theta_deg, occlusion="full", tri=None, mesh=None, out=None):
        torch = _torch()
        pos = _dev(pos, torch.float32, 3)
        tri = _dev(tri, torch.int32)
        mesh = _dev(mesh, torch.int32)
        n = int(pos.shape[0])
        if out is None:
            out = Density(torch.empty(n, dtype=torch.float32, device="cuda"),
                          torch.empty(n, dtype=torch.float32, device="cuda"),
                          torch.empty(1, dtype=torch.float32, device="cuda"))
        _check(_lib.accumulate_density(self._h, _ptr(pos), _ptr(tri), _ptr(mesh), n, ctypes.byref(fix._c),
                                       float(theta_deg), OCC[occlusion] if isinstance(occlusion, str) else occlusion,
                                       _ptr(out.density), _ptr(out.density_norm), _ptr(out.max), _stream()))
        return out

    def accumulate_noalloc(self, pos, fix: Fixations, theta_deg, occlusion="full", tri=None, mesh=None, out=None):
        """accumulate() through accumulate_density_noalloc: no device allocation inside the
        call (the caller passes `out`; its intermediate buffers are the library's fixed
        per-device array)."""
        torch = _torch()
        pos = _dev(pos, torch.float32, 3)
        tri = _dev(tri, torch.int32)
        mesh = _dev(mesh, torch.int32)
        n = int(pos.shape[0])
        if out is None:
            out = Density(torch.empty(n, dtype=torch.float32, device="cuda"),
                          torch.empty(n, dtype=torch.float32, device="cuda"),
                          torch.empty(1, dtype=torch.float32, device="cuda"))
        _check(_lib.accumulate_density_noalloc(self._h, _ptr(pos), _ptr(tri), _ptr(mesh), n, ctypes.byref(fix._c),
                                               float(theta_deg),
                                               OCC[occlusion] if isinstance(occlusion, str) else occlusion,
                                               _ptr(out.density), _ptr(out.density_norm), _ptr(out.max),
                                               _stream()))
        return out

    def _zparams(self, resolution, depth_eps, near, far, head, n):
        torch = _torch()
        head = _dev(head, torch.float32, 3)
        if head is not None and int(head.shape[0]) != n:
            raise ValueError("head must hold one direction per fixation")
        return _ZParams(int(resolution), float(depth_eps), float(near), float(far),
                        None if head is None else head.data_ptr()), head

    def render_zbuffers(self, fix: Fixations, theta_deg, resolution=128, depth_eps=1e-2, near=0.05, far=1000.0,
                        head=None):
        """The paper's per-fixation z-buffers: float32 [F][R][R] nearest depths (+inf: none)."""
        torch = _torch()
        zp, keep = self._zparams(resolution, depth_eps, near, far, head, fix.n)
        out = torch.empty((fix.n, resolution, resolution), dtype=torch.float32, device="cuda")
        _check(_lib.gm_render_zbuffers(self._h, ctypes.byref(fix._c), float(theta_deg), ctypes.byref(zp), _ptr(out),
                                       _stream()))
        return out

    def accumulate_zbuffer(self, pos, fix: Fixations, theta_deg, resolution=128, depth_eps=1e-2, near=0.05,
                           far=1000.0, head=None, out=None):
        """The map under the paper's approximation (crop frustum + z-buffer test)."""
        torch = _torch()
        pos = _dev(pos, torch.float32, 3)
        n = int(pos.shape[0])
        zp, keep = self._zparams(resolution, depth_eps, near, far, head, fix.n)
        if out is None:
            out = Density(torch.empty(n, dtype=torch.float32, device="cuda"),
                          torch.empty(n, dtype=torch.float32, device="cuda"),
                          torch.empty(1, dtype=torch.float32, device="cuda"))
        _check(_lib.accumulate_density_zbuffer(self._h, _ptr(pos), n, ctypes.byref(fix._c), float(theta_deg),
                                               ctypes.byref(zp), _ptr(out.density), _ptr(out.density_norm),
                                               _ptr(out.max), _stream()))
        return out

    def pair_visibility(self, pos, eye, pair_s, pair_f, occlusion="full", tri=None, mesh=None, gaze=None):
        """Visibility of explicit (sample, fixation) pairs; with the fixations' gaze, the
        density kernel's own answer for each pair."""
        torch = _torch()
        pos = _dev(pos, torch.float32, 3)
        eye = _dev(eye, torch.float32, 3)
        gaze = _dev(gaze, torch.float32, 3)
        ps = _dev(pair_s, torch.int32); pf = _dev(pair_f, torch.int32)
        tri = _dev(tri, torch.int32); mesh = _dev(mesh, torch.int32)
        vis = torch.empty(int(ps.shape[0]), dtype=torch.uint8, device="cuda")
        _check(_lib.gm_debug_pair_visibility(self._h, _ptr(pos), _ptr(tri), _ptr(mesh), int(pos.shape[0]),
                                             _ptr(eye), _ptr(gaze), int(eye.shape[0]), _ptr(ps), _ptr(pf),
                                             int(ps.shape[0]), OCC[occlusion], _ptr(vis), _stream()))
        return vis


class DensityMap:
    """Incremental map over a fixed set of points (gm_map_* in include/gazemap.h):
    fixations are added in blocks, optionally filtered by a start-time window
    [t_begin, t_end); `read()` gives the map of everything added so far."""

    def __init__(self, scene: Scene, pos, theta_deg, occlusion="full", tri=None, mesh=None,
                 max_total_duration=86400.0, posed=False):
        lib = load_library()
        torch = _torch()
        pos = _dev(pos, torch.float32, 3)
        tri = _dev(tri, torch.int32)
        mesh = _dev(mesh, torch.int32)
        self.n = int(pos.shape[0])
        self.scene = scene  # the scene must outlive the map
        flags = OCC[occlusion] if isinstance(occlusion, str) else occlusion
        if posed:
            flags |= GM_MAP_POSED
        h = ctypes.c_void_p()
        _check(lib.gm_map_create(scene._h, _ptr(pos), _ptr(tri), _ptr(mesh), self.n, float(theta_deg), flags,
                                 float(max_total_duration), ctypes.byref(h), _stream()))
        self._h = h

    def add_posed(self, fix: Fixations, pose, time=None, window=None):
        """Accumulate `fix` with the meshes placed by `pose` (float32 [F][n_meshes][12],
        row-major 3x4 mesh frame -> world at each fixation's time)."""
        torch = _torch()
        pose = _dev(pose, torch.float32)
        if pose.numel() != fix.n * self.scene.n_meshes * 12:
            raise ValueError("pose must be [F][n_meshes][12]")
        t = _dev(time, torch.float64)
        if t is not None:
            t = t.reshape(-1)
            if t.shape[0] != fix.n:
                raise ValueError("time must hold one start time per fixation")
        t0, t1 = window if window is not None else (-math.inf, math.inf)
        _check(_lib.gm_map_add_posed(self._h, ctypes.byref(fix._c), _ptr(pose), _ptr(t), float(t0), float(t1),
                                     _stream()))
        self._keep = (fix, pose, t)
        return self

    def add(self, fix: Fixations, time=None, window=None):
        """Accumulate `fix`; with `time` (float64 [F], start times) only fixations with
        window[0] <= time < window[1] are taken."""
        torch = _torch()
        t = _dev(time, torch.float64)
        if t is not None:
            t = t.reshape(-1)
            if t.shape[0] != fix.n:
                raise ValueError("time must hold one start time per fixation")
        t0, t1 = window if window is not None else (-math.inf, math.inf)
        _check(_lib.gm_map_add(self._h, ctypes.byref(fix._c), _ptr(t), float(t0), float(t1), _stream()))
        self._keep = (fix, t)  # alive until the next call on this map's stream
        return self

    def read(self, out: Density | None = None):
        torch = _torch()
        if out is None:
            out = Density(torch.empty(self.n, dtype=torch.float32, device="cuda"),
                          torch.empty(self.n, dtype=torch.float32, device="cuda"),
                          torch.empty(1, dtype=torch.float32, device="cuda"))
        _check(_lib.gm_map_read(self._h, _ptr(out.density), _ptr(out.density_norm), _ptr(out.max), _stream()))
        return out

    def reset(self):
        _check(_lib.gm_map_reset(self._h, _stream()))

    def info(self):
        out = (ctypes.c_int64 * 4)()
        _check(_lib.gm_map_info(self._h, out))
        return {"added": out[0], "invalid": out[1], "over_budget": out[2], "budget_used_s": out[3] / 1024.0}

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gm_map_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()


def export_samples(scene: Scene, samples: Samples, density: Density, pose=None):
    """The export format of Sec. 3.3.3 on the device: uint8 [n][48] records
    (gm_export_record); `pose` float32 [n_meshes][12] places each mesh in the world
    (None: world = local).  `records_to_numpy` gives the host structured array."""
    torch = _torch()
    n = int(samples.pos.shape[0])
    out = torch.empty((n, EXPORT_DTYPE.itemsize), dtype=torch.uint8, device="cuda")
    pose = _dev(pose, torch.float32)
    _check(_lib.gm_export_samples(scene._h, _ptr(samples.tri), _ptr(samples.mesh), _ptr(samples.bary),
                                  _ptr(samples.pos), _ptr(density.density), _ptr(density.density_norm), _ptr(pose),
                                  n, _ptr(out), _stream()))
    return out


def records_to_numpy(records):
    return records.cpu().numpy().reshape(-1).view(EXPORT_DTYPE)


def write_csv(path, records):
    """One line per sample: value, value_norm, mesh, triangle, b1, b2, local xyz, world xyz."""
    r = records_to_numpy(records) if not isinstance(records, np.ndarray) else records
    cols = np.column_stack([r["value"], r["value_norm"], r["mesh"], r["triangle"], r["bary"], r["local"],
                            r["world"]])
    fmt = ["%.9g", "%.9g", "%d", "%d"] + ["%.9g"] * 8
    np.savetxt(path, cols, fmt=fmt, delimiter=",",
               header="value,value_norm,mesh,triangle,b1,b2,local_x,local_y,local_z,world_x,world_y,world_z",
               comments="")


def pair_values(pos, fix: Fixations, theta_deg, pair_s, pair_f):
    """g for explicit (sample, fixation) pairs, 0 outside the 4-sigma cone (no visibility)."""
    load_library()
    torch = _torch()
    pos = _dev(pos, torch.float32, 3)
    ps = _dev(pair_s, torch.int32); pf = _dev(pair_f, torch.int32)
    g = torch.empty(int(ps.shape[0]), dtype=torch.float32, device="cuda")
    _check(_lib.gm_debug_pair_values(_ptr(pos), int(pos.shape[0]), ctypes.byref(fix._c), float(theta_deg),
                                     _ptr(ps), _ptr(pf), int(ps.shape[0]), _ptr(g), _stream()))
    return g


def sqrt_f64(x):
    """The device's FP64 square root as the sampler evaluates it (diagnostic of its rounding)."""
    load_library()
    torch = _torch()
    x = _dev(x, torch.float64)
    y = torch.empty_like(x)
    _check(_lib.gm_debug_sqrt_f64(_ptr(x), _ptr(y), int(x.numel()), _stream()))
    return y


def adam_step(params, m, v, grad, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update with the training loop's kernel, in place on device float32 tensors
    (params, m, v); grad is zeroed afterwards.  step counts from 1."""
    load_library()
    for t in (params, m, v, grad):
        assert t.is_cuda and t.dtype == _torch().float32 and t.is_contiguous() and t.numel() == params.numel()
    _check(_lib.gm_debug_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(params.numel()), int(step),
                                   float(lr), float(beta1), float(beta2), float(eps), _stream()))


class Field:
    """Neural density field over a scene, one network per mesh (see include/gazemap.h).
    Parameters are [n_meshes][FIELD_PARAMS] (flat when the scene has one mesh)."""

    def __init__(self, scene: Scene, seed=0, max_cycles=32.0):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.gm_field_create(scene._h, int(seed) & (2 ** 64 - 1), float(max_cycles), ctypes.byref(h)))
        self.max_cycles = float(max_cycles)
        self._h = h
        self.scene = scene

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gm_field_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_params(self, params):
        M = self.scene.n_meshes
        p = np.ascontiguousarray(params, np.float32).reshape(-1)
        assert p.size == M * FIELD_PARAMS
        _check(_lib.gm_field_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self):
        M = self.scene.n_meshes
        p = np.zeros(M * FIELD_PARAMS, np.float32)
        _check(_lib.gm_field_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p if M == 1 else p.reshape(M, FIELD_PARAMS)

    def predict(self, pos, mesh=None, out=None):
        torch = _torch()
        pos = _dev(pos, torch.float32, 3)
        mesh = _dev(mesh, torch.int32)
        q = int(pos.shape[0])
        if out is None:
            out = torch.empty(q, dtype=torch.float32, device="cuda")
        _check(_lib.gm_field_predict(self._h, _ptr(pos), _ptr(mesh), q, _ptr(out), _stream()))
        return out

    def gradient(self, pos, target, net=0):
        torch = _torch()
        pos = _dev(pos, torch.float32, 3)
        target = _dev(target, torch.float32).reshape(-1)
        g = np.zeros(FIELD_PARAMS, np.float32)
        loss = ctypes.c_double(0.0)
        _check(_lib.gm_field_gradient(self._h, int(net), _ptr(pos), _ptr(target), int(pos.shape[0]),
                                      g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss)))
        return g, loss.value

    def train(self, pos, mesh, target, steps=2000, batch=16384, lr=2e-3, lr_final=1e-4, beta1=0.9, beta2=0.999,
              eps=1e-8, holdout=0.1, max_rel_l2=0.02, target_max=1.0, seed=0):
        torch = _torch()
        pos = _dev(pos, torch.float32, 3)
        mesh = _dev(mesh, torch.int32).reshape(-1)
        target = _dev(target, torch.float32).reshape(-1)
        P = _TrainParams(steps, batch, lr, lr_final, beta1, beta2, eps, holdout, max_rel_l2, target_max,
                         int(seed) & (2 ** 64 - 1))
        _check(_lib.gm_field_train(self._h, _ptr(pos), _ptr(mesh), _ptr(target), int(pos.shape[0]),
                                   ctypes.byref(P), _stream()))
        return self.info()

    def info(self):
        M = self.scene.n_meshes
        rel = np.zeros(M, np.float32); gate = np.zeros(M, np.uint8)
        loss = ctypes.c_double(0.0); steps = ctypes.c_int64(0)
        _check(_lib.gm_field_info(self._h, rel.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                  gate.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), ctypes.byref(loss),
                                  ctypes.byref(steps)))
        return {"rel_l2": rel, "gate": gate.astype(bool), "loss": loss.value, "steps": steps.value}


def query_density(field, scene: Scene, fix: Fixations, theta_deg, pos, tri=None, mesh=None, occlusion="full",
                  ref_max=0.0, out=None, used=None):
    """Normalised density at query points: the field where its mesh gate is open, else the plain path."""
    torch = _torch()
    pos = _dev(pos, torch.float32, 3)
    tri = _dev(tri, torch.int32)
    mesh = _dev(mesh, torch.int32)
    q = int(pos.shape[0])
    if out is None:
        out = torch.empty(q, dtype=torch.float32, device="cuda")
    if used is None:
        used = torch.empty(q, dtype=torch.uint8, device="cuda")
    _check(_lib.query_density(field._h if field is not None else None, scene._h, ctypes.byref(fix._c),
                              float(theta_deg), OCC[occlusion], _ptr(pos), _ptr(tri), _ptr(mesh), q, float(ref_max),
                              _ptr(out), _ptr(used), _stream()))
    return out, used


class Batch:
    """Many density maps in one persistent, graph-captured launch.

    sessions: list of dicts with keys scene, pos, fix (Fixations), theta_deg and optional
    tri, mesh, occlusion.  Output tensors are allocated here and rewritten by run()."""

    def __init__(self, sessions, tune_cache=None, tune=False):
        torch = _torch()
        load_library()
        self._keep = []
        arr = (_Session * len(sessions))()
        self.outputs = []
        for i, ss in enumerate(sessions):
            pos = _dev(ss["pos"], torch.float32, 3)
            tri = _dev(ss.get("tri"), torch.int32)
            mesh = _dev(ss.get("mesh"), torch.int32)
            n = int(pos.shape[0])
            out = Density(torch.empty(n, dtype=torch.float32, device="cuda"),
                          torch.empty(n, dtype=torch.float32, device="cuda"),
                          torch.empty(1, dtype=torch.float32, device="cuda"))
            fix = ss["fix"]
            self._keep += [pos, tri, mesh, fix, ss["scene"]]
            self.outputs.append(out)
            arr[i] = _Session(ss["scene"]._h.value, pos.data_ptr(), tri.data_ptr() if tri is not None else None,
                              mesh.data_ptr() if mesh is not None else None, n, fix._c, float(ss["theta_deg"]),
                              OCC[ss.get("occlusion", "full")], out.density.data_ptr(), out.density_norm.data_ptr(),
                              out.max.data_ptr())
        h = ctypes.c_void_p()
        _check(_lib.gm_batch_create(arr, len(sessions), tune_cache.encode() if tune_cache else None, 1 if tune else 0,
                                    ctypes.byref(h), _stream()))
        self._h = h

    def run(self):
        _check(_lib.gm_batch_run(self._h, _stream()))
        return self.outputs

    def info(self):
        spl = ctypes.c_int32(); fb = ctypes.c_int32(); ch = ctypes.c_int32(); items = ctypes.c_int64()
        ms = ctypes.c_double(); cached = ctypes.c_int32()
        _check(_lib.gm_batch_info(self._h, ctypes.byref(spl), ctypes.byref(fb), ctypes.byref(ch), ctypes.byref(items),
                                  ctypes.byref(ms), ctypes.byref(cached)))
        return {"samples_per_lane": spl.value, "fix_block": fb.value, "fix_per_chunk": ch.value,
                "work_items": items.value, "tuned_ms": ms.value, "from_cache": bool(cached.value)}

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.gm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()
