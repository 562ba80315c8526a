"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds inputs: triangle meshes, eye trajectories, gaze rays
and durations.  It holds none of the density-map arithmetic (no areas,
sampling, Philox, angular kernel or visibility) and it is shared by the tests,
the benchmark and the smoke check; neither the oracle nor the HIP path import
each other through it.

Scenes (the paper's own scenes and eye-tracking recordings are not available;
these stand in for them, see the recipe in the design doc):
  * tiny_icosphere_scene .... one icosphere, subdivision level 3 (1,280 tris),
                              radius 0.5 m, 100 fixations from a shell 1.5-2.5 m;
  * paper_shaped_scene ...... four meshes, ~806k triangles (noise-displaced
                              icosphere, cube, torus knot, two-density
                              heightfield), 6,000 fixations from a head walk;
  * scale_up_scene .......... 25 displaced geodesic spheres (5M triangles),
                              50,000 fixations from 10 head walks;
  * batched_sessions ........ 64 independent sessions of uneven size.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    V: np.ndarray                 # float32 [nv][3]
    I: np.ndarray                 # int32 [nt][3]
    name: str = ""
    # analytic surface sampler used only to aim gaze rays: rng, n -> (points, normals)
    aim: object = None


@dataclass
class Fixations:
    eye: np.ndarray               # float32 [F][3]
    gaze: np.ndarray              # float32 [F][3], not necessarily unit length
    dur: np.ndarray               # float32 [F]


@dataclass
class Workload:
    name: str
    meshes: list
    fix: Fixations
    theta_deg: float
    k: float                      # samples per square metre
    seed: int
    occlusion: str                # "none" | "self" | "full"
    extra: dict = field(default_factory=dict)

    @property
    def n_triangles(self):
        return int(sum(len(m.I) for m in self.meshes))


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------

def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
                  [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    F = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return V / np.linalg.norm(V, axis=1, keepdims=True), F


def icosphere_unit(level: int):
    """Unit icosphere: each level splits every face in four, midpoints pushed to the sphere."""
    V, F = _icosahedron()
    for _ in range(level):
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
        e.sort(axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = V[uniq[:, 0]] + V[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = len(V)
        V = np.concatenate([V, mid])
        nf = len(F)
        ab, bc, ca = inv[:nf] + base, inv[nf:2 * nf] + base, inv[2 * nf:] + base
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        F = np.concatenate([np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1),
                            np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)])
    return V, F


def geodesic_unit(freq: int):
    """Class-I geodesic sphere: every icosahedron face cut into freq^2 triangles."""
    V0, F0 = _icosahedron()
    pts, tris = [], []
    base = 0
    ij = [(i, j) for i in range(freq + 1) for j in range(freq + 1 - i)]
    index = {p: n for n, p in enumerate(ij)}
    local = []
    for i in range(freq):
        for j in range(freq - i):
            local.append((index[(i, j)], index[(i + 1, j)], index[(i, j + 1)]))
            if i + j + 1 < freq:
                local.append((index[(i + 1, j)], index[(i + 1, j + 1)], index[(i, j + 1)]))
    local = np.array(local, np.int64)
    ij = np.array(ij, np.float64) / freq
    for a, b, c in F0:
        A, B, C = V0[a], V0[b], V0[c]
        P = A[None] + ij[:, :1] * (B - A)[None] + ij[:, 1:] * (C - A)[None]
        pts.append(P)
        tris.append(local + base)
        base += len(P)
    P = np.concatenate(pts)
    P /= np.linalg.norm(P, axis=1, keepdims=True)
    T = np.concatenate(tris)
    key = np.round(P * 1e9).astype(np.int64)
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    return P[first], inv.reshape(-1)[T]


def _noise_field(rng, octaves=4, waves=6, base_freq=3.0, gain=0.5):
    dirs, freqs, phases, amps = [], [], [], []
    for o in range(octaves):
        w = rng.normal(size=(waves, 3))
        w /= np.linalg.norm(w, axis=1, keepdims=True)
        dirs.append(w)
        freqs.append(np.full(waves, base_freq * 2.0 ** o))
        phases.append(rng.uniform(0, 2 * np.pi, waves))
        amps.append(np.full(waves, gain ** o / math.sqrt(waves)))
    D, Fq, Ph, Am = map(np.concatenate, (dirs, freqs, phases, amps))

    def f(p):
        p = np.asarray(p, np.float64)
        flat = p.reshape(-1, 3)
        return (np.sin((flat @ D.T) * Fq + Ph) * Am).sum(axis=1).reshape(p.shape[:-1])
    return f


def _sphere_aim(center, radius):
    c = np.asarray(center, np.float64)

    def aim(rng, n):
        d = rng.normal(size=(n, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        return c + radius * d, d
    return aim


def sphere_mesh(level=None, freq=None, radius=0.5, center=(0, 0, 0), displace=0.0, seed=0, name="sphere"):
    V, F = icosphere_unit(level) if level is not None else geodesic_unit(freq)
    r = np.full(len(V), radius)
    if displace:
        noise = _noise_field(np.random.default_rng(seed))
        n = noise(V)
        n = n / max(1e-12, np.abs(n).max())
        r = radius * (1.0 + displace * n)
    P = V * r[:, None] + np.asarray(center)[None]
    return Mesh(P.astype(np.float32), F.astype(np.int32), name, _sphere_aim(center, radius))


def cube_mesh(edge=0.5, center=(0, 0, 0), name="cube"):
    h = edge / 2.0
    c = np.asarray(center, np.float64)
    V = np.array([[x, y, z] for x in (-h, h) for y in (-h, h) for z in (-h, h)]) + c
    # faces wound counter-clockwise seen from outside
    quads = [(0, 1, 3, 2), (4, 6, 7, 5), (0, 4, 5, 1), (2, 3, 7, 6), (0, 2, 6, 4), (1, 5, 7, 3)]
    F = []
    for a, b, cc, d in quads:
        F += [(a, b, cc), (a, cc, d)]

    def aim(rng, n):
        face = rng.integers(0, 6, n)
        st = rng.uniform(-h, h, (n, 2))
        axis = face // 2
        sign = np.where(face % 2 == 0, -1.0, 1.0)
        P = np.zeros((n, 3)); N = np.zeros((n, 3))
        for a in range(3):
            m = axis == a
            o = [b for b in range(3) if b != a]
            P[m, a] = sign[m] * h
            P[m, o[0]] = st[m, 0]; P[m, o[1]] = st[m, 1]
            N[m, a] = sign[m]
        return P + c, N
    return Mesh(V.astype(np.float32), np.array(F, np.int32), name, aim)


def torus_knot_mesh(p=2, q=3, seg=1000, ring=100, R=0.3, r=0.12, tube=0.04, center=(0, 0, 0), name="torus_knot"):
    """Tube of radius `tube` around the (p,q) torus knot, seg x ring quads, lying in the x-z plane."""
    c = np.asarray(center, np.float64)

    def curve(phi):
        rr = R + r * np.cos(q * phi)
        return np.stack([rr * np.cos(p * phi), -r * np.sin(q * phi), rr * np.sin(p * phi)], -1)

    phi = np.arange(seg) * (2 * np.pi / seg)
    C = curve(phi)
    Tg = curve(phi + 1e-4) - curve(phi - 1e-4)
    Tg /= np.linalg.norm(Tg, axis=1, keepdims=True)
    up = np.array([0.0, 1.0, 0.0])
    N = np.cross(Tg, up)
    N /= np.linalg.norm(N, axis=1, keepdims=True)
    B = np.cross(Tg, N)
    psi = np.arange(ring) * (2 * np.pi / ring)
    off = np.cos(psi)[None, :, None] * N[:, None] + np.sin(psi)[None, :, None] * B[:, None]
    V = (C[:, None] + tube * off).reshape(-1, 3) + c
    i = np.arange(seg)[:, None]; j = np.arange(ring)[None, :]
    a = i * ring + j; b = ((i + 1) % seg) * ring + j
    cc = ((i + 1) % seg) * ring + (j + 1) % ring; d = i * ring + (j + 1) % ring
    F = np.concatenate([np.stack([a, b, cc], -1).reshape(-1, 3), np.stack([a, cc, d], -1).reshape(-1, 3)])
    # outward winding check on one face, flip all if needed
    v0, v1, v2 = V[F[0, 0]], V[F[0, 1]], V[F[0, 2]]
    if np.dot(np.cross(v1 - v0, v2 - v0), v0 - (C[0] + c)) < 0:
        F = F[:, [0, 2, 1]]

    def aim(rng, n):
        ph = rng.uniform(0, 2 * np.pi, n); ps = rng.uniform(0, 2 * np.pi, n)
        Cn = curve(ph)
        Tn = curve(ph + 1e-4) - curve(ph - 1e-4)
        Tn /= np.linalg.norm(Tn, axis=1, keepdims=True)
        Nn = np.cross(Tn, up); Nn /= np.linalg.norm(Nn, axis=1, keepdims=True)
        Bn = np.cross(Tn, Nn)
        o = np.cos(ps)[:, None] * Nn + np.sin(ps)[:, None] * Bn
        return Cn + tube * o + c, o
    return Mesh(V.astype(np.float32), F.astype(np.int32), name, aim)


def heightfield_mesh(size=2.0, fine=(256, 512), coarse=(64, 128), amp=0.05, center=(0, 0, 0), seed=1,
                     name="heightfield"):
    """size x size terrain in the x-z plane (y up).  The left half (x < 0) has fine[0] x fine[1]
    cells, the right half coarse[0] x coarse[1] (16x fewer).  The relief fades to zero at the
    seam x = 0 so the two halves meet without a crack."""
    c = np.asarray(center, np.float64)
    noise = _noise_field(np.random.default_rng(seed), base_freq=2.0)
    h2 = size / 2.0

    def height(x, z):
        fade = np.clip(np.abs(x) / (0.1 * size), 0.0, 1.0)
        p = np.stack([x, np.zeros_like(x), z], -1)
        return amp * fade * noise(p)

    def grid(x0, x1, nx, nz):
        xs = np.linspace(x0, x1, nx + 1); zs = np.linspace(-h2, h2, nz + 1)
        X, Z = np.meshgrid(xs, zs, indexing="ij")
        P = np.stack([X, height(X, Z), Z], -1).reshape(-1, 3)
        i = np.arange(nx)[:, None]; j = np.arange(nz)[None, :]
        a = i * (nz + 1) + j; b = (i + 1) * (nz + 1) + j
        F = np.concatenate([np.stack([a, a + 1, b + 1], -1).reshape(-1, 3),
                            np.stack([a, b + 1, b], -1).reshape(-1, 3)])
        return P, F

    P1, F1 = grid(-h2, 0.0, *fine)
    P2, F2 = grid(0.0, h2, *coarse)
    V = np.concatenate([P1, P2]) + c
    F = np.concatenate([F1, F2 + len(P1)])
    # wind so that normals point up (+y)
    v0, v1, v2 = V[F[0, 0]], V[F[0, 1]], V[F[0, 2]]
    if np.cross(v1 - v0, v2 - v0)[1] < 0:
        F = F[:, [0, 2, 1]]

    def aim(rng, n):
        x = rng.uniform(-h2, h2, n); z = rng.uniform(-h2, h2, n)
        P = np.stack([x, height(x, z), z], -1) + c
        N = np.tile([0.0, 1.0, 0.0], (n, 1))
        return P, N
    return Mesh(V.astype(np.float32), F.astype(np.int32), name, aim)


# ----------------------------------------------------------------------------
# fixations
# ----------------------------------------------------------------------------

def _jitter(rng, d, deg):
    """Rotate each direction by a 2-D isotropic Gaussian angle (std `deg` per axis)."""
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    a = np.where(np.abs(d[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    u = np.cross(d, a); u /= np.linalg.norm(u, axis=1, keepdims=True)
    v = np.cross(d, u)
    ang = np.radians(deg) * rng.normal(size=(len(d), 2))
    return d + np.tan(ang[:, :1]) * u + np.tan(ang[:, 1:]) * v


def _aim_targets(rng, meshes, eyes, weights, front_facing=True, tries=32):
    """One gaze target per eye: an object picked by `weights`, then a point of its analytic
    surface; with front_facing, retried until the outward normal faces the eye."""
    n = len(eyes)
    obj = rng.choice(len(meshes), size=n, p=np.asarray(weights) / np.sum(weights))
    T = np.zeros((n, 3))
    for m, mesh in enumerate(meshes):
        idx = np.nonzero(obj == m)[0]
        todo = idx
        for _ in range(tries):
            if len(todo) == 0:
                break
            P, N = mesh.aim(rng, len(todo))
            T[todo] = P
            if not front_facing:
                todo = todo[:0]
                break
            ok = np.einsum("ij,ij->i", eyes[todo] - P, N) > 0
            todo = todo[~ok]
    return T


def shell_fixations(rng, meshes, F, center=(0, 0, 0), r_in=1.5, r_out=2.5, jitter_deg=1.0, dur=1.0):
    """Eyes uniform in the volume of a spherical shell; gaze at uniformly chosen surface points."""
    u = rng.uniform(r_in ** 3, r_out ** 3, F) ** (1.0 / 3.0)
    d = rng.normal(size=(F, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    eye = np.asarray(center)[None] + u[:, None] * d
    tgt = _aim_targets(rng, meshes, eye, np.ones(len(meshes)), front_facing=False)
    gaze = _jitter(rng, tgt - eye, jitter_deg)
    t = np.full(F, dur) if np.isscalar(dur) else rng.uniform(dur[0], dur[1], F)
    return Fixations(eye.astype(np.float32), gaze.astype(np.float32), t.astype(np.float32))


def walk_fixations(rng, meshes, F, weights, r_in, r_out, height=1.6, step=0.05, center=(0, 0, 0),
                   jitter_deg=1.0, dur=(0.1, 0.5)):
    """Head random walk at eye height `height`: `step` metres per fixation at a uniformly
    random heading, reflected to stay in the annulus r_in..r_out around `center`; gaze at a
    front-facing surface point plus Gaussian angular jitter; durations uniform in `dur`."""
    c = np.asarray(center, np.float64)
    ang = rng.uniform(0, 2 * np.pi)
    rad = 0.5 * (r_in + r_out)
    pos = np.array([rad * math.cos(ang), rad * math.sin(ang)])
    eyes = np.zeros((F, 3))
    for i in range(F):
        h = rng.uniform(0, 2 * np.pi)
        nxt = pos + step * np.array([math.cos(h), math.sin(h)])
        r = np.linalg.norm(nxt)
        if r > r_out:
            nxt *= (2 * r_out - r) / r
        elif r < r_in:
            nxt *= (2 * r_in - r) / max(r, 1e-9)
        pos = nxt
        eyes[i] = [c[0] + pos[0], height, c[2] + pos[1]]
    tgt = _aim_targets(rng, meshes, eyes, weights, front_facing=True)
    gaze = _jitter(rng, tgt - eyes, jitter_deg)
    t = rng.uniform(dur[0], dur[1], F)
    return Fixations(eyes.astype(np.float32), gaze.astype(np.float32), t.astype(np.float32))


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def start_times(dur, gap=0.03):
    """Start time (s, float64) of each fixation of a recording that plays them in order,
    each followed by a saccade of `gap` seconds: t_0 = 0, t_f = sum over j < f of
    (dur_j + gap)."""
    d = np.asarray(dur, np.float64).reshape(-1) + gap
    return np.concatenate([[0.0], np.cumsum(d)[:-1]]) if len(d) else np.zeros(0)


def plate_mesh(size=0.8, cells=8, name="plate"):
    """Square grid of cells x cells quads in the local x-y plane, centred at the origin."""
    h = size / 2.0
    g = np.linspace(-h, h, cells + 1)
    V = np.array([[x, y, 0.0] for y in g for x in g])
    F = []
    for j in range(cells):
        for i in range(cells):
            a = j * (cells + 1) + i
            F += [(a, a + 1, a + cells + 2), (a, a + cells + 2, a + cells + 1)]

    def aim(rng, n):
        P = np.zeros((n, 3)); P[:, :2] = rng.uniform(-h, h, (n, 2))
        N = np.zeros((n, 3)); N[:, 2] = 1.0
        return P, N
    return Mesh(V.astype(np.float32), np.array(F, np.int32), name, aim)


def _rot(axis, ang):
    a = np.asarray(axis, np.float64); a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * (K @ K)


def posed_scene(seed=0, F=40, k=6000.0):
    """Objects that move during a recording: a sphere (R 0.4 m, 1,280 triangles) sliding and
    turning, a cube (0.4 m, scaled by 1.25) orbiting and tumbling, and a 0.8 m plate that
    slides back and forth in front of the sphere; each mesh in its own frame, centred at its
    origin.  pose [F][3][12]: row-major 3x4 (A | b), mesh frame -> world at each fixation's
    start time.  Eyes in the 1.8-2.6 m shell on the -y side, gaze at a surface point of a
    posed object with 1 degree jitter, t ~ U[0.1, 0.5] s; theta = 1 degree."""
    rng = np.random.default_rng(seed)
    meshes = [sphere_mesh(level=3, radius=0.4, name="sphere"), cube_mesh(0.4, name="cube"),
              plate_mesh(0.8, 8, name="plate")]
    dur = rng.uniform(0.1, 0.5, F)
    t = start_times(dur)
    pose = np.zeros((F, 3, 3, 4))
    for f in range(F):
        tau = t[f]
        pose[f, 0, :, :3] = _rot((0, 0, 1), 0.2 * tau)
        pose[f, 0, :, 3] = (0.6 * math.sin(0.3 * tau), 0.3, 0.0)
        pose[f, 1, :, :3] = 1.25 * _rot((1, 1, 0), 0.5 * tau)
        pose[f, 1, :, 3] = (0.9 * math.cos(0.4 * tau), 0.9 * math.sin(0.4 * tau), 0.5)
        pose[f, 2, :, :3] = _rot((1, 0, 0), math.pi / 2)
        pose[f, 2, :, 3] = (-0.2 + 0.8 * math.sin(0.9 * tau), -0.45, 0.0)
    u = rng.uniform(1.8 ** 3, 2.6 ** 3, F) ** (1.0 / 3.0)
    d = rng.normal(size=(F, 3)); d /= np.linalg.norm(d, axis=1, keepdims=True)
    d[:, 1] = -np.abs(d[:, 1]) - 0.5
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    eye = u[:, None] * d
    obj = rng.integers(0, 3, F)
    tgt = np.zeros((F, 3))
    for f in range(F):
        P, _ = meshes[obj[f]].aim(rng, 1)
        A = pose[f, obj[f], :, :3]; b = pose[f, obj[f], :, 3]
        tgt[f] = A @ P[0] + b
    gaze = _jitter(rng, tgt - eye, 1.0)
    fix = Fixations(eye.astype(np.float32), gaze.astype(np.float32), dur.astype(np.float32))
    return Workload("posed", meshes, fix, 1.0, k, seed, "full",
                    {"pose": pose.reshape(F, 3, 12).astype(np.float32), "time": t})


def tiny_icosphere_scene(seed=0):
    """Icosphere level 3 (1,280 triangles), R = 0.5 m at the origin, 2,000 samples/m^2,
    Philox seed 0; 100 fixations, eyes uniform in the 1.5-2.5 m shell, gaze at uniform
    surface points with 1 degree jitter, t = 1 s; theta = 1 degree; self occlusion."""
    mesh = sphere_mesh(level=3, radius=0.5, name="icosphere_l3")
    fix = shell_fixations(np.random.default_rng(1000 + seed), [mesh], 100)
    return Workload("icosphere-l3 1280 tris, 2000/m^2, 100 fixations", [mesh], fix, 1.0, 2000.0, 0, "self")


def paper_shaped_meshes(seed=0):
    sphere = sphere_mesh(level=7, radius=0.5, center=(-0.5, 0.62, -0.45), displace=0.05, seed=seed + 11,
                         name="displaced_icosphere_l7")
    cube = cube_mesh(0.5, center=(0.55, 0.2505, -0.45))
    knot = torus_knot_mesh(center=(0.0, 0.62, 0.45))
    hf = heightfield_mesh(center=(0.0, 0.0, 0.0), seed=seed + 12)
    return [sphere, cube, knot, hf]


def paper_shaped_scene(seed=0, n_samples=2_000_000, F=6000, area_estimate=None):
    """~806k triangles in four meshes, 2M samples at one uniform rate, 6,000 fixations from a
    head walk (5 cm steps, eye height 1.6 m), theta = 1 degree, full inter-mesh occlusion.
    `k` is set from the total area so that about n_samples samples result; the caller passes
    the area (computed by whichever side it is testing) or the nominal estimate is used."""
    meshes = paper_shaped_meshes(seed)
    fix = walk_fixations(np.random.default_rng(2000 + seed), meshes, F, weights=[3.2, 1.5, 1.6, 4.0],
                         r_in=1.8, r_out=2.6)
    A = area_estimate if area_estimate is not None else 10.5
    return Workload("paper-shaped 806k tris, 2M samples, 6000 fixations", meshes, fix, 1.0, n_samples / A,
                    0, "full", {"n_samples": n_samples})


def scale_up_meshes(seed=0, freq=100):
    meshes = []
    for gi in range(5):
        for gj in range(5):
            c = (1.5 * (gi - 2), 0.6, 1.5 * (gj - 2))
            meshes.append(sphere_mesh(freq=freq, radius=0.6, center=c, displace=0.04,
                                      seed=seed + 100 + 5 * gi + gj, name=f"geodesic_{gi}{gj}"))
    return meshes


def scale_up_scene(seed=0, n_samples=20_000_000, F=50_000, trajectories=10, freq=100):
    """25 displaced class-I geodesic spheres (frequency 100: 200k triangles each) on a 5x5 grid
    with 1.5 m spacing; 50,000 fixations from 10 head walks; theta = 1 degree; occlusion on."""
    meshes = scale_up_meshes(seed, freq)
    rng = np.random.default_rng(3000 + seed)
    parts = [walk_fixations(rng, meshes, F // trajectories, weights=np.ones(len(meshes)), r_in=4.2, r_out=5.5)
             for _ in range(trajectories)]
    fix = Fixations(*[np.concatenate([getattr(p, a) for p in parts]) for a in ("eye", "gaze", "dur")])
    return Workload("scale-up 5M tris, 20M samples, 50k fixations", meshes, fix, 1.0,
                    n_samples / (25 * 4.6), 0, "full", {"n_samples": n_samples})


def batched_sessions(n_sessions=64, seed=0, t_range=(10_000, 400_000), f_range=(500, 20_000),
                     k_range=(1000.0, 8000.0), theta_range=(0.5, 2.0)):
    """Independent sessions of uneven size: one displaced sphere or heightfield each, triangle
    count log-uniform in t_range, fixation count log-uniform in f_range, samples/m^2 uniform in
    k_range, theta uniform in theta_range (degrees)."""
    rng = np.random.default_rng(4000 + seed)
    out = []
    for s in range(n_sessions):
        T = int(math.exp(rng.uniform(math.log(t_range[0]), math.log(t_range[1]))))
        F = int(math.exp(rng.uniform(math.log(f_range[0]), math.log(f_range[1]))))
        k = float(rng.uniform(*k_range)); th = float(rng.uniform(*theta_range))
        if rng.uniform() < 0.6:
            freq = max(2, int(round(math.sqrt(T / 20.0))))
            R = float(rng.uniform(0.3, 0.6))
            mesh = sphere_mesh(freq=freq, radius=R, displace=0.04, seed=seed * 1000 + s)
            fix = shell_fixations(rng, [mesh], F, r_in=3 * R, r_out=5 * R, dur=(0.1, 0.5))
        else:
            side = float(rng.uniform(1.0, 2.0))
            cells = max(4, int(math.sqrt(T / 2.0)))
            half = max(2, cells // 2)
            mesh = heightfield_mesh(size=side, fine=(half, cells), coarse=(max(1, half // 4), max(1, cells // 4)),
                                    seed=seed * 1000 + s)
            fix = walk_fixations(rng, [mesh], F, weights=[1.0], r_in=0.6 * side, r_out=1.2 * side,
                                 height=1.6, dur=(0.1, 0.5))
        out.append(Workload(f"session{s}", [mesh], fix, th, k, s, "full"))
    return out
