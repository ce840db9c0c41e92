"""Seeded synthetic scene generators shared by the CPU oracle and the HIP path.

This module only *creates inputs*: triangle meshes, materials, lights, the
caustic receiver rectangle, photon target spheres, cameras and wavelength
settings.  It holds none of the rendering arithmetic (no ray tests, no
optics, no random-number streams of the method); both implementations
receive the arrays built here and compute everything else on their own.

Units are metres, the world is right-handed with +z up.  Object id 0 is
reserved for "no hit"; every triangle carries an object id >= 1 and each
object has exactly one material.

The scenes stand in for the paper's dataset (1920x1080 images of glass
objects with caustics, Sec. IV-A); its HDRI maps, backdrops and prop assets
are not available, so procedural geometry of the same flavour is used.
"""
from __future__ import annotations

import functools
import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

MAT_DIFFUSE = 0
MAT_DIELECTRIC = 1
MAT_EMISSIVE = 2

ALBEDO_CONST = 0
ALBEDO_CHECKER = 1
ALBEDO_TEXTURE = 2
ALBEDO_TEXTURE_RGB = 3

WL_FIXED = 0
WL_UNIFORM = 1

# One record per object (48 bytes).  Dielectrics also carry a nesting
# priority, absorption coefficients in 1/m at 450, 550 and 650 nm, and a
# GGX roughness (0 = smooth); the other types ignore those fields.
MATERIAL_DTYPE = np.dtype([
    ("type", "<u4"), ("albedo_mode", "<u4"),
    ("rho_a", "<f4"), ("rho_b", "<f4"),
    ("cauchy_a", "<f4"), ("cauchy_b", "<f4"),
    ("le", "<f4"), ("priority", "<u4"),
    ("sigma", "<f4", (3,)), ("roughness", "<f4"),
])


@dataclass
class Camera:
    eye: np.ndarray          # float32[3]
    fwd: np.ndarray          # float32[3], unit
    right: np.ndarray        # float32[3], unit right * tan(vfov/2) * aspect
    up: np.ndarray           # float32[3], unit up * tan(vfov/2)
    w: int
    h: int


@dataclass
class Wavelengths:
    mode: int = WL_FIXED
    k: int = 3
    nm: tuple = (650.0, 550.0, 450.0)   # channel order R, G, B
    lo: float = 380.0
    hi: float = 720.0
    bins: int = 16

    @property
    def channels(self) -> int:
        """Number of caustic-map channels: one per slot (FIXED) or per bin."""
        return self.k if self.mode == WL_FIXED else self.bins


@dataclass
class Receiver:
    obj: int
    wc: int
    hc: int
    x0: float
    y0: float
    ext_u: float
    ext_v: float


@dataclass
class Scene:
    V: np.ndarray                      # float32 [nv,3]
    I: np.ndarray                      # uint32 [nt,3]
    VN: Optional[np.ndarray]           # float32 [nv,3] or None
    tri_obj: np.ndarray                # uint32 [nt]
    materials: np.ndarray              # MATERIAL_DTYPE [n_obj+1], row 0 unused
    point_lights: np.ndarray           # float32 [n_pl,4]: x,y,z,intensity (W/sr)
    targets_obj: np.ndarray            # uint32 [n_tg]
    targets_sphere: np.ndarray         # float32 [n_tg,4]: cx,cy,cz,radius
    receiver: Optional[Receiver]
    tex: Optional[np.ndarray] = None   # float32 [th,tw] grey albedo
    tex_rect: tuple = (0.0, 0.0, 1.0, 1.0)   # x0, y0, ext_u, ext_v
    name: str = ""
    tex_rgb: Optional[np.ndarray] = None   # float32 [th,tw,3] RGB albedo (same size and rectangle as tex)

    @property
    def nt(self) -> int:
        return int(self.I.shape[0])

    @property
    def nv(self) -> int:
        return int(self.V.shape[0])

    def validate(self) -> None:
        assert self.V.dtype == np.float32 and self.V.ndim == 2 and self.V.shape[1] == 3
        assert self.I.dtype == np.uint32 and self.I.ndim == 2 and self.I.shape[1] == 3
        assert self.tri_obj.dtype == np.uint32 and self.tri_obj.shape == (self.nt,)
        assert self.materials.dtype == MATERIAL_DTYPE
        assert int(self.I.max(initial=0)) < self.nv
        assert int(self.tri_obj.min(initial=1)) >= 1
        assert int(self.tri_obj.max(initial=1)) < len(self.materials)
        if self.VN is not None:
            assert self.VN.dtype == np.float32 and self.VN.shape == self.V.shape
        if self.tex_rgb is not None:
            assert self.tex_rgb.dtype == np.float32 and self.tex_rgb.ndim == 3 and self.tex_rgb.shape[2] == 3
            assert self.tex is None or self.tex.shape == self.tex_rgb.shape[:2]
            assert self.tex_rgb.flags["C_CONTIGUOUS"]
        for a in ("V", "I", "tri_obj", "materials", "point_lights", "targets_obj", "targets_sphere"):
            assert getattr(self, a).flags["C_CONTIGUOUS"], a


# --------------------------------------------------------------------------
# mesh primitives (all built in float64, rounded to float32 at the end)
# --------------------------------------------------------------------------

@dataclass
class Mesh:
    V: np.ndarray          # float64 [nv,3]
    I: np.ndarray          # int64 [nt,3]
    VN: np.ndarray         # float64 [nv,3]


def _orient_outward(V, I, center):
    """Flip faces whose geometric normal points towards ``center``."""
    a, b, c = V[I[:, 0]], V[I[:, 1]], V[I[:, 2]]
    n = np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0 - center
    flip = np.einsum("ij,ij->i", n, cen) < 0
    I = I.copy()
    I[flip] = I[flip][:, [0, 2, 1]]
    return I


def _area_weighted_normals(V, I):
    a, b, c = V[I[:, 0]], V[I[:, 1]], V[I[:, 2]]
    n = np.cross(b - a, c - a)
    VN = np.zeros_like(V)
    for k in range(3):
        np.add.at(VN, I[:, k], n)
    ln = np.linalg.norm(VN, axis=1, keepdims=True)
    ln[ln == 0] = 1.0
    return VN / ln


def icosphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)) -> Mesh:
    U, I = _unit_icosphere(level)
    cen = np.asarray(center, dtype=np.float64)
    return Mesh(U * radius + cen, I.copy(), U.copy())


@functools.lru_cache(maxsize=None)
def _unit_icosphere(level: int):
    """Subdivided icosahedron with vertices projected to the sphere.

    Level L has 20*4^L triangles and 10*4^L+2 vertices (level 3: 1,280 and
    642).  Vertex normals are the exact radial directions.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
             (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
             (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
             (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
             (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
             (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    P = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in verts]
    F = list(faces)
    for _ in range(level):
        cache = {}

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = P[i] + P[j]
                P.append(m / np.linalg.norm(m))
                cache[key] = len(P) - 1
            return cache[key]

        nf = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        F = nf
    U = np.array(P)
    I = _orient_outward(U, np.array(F, dtype=np.int64), np.zeros(3))
    U.setflags(write=False)
    I.setflags(write=False)
    return U, I


def quad(p0, p1, p2, p3, normal) -> Mesh:
    """Two triangles (p0,p1,p2),(p0,p2,p3); winding must agree with ``normal``."""
    V = np.array([p0, p1, p2, p3], dtype=np.float64)
    I = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int64)
    n = np.cross(V[1] - V[0], V[2] - V[0])
    if np.dot(n, normal) < 0:
        I = I[:, [0, 2, 1]]
    VN = np.tile(np.asarray(normal, dtype=np.float64) / np.linalg.norm(normal), (4, 1))
    return Mesh(V, I, VN)


def _ring_faces(s: int, m: int) -> np.ndarray:
    """Faces of a closed grid with a pole at each end: vertex 0 is the bottom
    pole, rings 1..s-2 hold m vertices each, the last vertex is the top pole."""
    i = np.arange(m)
    i1 = (i + 1) % m
    bottom = np.stack([np.zeros(m, np.int64), 1 + i1, 1 + i], 1)
    k = np.arange(s - 3)[:, None]
    b0 = 1 + k * m
    b1 = 1 + (k + 1) * m
    q1 = np.stack([b0 + i, b0 + i1, b1 + i1], -1).reshape(-1, 3)
    q2 = np.stack([b0 + i, b1 + i1, b1 + i], -1).reshape(-1, 3)
    quads = np.stack([q1, q2], 1).reshape(-1, 3)
    bl = 1 + (s - 3) * m
    top_idx = 1 + (s - 2) * m
    top = np.stack([bl + i, bl + i1, np.full(m, top_idx, np.int64)], 1)
    return np.concatenate([bottom, quads, top]).astype(np.int64)


def _revolve(rings_r, rings_z, m):
    """Closed surface of revolution around +z: rings_r[0] and rings_r[-1]
    are 0 (the poles)."""
    s = len(rings_r)
    assert rings_r[0] == 0 and rings_r[-1] == 0
    phi = np.arange(m) * (2.0 * math.pi / m)
    r = np.asarray(rings_r[1:-1], dtype=np.float64)[:, None]
    z = np.asarray(rings_z[1:-1], dtype=np.float64)[:, None]
    ring = np.stack([r * np.cos(phi), r * np.sin(phi), np.broadcast_to(z, (len(r), m))], -1)
    V = np.concatenate([[[0.0, 0.0, rings_z[0]]], ring.reshape(-1, 3), [[0.0, 0.0, rings_z[-1]]]])
    return V, _ring_faces(s, m)


def lathe(rng: np.random.Generator, n_tris: int, height: float, max_radius: float) -> Mesh:
    """Closed solid of revolution from a seeded 6-knot radius profile."""
    knots_h = np.linspace(0.0, 1.0, 6)
    knots_r = rng.uniform(0.35, 1.0, size=6)
    # segments around (m) and along (s) sized to the triangle target: ~2*m*s
    m = max(8, int(round(math.sqrt(n_tris / 2.0 * 1.5))))
    s = max(4, int(round(n_tris / (2.0 * m))) + 1)
    hz = np.linspace(0.0, 1.0, s)
    r = np.interp(hz, knots_h, knots_r)
    # round the ends smoothly to the axis so the profile closes
    taper = np.sqrt(np.clip(np.sin(np.pi * hz), 0.0, 1.0))
    r = r * taper * max_radius
    r[0] = 0.0
    r[-1] = 0.0
    V, I = _revolve(r, hz * height, m)
    I = _orient_outward(V, I, np.array([0.0, 0.0, 0.5 * height]))
    return Mesh(V, I, _area_weighted_normals(V, I))


def superquadric(rng: np.random.Generator, n_tris: int, size: float) -> Mesh:
    """Closed superellipsoid with exponents e1, e2 ~ U[0.3, 2.5]."""
    e1, e2 = rng.uniform(0.3, 2.5, size=2)
    ax = size * rng.uniform(0.6, 1.0, size=3)
    m = max(8, int(round(math.sqrt(n_tris))))
    s = max(4, int(round(n_tris / (2.0 * m))) + 1)

    def f(w, e):
        return np.sign(w) * np.abs(w) ** e

    eta = np.linspace(-math.pi / 2, math.pi / 2, s)[1:-1, None]
    omg = (np.arange(m) * (2.0 * math.pi / m))[None, :]
    ce, se = f(np.cos(eta), e1), f(np.sin(eta), e1)
    X = ax[0] * ce * f(np.cos(omg), e2)
    Y = ax[1] * ce * f(np.sin(omg), e2)
    Z = np.broadcast_to(ax[2] * se, X.shape)
    V = np.concatenate([[[0.0, 0.0, -ax[2]]], np.stack([X, Y, Z], -1).reshape(-1, 3), [[0.0, 0.0, ax[2]]]])
    I = _ring_faces(s, m)
    I = _orient_outward(V, I, np.zeros(3))
    return Mesh(V, I, _area_weighted_normals(V, I))


def box(size) -> Mesh:
    """Axis-aligned box centred at the origin with flat faces (24 vertices)."""
    sx, sy, sz = (np.asarray(size, dtype=np.float64) * 0.5)
    Vs, Is, Ns = [], [], []
    faces = [((1, 0, 0), (0, 1, 0), (0, 0, 1)), ((-1, 0, 0), (0, -1, 0), (0, 0, 1)),
             ((0, 1, 0), (-1, 0, 0), (0, 0, 1)), ((0, -1, 0), (1, 0, 0), (0, 0, 1)),
             ((0, 0, 1), (1, 0, 0), (0, 1, 0)), ((0, 0, -1), (-1, 0, 0), (0, 1, 0))]
    h = np.array([sx, sy, sz])
    for n, u, v in faces:
        n, u, v = map(np.array, (n, u, v))
        c = n * h
        du, dv = u * h, v * h
        q = quad(c - du - dv, c + du - dv, c + du + dv, c - du + dv, n)
        Is.append(q.I + 4 * len(Vs))
        Vs.append(q.V)
        Ns.append(q.VN)
    return Mesh(np.concatenate(Vs), np.concatenate(Is), np.concatenate(Ns))


def cylinder(n_tris: int, radius: float, height: float) -> Mesh:
    m = max(6, n_tris // 4)
    r = np.array([0.0, radius, radius, 0.0])
    z = np.array([0.0, 0.0, height, height])
    # duplicate cap/side rings are not needed: smooth-ish normals are fine for clutter
    V, I = _revolve(r, z, m)
    I = _orient_outward(V, I, np.array([0.0, 0.0, 0.5 * height]))
    return Mesh(V, I, _area_weighted_normals(V, I))


def displaced_sphere(rng: np.random.Generator, level: int, radius: float, amp: float) -> Mesh:
    base = icosphere(level)
    k = rng.normal(size=(6, 3))
    ph = rng.uniform(0, 2 * math.pi, size=6)
    d = np.zeros(len(base.V))
    for i in range(6):
        d += np.sin(base.V @ k[i] * 3.0 + ph[i])
    V = base.V * (radius * (1.0 + amp * d / 6.0))[:, None]
    I = _orient_outward(V, base.I, np.zeros(3))
    return Mesh(V, I, _area_weighted_normals(V, I))


def _rotation(yaw, tilt, tilt_axis_angle):
    cy, sy = math.cos(yaw), math.sin(yaw)
    Rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]])
    a = tilt_axis_angle
    axis = np.array([math.cos(a), math.sin(a), 0.0])
    K = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    Rt = np.eye(3) + math.sin(tilt) * K + (1 - math.cos(tilt)) * (K @ K)
    return Rt @ Rz


def place(mesh: Mesh, R: np.ndarray, t: np.ndarray, rest_on: Optional[float] = None) -> Mesh:
    V = mesh.V @ R.T
    if rest_on is not None:
        V[:, 2] += rest_on - V[:, 2].min() + 1e-3
    V = V + t
    return Mesh(V, mesh.I.copy(), mesh.VN @ R.T)


# --------------------------------------------------------------------------
# scene assembly
# --------------------------------------------------------------------------

class SceneBuilder:
    def __init__(self):
        self.Vs: List[np.ndarray] = []
        self.Is: List[np.ndarray] = []
        self.Ns: List[np.ndarray] = []
        self.objs: List[np.ndarray] = []
        self.mats = [np.zeros((), dtype=MATERIAL_DTYPE)]
        self.nv = 0
        self.targets = []
        self.lights = []

    def add(self, mesh: Mesh, mat: dict, photon_target: bool = False) -> int:
        obj = len(self.mats)
        m = np.zeros((), dtype=MATERIAL_DTYPE)
        for k, v in mat.items():
            m[k] = v
        self.mats.append(m)
        self.Vs.append(mesh.V)
        self.Is.append(mesh.I + self.nv)
        self.Ns.append(mesh.VN)
        self.objs.append(np.full(len(mesh.I), obj, dtype=np.uint32))
        self.nv += len(mesh.V)
        if photon_target:
            lo, hi = mesh.V.min(0), mesh.V.max(0)
            c = 0.5 * (lo + hi)
            r = float(np.linalg.norm(mesh.V - c, axis=1).max()) * (1.0 + 1e-5) + 1e-6
            self.targets.append((obj, c, r))
        return obj

    def point_light(self, pos, intensity):
        self.lights.append((*pos, intensity))

    def build(self, receiver: Optional[Receiver], tex=None, tex_rect=(0, 0, 1, 1), name="", tex_rgb=None) -> Scene:
        V = np.concatenate(self.Vs).astype(np.float32)
        N = np.concatenate(self.Ns)
        N = (N / np.maximum(np.linalg.norm(N, axis=1, keepdims=True), 1e-300)).astype(np.float32)
        tg_obj = np.array([t[0] for t in self.targets], dtype=np.uint32)
        tg_sph = np.array([[*t[1], t[2]] for t in self.targets], dtype=np.float32).reshape(-1, 4)
        s = Scene(
            V=np.ascontiguousarray(V),
            I=np.ascontiguousarray(np.concatenate(self.Is).astype(np.uint32)),
            VN=np.ascontiguousarray(N),
            tri_obj=np.ascontiguousarray(np.concatenate(self.objs)),
            materials=np.ascontiguousarray(np.array(self.mats, dtype=MATERIAL_DTYPE)),
            point_lights=np.ascontiguousarray(np.array(self.lights, dtype=np.float32).reshape(-1, 4)),
            targets_obj=np.ascontiguousarray(tg_obj),
            targets_sphere=np.ascontiguousarray(tg_sph),
            receiver=receiver,
            tex=None if tex is None else np.ascontiguousarray(tex.astype(np.float32)),
            tex_rect=tuple(float(x) for x in tex_rect),
            name=name,
            tex_rgb=None if tex_rgb is None else np.ascontiguousarray(tex_rgb.astype(np.float32)),
        )
        s.validate()
        return s


def look_at(eye, target, up, vfov_deg, w, h) -> Camera:
    """Pinhole camera; tan(vfov/2) and the aspect ratio are folded in here."""
    eye = np.asarray(eye, dtype=np.float64)
    f = np.asarray(target, dtype=np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, dtype=np.float64))
    r /= np.linalg.norm(r)
    u = np.cross(r, f)
    th = math.tan(math.radians(vfov_deg) * 0.5)
    return Camera(eye.astype(np.float32), f.astype(np.float32),
                  (r * th * (w / h)).astype(np.float32), (u * th).astype(np.float32), int(w), int(h))


def value_noise(rng: np.random.Generator, n: int, octaves: int = 4, lo=0.2, hi=0.8) -> np.ndarray:
    img = np.zeros((n, n))
    amp, tot = 1.0, 0.0
    for o in range(octaves):
        g = 4 * 2 ** o
        grid = rng.uniform(size=(g + 1, g + 1))
        x = np.linspace(0, g, n, endpoint=False)
        i = x.astype(int)
        f = x - i
        f = f * f * (3 - 2 * f)
        a = grid[i][:, i] * (1 - f)[None, :] + grid[i][:, i + 1] * f[None, :]
        b = grid[i + 1][:, i] * (1 - f)[None, :] + grid[i + 1][:, i + 1] * f[None, :]
        img += amp * (a * (1 - f)[:, None] + b * f[:, None])
        tot += amp
        amp *= 0.5
    img /= tot
    img = (img - img.min()) / max(img.max() - img.min(), 1e-12)
    return (lo + (hi - lo) * img).astype(np.float32)


# --------------------------------------------------------------------------
# the workloads
# --------------------------------------------------------------------------

GLASS_C1 = dict(type=MAT_DIELECTRIC, cauchy_a=1.5, cauchy_b=0.0042)


def _square_light(center, side, down_intensity):
    """Downward-facing square emitter of the given side whose intensity
    along its normal (le * area) equals ``down_intensity`` W/sr."""
    cx, cy, cz = center
    h = 0.5 * side
    q = quad((cx - h, cy - h, cz), (cx - h, cy + h, cz), (cx + h, cy + h, cz), (cx + h, cy - h, cz), (0, 0, -1))
    return q, dict(type=MAT_EMISSIVE, le=down_intensity / (side * side))


def _scaled_light(p0, p1, p2, p3, le, scale):
    """An area light quad scaled by ``scale`` about its centre, radiance
    divided by scale^2 so that its power stays the same."""
    P = np.array([p0, p1, p2, p3], dtype=np.float64)
    c = P.mean(0)
    P = c + (P - c) * scale
    return quad(*[tuple(p) for p in P], (0, 0, -1)), dict(type=MAT_EMISSIVE, le=le / (scale * scale))


def config1(level: int = 3, light_size: float = 0.0):
    """Tiny scene: glass icosphere over an 8x8 m checker plane, one point light.

    Glass icosphere (level 3 = 1,280 triangles, radius 1, centre (0,0,1.5))
    with Cauchy n = 1.5 + 0.0042/lambda^2 (lambda in micrometres); a
    two-triangle plane [-4,4]^2 at z=0 with a 1 m checker of albedo 0.8/0.2;
    a 50 W/sr point light at (2,3,6); a 128x128 pinhole camera; three fixed
    wavelengths 650/550/450 nm (R,G,B); a 256x256 caustic map on the plane.

    ``light_size`` > 0 is the caustic-softness knob: the point light becomes
    a downward-facing square emitter of that side with the same intensity
    along its normal, so caustics blur as it grows.
    """
    b = SceneBuilder()
    plane = quad((-4, -4, 0), (4, -4, 0), (4, 4, 0), (-4, 4, 0), (0, 0, 1))
    recv_obj = b.add(plane, dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_CHECKER, rho_a=0.8, rho_b=0.2))
    b.add(icosphere(level, 1.0, (0.0, 0.0, 1.5)), GLASS_C1, photon_target=True)
    if light_size > 0.0:
        b.add(*_square_light((2.0, 3.0, 6.0), light_size, 50.0))
    else:
        b.point_light((2.0, 3.0, 6.0), 50.0)
    scene = b.build(Receiver(recv_obj, 256, 256, -4.0, -4.0, 8.0, 8.0), name=f"c1-ico{level}" + (f"-light{light_size:g}" if light_size > 0.0 else ""))
    cam = look_at((0.0, -7.0, 5.0), (0.0, 0.0, 0.8), (0, 0, 1), 40.0, 128, 128)
    wl = Wavelengths(WL_FIXED, 3, (650.0, 550.0, 450.0))
    return dict(scene=scene, camera=cam, wavelengths=wl, spp=1, max_depth=8,
                n_photons=1 << 16, scene_seed=1000, render_seed=1001, photon_seed=1002)


def _glass(rng):
    return dict(type=MAT_DIELECTRIC, cauchy_a=float(rng.uniform(1.45, 1.6)),
                cauchy_b=float(rng.uniform(0.003, 0.01)))


def config2(seed: int = 2000, tri_scale: float = 1.0, w: int = 512, h: int = 512, light_scale: float = 1.0,
            glass_style: str = "clear"):
    """Medium scene: eight seeded glass objects (4 lathe + 4 superquadric,
    10k-50k triangles each, ~2e5 total) resting on a 4x4 m value-noise
    textured plane, one 0.5x0.5 m area light, 512x512, spectral 380-720 nm.
    ``tri_scale`` shrinks the triangle counts for quick tests;
    ``light_scale`` resizes the light at constant power (caustic softness);
    ``glass_style="rich"`` tints every object (absorption 0.5-6 per metre
    per wavelength knot) and roughens every second one (GGX alpha
    0.05-0.3), same geometry."""
    rng = np.random.default_rng(seed)
    rich = np.random.default_rng(seed + 7) if glass_style == "rich" else None
    if glass_style not in ("clear", "rich"):
        raise ValueError(glass_style)
    b = SceneBuilder()
    plane = quad((-2, -2, 0), (2, -2, 0), (2, 2, 0), (-2, 2, 0), (0, 0, 1))
    tex = value_noise(rng, 512)
    recv = b.add(plane, dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_TEXTURE))
    counts = rng.integers(10_000, 50_001, size=8)
    counts = np.maximum((counts * (200_000 / counts.sum()) * tri_scale).astype(int), 200)
    slots = [(x, y) for x in (-0.45, -0.15, 0.15, 0.45) for y in (-0.3, 0.3)]
    order = rng.permutation(8)
    for i in range(8):
        n = int(counts[i])
        if i < 4:
            mesh = lathe(rng, n, height=float(rng.uniform(0.15, 0.35)), max_radius=float(rng.uniform(0.06, 0.12)))
            mesh = Mesh(mesh.V, mesh.I, mesh.VN)
        else:
            mesh = superquadric(rng, n, size=float(rng.uniform(0.06, 0.12)))
        R = _rotation(rng.uniform(0, 2 * math.pi), math.radians(rng.uniform(0, 30)), rng.uniform(0, 2 * math.pi))
        sx, sy = slots[order[i]]
        t = np.array([sx + rng.uniform(-0.04, 0.04), sy + rng.uniform(-0.06, 0.06), 0.0])
        mat = _glass(rng)
        if rich is not None:
            mat["sigma"] = rich.uniform(0.5, 6.0, size=3).astype(np.float32)
            mat["roughness"] = float(rich.uniform(0.05, 0.3)) if i % 2 else 0.0
        b.add(place(mesh, R, t, rest_on=0.0), mat, photon_target=True)
    b.add(*_scaled_light((0.05, -0.45, 2.5), (0.05, 0.05, 2.5), (0.55, 0.05, 2.5), (0.55, -0.45, 2.5), 12.0,
                         light_scale))
    scene = b.build(Receiver(recv, 1024, 1024, -2.0, -2.0, 4.0, 4.0), tex=tex, tex_rect=(-2.0, -2.0, 4.0, 4.0),
                    name=f"c2-{seed}")
    cam = look_at((0.0, -1.6, 1.6), (0.0, 0.0, 0.05), (0, 0, 1), 40.0, w, h)
    wl = Wavelengths(WL_UNIFORM, 1, (550.0,), 380.0, 720.0, 16)
    return dict(scene=scene, camera=cam, wavelengths=wl, spp=16, max_depth=12,
                n_photons=1 << 22, scene_seed=seed, render_seed=seed + 1, photon_seed=seed + 2)


def config3(seed: int = 3000, tri_scale: float = 1.0, w: int = 1920, h: int = 1080, light_scale: float = 1.0,
            floor: str = "grey"):
    """Large scene: 40 overlapping glass meshes (~1.2M triangles) plus opaque
    diffuse clutter (~0.8M triangles) on a textured floor, two area lights,
    1920x1080, 64 spp spectral, depth 16.  ``light_scale`` resizes both
    lights at constant power (caustic softness); ``floor="rgb"`` gives the
    floor an RGB value-noise albedo texture (same geometry)."""
    rng = np.random.default_rng(seed)
    b = SceneBuilder()
    plane = quad((-3, -3, 0), (3, -3, 0), (3, 3, 0), (-3, 3, 0), (0, 0, 1))
    tex = value_noise(rng, 1024)
    tex_rgb = None
    if floor == "rgb":
        crng = np.random.default_rng(seed + 11)
        tex_rgb = np.stack([value_noise(crng, 1024, lo=0.1, hi=0.9) for _ in range(3)], -1)
    elif floor != "grey":
        raise ValueError(floor)
    recv = b.add(plane, dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_TEXTURE if tex_rgb is None else ALBEDO_TEXTURE_RGB))
    glass_tris = int(1_200_000 * tri_scale)
    per = max(200, glass_tris // 40)
    for i in range(40):
        n = int(per * rng.uniform(0.6, 1.4))
        if i % 2 == 0:
            mesh = lathe(rng, n, height=float(rng.uniform(0.15, 0.45)), max_radius=float(rng.uniform(0.05, 0.14)))
        else:
            mesh = superquadric(rng, n, size=float(rng.uniform(0.05, 0.14)))
        R = _rotation(rng.uniform(0, 2 * math.pi), math.radians(rng.uniform(0, 30)), rng.uniform(0, 2 * math.pi))
        t = np.array([rng.uniform(-1.1, 1.1), rng.uniform(-0.8, 0.8), 0.0])
        b.add(place(mesh, R, t, rest_on=0.0), _glass(rng), photon_target=True)
    clutter_tris = int(800_000 * tri_scale)
    made = 0
    while made < clutter_tris:
        kind = rng.integers(0, 3)
        R = _rotation(rng.uniform(0, 2 * math.pi), 0.0, 0.0)
        t = np.array([rng.uniform(-2.5, 2.5), rng.uniform(-1.5, 2.5), 0.0])
        if kind == 0:
            mesh = box(rng.uniform(0.05, 0.4, size=3))
        elif kind == 1:
            mesh = cylinder(int(rng.integers(64, 512)), float(rng.uniform(0.03, 0.15)), float(rng.uniform(0.05, 0.5)))
        else:
            lvl = int(rng.integers(3, 7))
            mesh = displaced_sphere(rng, lvl, float(rng.uniform(0.05, 0.25)), 0.15)
        rho = float(rng.uniform(0.2, 0.8))
        b.add(place(mesh, R, t, rest_on=0.0), dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_CONST, rho_a=rho))
        made += len(mesh.I)
    b.add(*_scaled_light((-1.2, -0.6, 3.0), (-1.2, 0.0, 3.0), (-0.6, 0.0, 3.0), (-0.6, -0.6, 3.0), 8.0, light_scale))
    b.add(*_scaled_light((0.8, 0.4, 2.6), (0.8, 0.8, 2.6), (1.2, 0.8, 2.6), (1.2, 0.4, 2.6), 10.0, light_scale))
    scene = b.build(Receiver(recv, 2048, 2048, -3.0, -3.0, 6.0, 6.0), tex=tex, tex_rect=(-3.0, -3.0, 6.0, 6.0),
                    name=f"c3-{seed}" + ("-rgb" if tex_rgb is not None else ""), tex_rgb=tex_rgb)
    cam = look_at((0.0, -3.2, 2.2), (0.0, 0.0, 0.1), (0, 0, 1), 45.0, w, h)
    wl = Wavelengths(WL_UNIFORM, 1, (550.0,), 380.0, 720.0, 16)
    return dict(scene=scene, camera=cam, wavelengths=wl, spp=64, max_depth=16,
                n_photons=1 << 24, scene_seed=seed, render_seed=seed + 1, photon_seed=seed + 2)


def config4_item(j: int, base_seed: int = 4000):
    """One scene of the 64-scene batch: triangle count log-uniform in
    [1e3, 5e5], square resolution log-uniform in [256, 1024] rounded to a
    multiple of 32, 8 spp, depth 12, 2^18 photons into a 512x512x16 map."""
    rng = np.random.default_rng(base_seed + j)
    nt = int(math.exp(rng.uniform(math.log(1e3), math.log(5e5))))
    side = int(round(math.exp(rng.uniform(math.log(256), math.log(1024))) / 32.0) * 32)
    n_obj = int(rng.integers(1, 6))
    b = SceneBuilder()
    plane = quad((-1.5, -1.5, 0), (1.5, -1.5, 0), (1.5, 1.5, 0), (-1.5, 1.5, 0), (0, 0, 1))
    recv = b.add(plane, dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_CHECKER, rho_a=0.7, rho_b=0.3))
    per = max(100, (nt - 4) // n_obj)
    for i in range(n_obj):
        if rng.uniform() < 0.5:
            mesh = lathe(rng, per, height=float(rng.uniform(0.15, 0.4)), max_radius=float(rng.uniform(0.06, 0.15)))
        else:
            mesh = superquadric(rng, per, size=float(rng.uniform(0.06, 0.15)))
        R = _rotation(rng.uniform(0, 2 * math.pi), math.radians(rng.uniform(0, 30)), rng.uniform(0, 2 * math.pi))
        t = np.array([rng.uniform(-0.6, 0.6), rng.uniform(-0.5, 0.5), 0.0])
        b.add(place(mesh, R, t, rest_on=0.0), _glass(rng), photon_target=True)
    light = quad((0.2, -0.5, 2.2), (0.2, -0.1, 2.2), (0.6, -0.1, 2.2), (0.6, -0.5, 2.2), (0, 0, -1))
    b.add(light, dict(type=MAT_EMISSIVE, le=14.0))
    scene = b.build(Receiver(recv, 512, 512, -1.5, -1.5, 3.0, 3.0), name=f"c4-{j}")
    cam = look_at((0.0, -1.8, 1.5), (0.0, 0.0, 0.05), (0, 0, 1), 40.0, side, side)
    wl = Wavelengths(WL_UNIFORM, 1, (550.0,), 380.0, 720.0, 16)
    return dict(scene=scene, camera=cam, wavelengths=wl, spp=8, max_depth=12,
                n_photons=1 << 18, scene_seed=base_seed + j, render_seed=base_seed + j + 100000,
                photon_seed=base_seed + j + 200000)


# --------------------------------------------------------------------------
# small scenes used by the pins
# --------------------------------------------------------------------------

def plane_only(albedo=0.8, light=(2.0, 3.0, 6.0), intensity=50.0, w=32, h=32, rgb=None):
    """``rgb``: an RGB albedo texture [th, tw, 3] over the plane instead of
    the constant ``albedo``."""
    b = SceneBuilder()
    plane = quad((-4, -4, 0), (4, -4, 0), (4, 4, 0), (-4, 4, 0), (0, 0, 1))
    if rgb is None:
        recv = b.add(plane, dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_CONST, rho_a=albedo))
    else:
        recv = b.add(plane, dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_TEXTURE_RGB))
    b.point_light(light, intensity)
    scene = b.build(Receiver(recv, 64, 64, -4.0, -4.0, 8.0, 8.0), name="plane",
                    tex_rgb=None if rgb is None else np.asarray(rgb, np.float32), tex_rect=(-4.0, -4.0, 8.0, 8.0))
    cam = look_at((0.0, -7.0, 5.0), (0.0, 0.0, 0.0), (0, 0, 1), 40.0, w, h)
    return scene, cam


def furnace(kind: str, level_inner: int = 3, level_outer: int = 3, w: int = 24, h: int = 24):
    """Closed furnace: an inward-emitting sphere (Le = 1) of radius 8 around
    either a glass sphere ('glass') or a white diffuse sphere ('diffuse')."""
    b = SceneBuilder()
    if kind == "glass":
        b.add(icosphere(level_inner, 1.0, (0, 0, 0)), GLASS_C1)
    else:
        b.add(icosphere(level_inner, 1.0, (0, 0, 0)),
              dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_CONST, rho_a=1.0))
    enc = icosphere(level_outer, 8.0, (0, 0, 0))
    enc = Mesh(enc.V, enc.I[:, [0, 2, 1]].copy(), -enc.VN)   # front faces point inwards
    b.add(enc, dict(type=MAT_EMISSIVE, le=1.0))
    scene = b.build(None, name=f"furnace-{kind}")
    cam = look_at((0.0, -4.0, 0.5), (0.0, 0.0, 0.0), (0, 0, 1), 40.0, w, h)
    return scene, cam


def ball_lens(level: int, receiver_z: float, light_dist: float = 1.0e4, aperture: float = 0.1,
              wc: int = 256, ext: float = 0.256):
    """Glass ball (c1 glass, radius 1, centre (0,0,0)) lit by a distant point
    light on the +z axis; the photon target is a small sphere of radius
    ``aperture`` at the centre, so photons form a paraxial beam.  A diffuse
    receiver square of side ``ext`` sits at height ``receiver_z``."""
    b = SceneBuilder()
    h = ext * 0.5
    plane = quad((-h, -h, receiver_z), (h, -h, receiver_z), (h, h, receiver_z), (-h, h, receiver_z), (0, 0, 1))
    recv = b.add(plane, dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_CONST, rho_a=0.5))
    lens = icosphere(level, 1.0, (0.0, 0.0, 0.0))
    b.add(lens, GLASS_C1)
    b.point_light((0.0, 0.0, light_dist), 1.0)
    scene = b.build(Receiver(recv, wc, wc, -h, -h, ext, ext), name=f"ball-{receiver_z}")
    scene.targets_obj = np.array([2], dtype=np.uint32)
    scene.targets_sphere = np.array([[0.0, 0.0, 0.0, aperture]], dtype=np.float32)
    return scene


def glass(n: float = 1.5, b: float = 0.0, sigma=(0.0, 0.0, 0.0), priority: int = 0, roughness: float = 0.0):
    """Dielectric material: Cauchy n(lambda) = n + b / lambda_um^2,
    absorption coefficients (1/m) at 450, 550 and 650 nm, nesting priority
    and GGX roughness."""
    return dict(type=MAT_DIELECTRIC, cauchy_a=n, cauchy_b=b, sigma=np.asarray(sigma, dtype=np.float32),
                priority=priority, roughness=roughness)


def slab_stack(layers, receiver_z: float = 0.0, light_dist: float = 1.0e4, aperture: float = 0.05,
               wc: int = 64, ext: float = 1.0):
    """Axis-aligned glass boxes centred on the z axis, given as
    (size_xyz, z_centre, material) from the outermost in, under a distant
    point light on +z.  The photon target is a sphere of radius
    ``aperture`` at the centre of the first box, so photons form a beam at
    normal incidence.  A diffuse receiver square of side ``ext`` lies at
    ``receiver_z`` below the boxes."""
    b = SceneBuilder()
    h = ext * 0.5
    plane = quad((-h, -h, receiver_z), (h, -h, receiver_z), (h, h, receiver_z), (-h, h, receiver_z), (0, 0, 1))
    recv = b.add(plane, dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_CONST, rho_a=0.5))
    for size, zc, mat in layers:
        m = box(size)
        b.add(Mesh(m.V + np.array([0.0, 0.0, zc]), m.I, m.VN), mat)
    b.point_light((0.0, 0.0, light_dist), 1.0)
    scene = b.build(Receiver(recv, wc, wc, -h, -h, ext, ext), name="slabs")
    scene.targets_obj = np.array([2], dtype=np.uint32)
    scene.targets_sphere = np.array([[0.0, 0.0, layers[0][1], aperture]], dtype=np.float32)
    return scene


def slab_over_light(thickness: float, mat: dict, le: float = 1.0, w: int = 8, h: int = 8):
    """A 2 x 2 m glass box of the given thickness (bottom face at z = 0.5)
    over an upward-facing emitter at z = 0, seen from straight above by a
    far camera (eye at z = 1000, 0.01 degree field), so every camera ray
    meets the glass at normal incidence to within 1e-4 rad."""
    b = SceneBuilder()
    light = quad((-2, -2, 0), (2, -2, 0), (2, 2, 0), (-2, 2, 0), (0, 0, 1))
    b.add(light, dict(type=MAT_EMISSIVE, le=le))
    m = box((2.0, 2.0, thickness))
    b.add(Mesh(m.V + np.array([0.0, 0.0, 0.5 + 0.5 * thickness]), m.I, m.VN), mat)
    scene = b.build(None, name="slab-light")
    cam = look_at((0.0, 0.0, 1000.0), (0.0, 0.0, 0.0), (0, 1, 0), 0.01, w, h)
    return scene, cam


def tinted_nested(level: int = 3, w: int = 48, h: int = 40, n_photons: int = 1 << 15):
    """Coloured, rough and nested glass over a checker plane: a tinted
    sphere A (radius 1) holding a denser, darker inclusion B (radius 0.45,
    higher priority), overlapped by a rough sphere C (GGX alpha 0.25) of
    middle priority, and a thin absorbing rough slab D (alpha 0.1); one
    point and one area light, spectral 380-720 nm, depth 12.  Every
    crossing rule shows up: air-glass, glass-glass, surfaces hidden inside
    a higher-priority medium, smooth and microfacet interfaces, absorption
    on camera paths, shadow rays and photons."""
    b = SceneBuilder()
    plane = quad((-4, -4, 0), (4, -4, 0), (4, 4, 0), (-4, 4, 0), (0, 0, 1))
    recv = b.add(plane, dict(type=MAT_DIFFUSE, albedo_mode=ALBEDO_CHECKER, rho_a=0.8, rho_b=0.3))
    b.add(icosphere(level, 1.0, (0.0, 0.0, 1.2)), glass(1.5, 0.0042, sigma=(0.2, 0.8, 1.6)), photon_target=True)
    b.add(icosphere(level, 0.45, (0.2, 0.0, 1.3)), glass(1.8, 0.01, sigma=(3.0, 1.0, 0.5), priority=2))
    b.add(icosphere(level, 0.7, (1.3, 0.3, 1.0)),
          glass(1.33, 0.003, sigma=(0.0, 0.3, 0.0), priority=1, roughness=0.25), photon_target=True)
    slab = box((0.8, 0.8, 0.06))
    b.add(Mesh(slab.V + np.array([-1.7, -0.6, 0.7]), slab.I, slab.VN),
          glass(1.6, 0.005, sigma=(4.0, 4.0, 0.5), roughness=0.1), photon_target=True)
    b.point_light((2.0, 3.0, 6.0), 40.0)
    light = quad((-1.5, 1.0, 4.0), (-1.5, 1.6, 4.0), (-0.9, 1.6, 4.0), (-0.9, 1.0, 4.0), (0, 0, -1))
    b.add(light, dict(type=MAT_EMISSIVE, le=20.0))
    scene = b.build(Receiver(recv, 128, 128, -4.0, -4.0, 8.0, 8.0), name="tinted-nested")
    cam = look_at((0.0, -6.0, 4.0), (0.0, 0.0, 0.9), (0, 0, 1), 40.0, w, h)
    wl = Wavelengths(WL_UNIFORM, 1, (550.0,), 380.0, 720.0, 8)
    return dict(scene=scene, camera=cam, wavelengths=wl, spp=2, max_depth=12,
                n_photons=n_photons, scene_seed=5000, render_seed=5001, photon_seed=5002)
