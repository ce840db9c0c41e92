"""CPU oracle of the SuperCaustics rendering hot path -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``libsco.so`` (plain C,
single-threaded, see ``sco.c``) with ctypes and shares no code with the HIP
library; the struct layouts are restated here independently.

Parity status of each function is listed in the module docstrings of the
tests that pin it; the full radiance image and the caustic-map magnitude on
the procedural scenes have no closed form ("parity unpinned" beyond the
invariants and special cases the tests check).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class Material(C.Structure):
    _fields_ = [("type", C.c_uint32), ("albedo_mode", C.c_uint32), ("rho_a", C.c_float), ("rho_b", C.c_float),
                ("cauchy_a", C.c_float), ("cauchy_b", C.c_float), ("le", C.c_float), ("priority", C.c_uint32),
                ("sigma", C.c_float * 3), ("roughness", C.c_float)]


class SceneS(C.Structure):
    _fields_ = [("V", C.c_void_p), ("I", C.c_void_p), ("VN", C.c_void_p), ("tri_obj", C.c_void_p),
                ("nv", C.c_uint32), ("nt", C.c_uint32),
                ("mat", C.c_void_p), ("n_mat", C.c_uint32),
                ("pl", C.c_void_p), ("n_pl", C.c_uint32),
                ("tg_obj", C.c_void_p), ("tg_sph", C.c_void_p), ("n_tg", C.c_uint32),
                ("tex", C.c_void_p), ("tex_w", C.c_uint32), ("tex_h", C.c_uint32),
                ("tex_x0", C.c_float), ("tex_y0", C.c_float), ("tex_ext_u", C.c_float), ("tex_ext_v", C.c_float),
                ("recv_obj", C.c_uint32), ("recv_wc", C.c_uint32), ("recv_hc", C.c_uint32),
                ("recv_x0", C.c_float), ("recv_y0", C.c_float), ("recv_ext_u", C.c_float), ("recv_ext_v", C.c_float),
                ("tex_rgb", C.c_void_p)]


class CameraS(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("fwd", C.c_float * 3), ("right", C.c_float * 3), ("up", C.c_float * 3),
                ("w", C.c_uint32), ("h", C.c_uint32)]


class WavelengthsS(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("k", C.c_uint32), ("nm", C.c_float * 4), ("lo", C.c_float),
                ("hi", C.c_float), ("bins", C.c_uint32)]


class AovS(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("obj", C.c_void_p), ("trans", C.c_void_p), ("tri", C.c_void_p),
                ("depth", C.c_void_p), ("depthn", C.c_void_p), ("normal", C.c_void_p),
                ("normal_cam", C.c_void_p), ("albedo", C.c_void_p), ("tie", C.c_void_p)]


class PhotonStatsS(C.Structure):
    _fields_ = [("flux", C.c_double * 9), ("count", C.c_uint64 * 9), ("segments", C.c_uint64)]


# one stored photon of the general photon map (40 bytes, as sco_pm_rec)
PM_REC_DTYPE = np.dtype([("pos", "<f4", (3,)), ("nrm", "<f4", (3,)), ("phi", "<f4"), ("channel", "<u4"),
                         ("photon", "<u8")])

PH_OUTCOMES = ("deposited", "outside", "direct", "elsewhere", "escaped", "absorbed", "truncated", "lost",
               "emit_dead")


def lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        _LIB = load(path)
    return _LIB


def load(path):
    """Open an oracle library at `path` and declare its functions (the
    mutation tests open deliberately broken builds of sco.c this way)."""
    L = C.CDLL(path)
    vp, u32, u64, f32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_float
    L.sco_philox.argtypes = [vp, vp, vp]
    L.sco_sincos2pi.argtypes = [f32, vp, vp]
    L.sco_bvh_build.argtypes = [vp]
    L.sco_bvh_build.restype = vp
    L.sco_bvh_free.argtypes = [vp]
    L.sco_closest.argtypes = [vp, vp, u32, vp, vp, vp, vp, vp, vp]
    L.sco_any.argtypes = [vp, vp, u32, vp, vp, vp, vp, vp]
    L.sco_dielectric.argtypes = [vp, vp, vp, vp, f32, f32, f32, f32, vp, vp, vp, vp]
    L.sco_fresnel.argtypes = [f32, f32, f32, f32]
    L.sco_rough_dielectric.argtypes = [vp, vp, f32, f32, f32, u32, vp, vp, vp, vp]
    L.sco_exp_neg.argtypes = [f32]
    L.sco_exp_neg.restype = f32
    L.sco_media_step.argtypes = [vp, vp, u32, u32, C.c_int, f32, vp, vp, vp, vp, vp]
    L.sco_fresnel.restype = f32
    L.sco_camera_ray.argtypes = [vp, u32, u32, f32, f32, vp, vp]
    L.sco_onb.argtypes = [vp, vp, vp]
    L.sco_cosine_dir.argtypes = [vp, u32, vp, vp]
    L.sco_trace_photons.argtypes = [vp, vp, u64, u64, u64, u32, vp, u64, vp, vp, vp]
    L.sco_render.argtypes = [vp, vp, vp, u32, u32, vp, u64, vp, vp, u32, vp, vp]
    L.sco_pm_trace.argtypes = [vp, vp, u64, u64, u64, u32, vp, u64, vp, u64, vp, vp]
    L.sco_pm_scale.argtypes = [vp, u64]
    L.sco_pm_scale.restype = C.c_double
    L.sco_pm_gather.argtypes = [vp, u64, f32, vp, vp, u32]
    L.sco_pm_gather.restype = f32
    L.sco_render_pm.argtypes = [vp, vp, vp, u32, u32, vp, u64, vp, u64, f32, vp, u32, vp, vp]
    L.sco_path_samples.argtypes = [vp, vp, vp, u32, u32, vp, u64, vp, vp, u32, vp, vp]
    return L


def _p(a):
    return None if a is None else a.ctypes.data


class OracleScene:
    """Holds a scenegen.Scene plus the C view of it and (optionally) the
    oracle's own BVH."""

    def __init__(self, scene, use_bvh: bool = True):
        self.scene = scene
        s = scene
        self._keep = [s.V, s.I, s.VN, s.tri_obj, s.materials, s.point_lights, s.targets_obj, s.targets_sphere, s.tex,
                      s.tex_rgb]
        st = SceneS()
        st.V, st.I, st.VN, st.tri_obj = _p(s.V), _p(s.I), _p(s.VN), _p(s.tri_obj)
        st.nv, st.nt = s.nv, s.nt
        st.mat, st.n_mat = _p(s.materials), len(s.materials)
        st.pl, st.n_pl = _p(s.point_lights), len(s.point_lights)
        st.tg_obj, st.tg_sph, st.n_tg = _p(s.targets_obj), _p(s.targets_sphere), len(s.targets_obj)
        if s.tex is not None:
            st.tex, st.tex_h, st.tex_w = _p(s.tex), s.tex.shape[0], s.tex.shape[1]
            st.tex_x0, st.tex_y0, st.tex_ext_u, st.tex_ext_v = s.tex_rect
        if s.tex_rgb is not None:
            st.tex_rgb, st.tex_h, st.tex_w = _p(s.tex_rgb), s.tex_rgb.shape[0], s.tex_rgb.shape[1]
            st.tex_x0, st.tex_y0, st.tex_ext_u, st.tex_ext_v = s.tex_rect
        r = s.receiver
        if r is not None:
            st.recv_obj, st.recv_wc, st.recv_hc = r.obj, r.wc, r.hc
            st.recv_x0, st.recv_y0, st.recv_ext_u, st.recv_ext_v = r.x0, r.y0, r.ext_u, r.ext_v
        self.c = st
        self.bvh = lib().sco_bvh_build(C.byref(st)) if use_bvh else None

    def __del__(self):
        try:
            if self.bvh:
                lib().sco_bvh_free(self.bvh)
        except Exception:
            pass


def camera_struct(cam) -> CameraS:
    c = CameraS()
    c.eye[:], c.fwd[:], c.right[:], c.up[:] = [float(x) for x in cam.eye], [float(x) for x in cam.fwd], \
        [float(x) for x in cam.right], [float(x) for x in cam.up]
    c.w, c.h = cam.w, cam.h
    return c


def wavelengths_struct(wl) -> WavelengthsS:
    w = WavelengthsS()
    w.mode, w.k = wl.mode, wl.k
    nm = list(wl.nm) + [0.0] * (4 - len(wl.nm))
    w.nm[:] = [float(x) for x in nm[:4]]
    w.lo, w.hi, w.bins = wl.lo, wl.hi, wl.bins
    return w


# ---------------------------------------------------------------- primitives

def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().sco_philox(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def sincos2pi(u: float):
    s, c = C.c_float(), C.c_float()
    lib().sco_sincos2pi(float(u), C.byref(s), C.byref(c))
    return s.value, c.value


def closest(osc: OracleScene, O, D, brute: bool = False):
    O = np.ascontiguousarray(O, dtype=np.float32).reshape(-1, 3)
    D = np.ascontiguousarray(D, dtype=np.float32).reshape(-1, 3)
    n = len(O)
    t = np.empty(n, np.float32)
    prim = np.empty(n, np.uint32)
    u = np.empty(n, np.float32)
    v = np.empty(n, np.float32)
    rc = lib().sco_closest(C.byref(osc.c), None if brute else osc.bvh, n, O.ctypes.data, D.ctypes.data,
                           t.ctypes.data, prim.ctypes.data, u.ctypes.data, v.ctypes.data)
    assert rc == 0
    return t, prim, u, v


def any_hit(osc: OracleScene, O, D, tmax, excl=None, brute: bool = False):
    O = np.ascontiguousarray(O, dtype=np.float32).reshape(-1, 3)
    D = np.ascontiguousarray(D, dtype=np.float32).reshape(-1, 3)
    tmax = np.ascontiguousarray(tmax, dtype=np.float32)
    n = len(O)
    occ = np.empty(n, np.uint8)
    ex = None if excl is None else np.ascontiguousarray(excl, dtype=np.uint32)
    rc = lib().sco_any(C.byref(osc.c), None if brute else osc.bvh, n, O.ctypes.data, D.ctypes.data,
                       tmax.ctypes.data, _p(ex), occ.ctypes.data)
    assert rc == 0
    return occ.astype(bool)


def dielectric(d, Ng, Ns, P, lam, ca, cb, uF):
    a = [np.ascontiguousarray(x, dtype=np.float32) for x in (d, Ng, Ns, P)]
    o = np.zeros(3, np.float32)
    dout = np.zeros(3, np.float32)
    refl = C.c_int()
    R = C.c_float()
    ok = lib().sco_dielectric(a[0].ctypes.data, a[1].ctypes.data, a[2].ctypes.data, a[3].ctypes.data,
                              float(lam), float(ca), float(cb), float(uF), o.ctypes.data, dout.ctypes.data,
                              C.byref(refl), C.byref(R))
    return bool(ok), o, dout, bool(refl.value), R.value


def fresnel(n1, n2, ci, ct):
    return lib().sco_fresnel(float(n1), float(n2), float(ci), float(ct))


def rough_dielectric(d, n, n1, n2, alpha, u):
    """GGX interface draws: u float32 [count, 3] -> (directions [count, 3],
    reflected int32 [count] (1, 0, or -1 for no valid direction), weights)."""
    u = np.ascontiguousarray(u, dtype=np.float32).reshape(-1, 3)
    d = np.ascontiguousarray(d, dtype=np.float32)
    n = np.ascontiguousarray(n, dtype=np.float32)
    out = np.zeros((len(u), 3), np.float32)
    refl = np.zeros(len(u), np.int32)
    w = np.zeros(len(u), np.float32)
    rc = lib().sco_rough_dielectric(_p(d), _p(n), float(n1), float(n2), float(alpha), len(u), _p(u), _p(out),
                                    _p(refl), _p(w))
    if rc != 0:
        raise ValueError("sco_rough_dielectric: invalid arguments")
    return out, refl, w


def exp_neg(x):
    return lib().sco_exp_neg(float(x))


def media_step(osc: "OracleScene", ids, k: int, entering: bool, lam: float):
    """One crossing of a dielectric surface of object k with the media set
    ``ids``: returns (ids_after, real, n1, n2)."""
    a = np.ascontiguousarray(np.asarray(ids, dtype=np.uint32).reshape(-1))
    out = np.zeros(4, np.uint32)
    n_after, real = C.c_uint32(0), C.c_int(0)
    n1, n2 = C.c_float(0.0), C.c_float(0.0)
    rc = lib().sco_media_step(C.byref(osc.c), _p(a), len(a), int(k), int(bool(entering)), float(lam), _p(out),
                              C.byref(n_after), C.byref(real), C.byref(n1), C.byref(n2))
    if rc != 0:
        raise ValueError("sco_media_step: invalid arguments")
    return [int(x) for x in out[: n_after.value]], bool(real.value), n1.value, n2.value


def onb(n):
    """Duff et al.'s orthonormal basis (t1, t2) about unit n (float32)."""
    n = np.ascontiguousarray(n, dtype=np.float32)
    t1 = np.zeros(3, np.float32)
    t2 = np.zeros(3, np.float32)
    lib().sco_onb(_p(n), _p(t1), _p(t2))
    return t1, t2


def cosine_dir(n, u):
    """The Lambert bounce of a diffuse vertex: directions [count, 3] about
    unit n from draws u float32 [count, 2] = (u0, u1)."""
    n = np.ascontiguousarray(n, dtype=np.float32)
    u = np.ascontiguousarray(u, dtype=np.float32).reshape(-1, 2)
    out = np.zeros((len(u), 3), np.float32)
    lib().sco_cosine_dir(_p(n), len(u), _p(u), _p(out))
    return out


def camera_ray(cam, x, y, jx=0.5, jy=0.5):
    cs = camera_struct(cam)
    o = np.zeros(3, np.float32)
    d = np.zeros(3, np.float32)
    lib().sco_camera_ray(C.byref(cs), x, y, float(jx), float(jy), o.ctypes.data, d.ctypes.data)
    return o, d


# ---------------------------------------------------------------- passes

def trace_photons(osc: OracleScene, n_photons: int, max_depth: int, wl, seed: int, p0: int = 0, p1=None,
                  brute: bool = False):
    """Returns (map float32 [hc,wc,C] rounded once from FP64 sums, map_sum
    float64, count uint32, stats dict)."""
    s = osc.scene
    r = s.receiver
    Cn = wl.channels
    p1 = n_photons if p1 is None else p1
    msum = np.zeros((r.hc, r.wc, Cn), np.float64)
    cnt = np.zeros((r.hc, r.wc, Cn), np.uint32)
    st = PhotonStatsS()
    w = wavelengths_struct(wl)
    rc = lib().sco_trace_photons(C.byref(osc.c), None if brute else osc.bvh, n_photons, p0, p1, max_depth,
                                 C.byref(w), seed, msum.ctypes.data, cnt.ctypes.data, C.byref(st))
    assert rc == 0, rc
    stats = {k: (st.flux[i], st.count[i]) for i, k in enumerate(PH_OUTCOMES)}
    stats["segments"] = st.segments
    return msum.astype(np.float32), msum, cnt, stats


def render_outputs(cam, want_tie: bool = False):
    """Full-size output arrays of a render (miss values where unwritten)."""
    H, W = cam.h, cam.w
    out = dict(rgb=np.zeros((H, W, 3), np.float32), obj=np.zeros((H, W), np.uint32),
               trans=np.zeros((H, W), np.uint8), tri=np.full((H, W), 0xFFFFFFFF, np.uint32),
               depth=np.zeros((H, W), np.float32), depthn=np.zeros((H, W), np.float32),
               normal=np.zeros((H, W, 3), np.float32), normal_cam=np.zeros((H, W, 3), np.float32),
               albedo=np.zeros((H, W), np.float32))
    if want_tie:
        out["tie"] = np.zeros((H, W), np.uint8)
    return out


def render(osc: OracleScene, cam, spp: int, max_depth: int, wl, seed: int, caustic_map=None, pixels=None,
           want_tie: bool = False, brute: bool = False, out=None):
    """Returns a dict of full-size arrays (only listed pixels written) and
    the number of ray queries made.  `out` (from render_outputs) is written
    in place when given; calls on disjoint pixel lists may share it."""
    if out is None:
        out = render_outputs(cam, want_tie)
    else:
        out = {k: v for k, v in out.items() if k != "segments"}
    a = AovS()
    for k, v in out.items():
        setattr(a, k, v.ctypes.data)
    cs = camera_struct(cam)
    w = wavelengths_struct(wl)
    cmap = None if caustic_map is None else np.ascontiguousarray(caustic_map, dtype=np.float32)
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.uint32)
    seg = C.c_uint64()
    rc = lib().sco_render(C.byref(osc.c), None if brute else osc.bvh, C.byref(cs), spp, max_depth, C.byref(w),
                          seed, _p(cmap), _p(pix), 0 if pix is None else len(pix), C.byref(a), C.byref(seg))
    assert rc == 0, rc
    out["segments"] = seg.value
    return out


def pm_trace(osc: OracleScene, n_photons: int, max_depth: int, wl, seed: int, p0: int = 0, p1=None):
    """General photon map pass: (records PM_REC_DTYPE in photon order, stats)."""
    p1 = n_photons if p1 is None else p1
    cap = max(p1 - p0, 1)
    recs = np.zeros(cap, PM_REC_DTYPE)
    n = C.c_uint64()
    st = PhotonStatsS()
    w = wavelengths_struct(wl)
    rc = lib().sco_pm_trace(C.byref(osc.c), osc.bvh, n_photons, p0, p1, max_depth, C.byref(w), seed,
                            recs.ctypes.data, cap, C.byref(n), C.byref(st))
    assert rc == 0, rc
    stats = {k: (st.flux[i], st.count[i]) for i, k in enumerate(PH_OUTCOMES)}
    stats["segments"] = st.segments
    return recs[: n.value].copy(), stats


def pm_scale(recs):
    recs = np.ascontiguousarray(recs, dtype=PM_REC_DTYPE)
    return lib().sco_pm_scale(recs.ctypes.data, len(recs))


def pm_gather(recs, radius, P, N, channel):
    recs = np.ascontiguousarray(recs, dtype=PM_REC_DTYPE)
    P = np.ascontiguousarray(P, dtype=np.float32)
    N = np.ascontiguousarray(N, dtype=np.float32)
    return lib().sco_pm_gather(recs.ctypes.data, len(recs), float(radius), P.ctypes.data, N.ctypes.data, int(channel))


def render_pm(osc: OracleScene, cam, spp: int, max_depth: int, wl, seed: int, recs, radius: float, pixels=None):
    """sco_render with the general photon map; returns the same dict as render()."""
    H, W = cam.h, cam.w
    out = dict(rgb=np.zeros((H, W, 3), np.float32), obj=np.zeros((H, W), np.uint32),
               trans=np.zeros((H, W), np.uint8), tri=np.full((H, W), 0xFFFFFFFF, np.uint32),
               depth=np.zeros((H, W), np.float32), depthn=np.zeros((H, W), np.float32),
               normal=np.zeros((H, W, 3), np.float32), normal_cam=np.zeros((H, W, 3), np.float32),
               albedo=np.zeros((H, W), np.float32))
    a = AovS()
    for k, v in out.items():
        setattr(a, k, v.ctypes.data)
    recs = np.ascontiguousarray(recs, dtype=PM_REC_DTYPE)
    pix = None if pixels is None else np.ascontiguousarray(pixels, dtype=np.uint32)
    seg = C.c_uint64()
    rc = lib().sco_render_pm(C.byref(osc.c), osc.bvh, C.byref(camera_struct(cam)), spp, max_depth,
                             C.byref(wavelengths_struct(wl)), seed, recs.ctypes.data if len(recs) else None,
                             len(recs), float(radius), _p(pix), 0 if pix is None else len(pix), C.byref(a),
                             C.byref(seg))
    assert rc == 0, rc
    out["segments"] = seg.value
    return out


def path_samples(osc: OracleScene, cam, spp, max_depth, wl, seed, pixels, caustic_map=None):
    pix = np.ascontiguousarray(pixels, dtype=np.uint32)
    K = wl.k if wl.mode == 0 else 1
    L = np.zeros((spp, len(pix), K), np.float32)
    lam = np.zeros((spp, len(pix), K), np.float32)
    cs = camera_struct(cam)
    w = wavelengths_struct(wl)
    cmap = None if caustic_map is None else np.ascontiguousarray(caustic_map, dtype=np.float32)
    rc = lib().sco_path_samples(C.byref(osc.c), osc.bvh, C.byref(cs), spp, max_depth, C.byref(w), seed,
                                _p(cmap), pix.ctypes.data, len(pix), L.ctypes.data, lam.ctypes.data)
    assert rc == 0
    return L, lam
