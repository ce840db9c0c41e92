"""ctypes binding of libsc.so (include/sc.h).

Argument marshalling only: every step of the rendering path runs in the
library's HIP kernels.  Device memory comes from PyTorch tensors on the
current ROCm device and kernels run on PyTorch's current stream.  If the
library is missing this module raises; there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsc.so")
_lib = None

# Live handles, released before the HIP runtime and PyTorch shut down: this
# hook is registered after torch's, so it runs first.
_live = {"batch": weakref.WeakSet(), "unet": weakref.WeakSet(), "pmap": weakref.WeakSet(), "bvh": weakref.WeakSet(),
         "ctx": weakref.WeakSet()}


def _release_all():
    for kind in ("batch", "unet", "pmap", "bvh", "ctx"):
        for obj in list(_live[kind]):
            try:
                obj.close()
            except Exception:
                pass


atexit.register(_release_all)

SC_OPT_COUNT_VISITS = 1
SC_OPT_PROFILE = 2
SC_OPT_QUEUE_CAP = 3
SC_OPT_STAGED_DEPTH = 4
SC_OPT_CONV_BIG_TILE = 5
SC_OPT_PHOTON_STAGED_DEPTH = 6
SC_OPT_PHOTON_CAP = 7
SC_OPT_BVH_BUILDER = 8
SC_OPT_TRACE_BLOCKS = 9


ABI_VERSION = 6   # must match SC_ABI_VERSION in include/sc.h


class ScError(RuntimeError):
    pass


class Material(C.Structure):
    _fields_ = [("type", C.c_uint32), ("albedo_mode", C.c_uint32), ("rho_a", C.c_float), ("rho_b", C.c_float),
                ("cauchy_a", C.c_float), ("cauchy_b", C.c_float), ("le", C.c_float), ("priority", C.c_uint32),
                ("sigma", C.c_float * 3), ("roughness", C.c_float)]


class Scene(C.Structure):
    _fields_ = [("V", C.c_void_p), ("I", C.c_void_p), ("VN", C.c_void_p), ("tri_obj", C.c_void_p),
                ("nv", C.c_uint32), ("nt", C.c_uint32),
                ("mat", C.c_void_p), ("n_mat", C.c_uint32),
                ("point_lights", C.c_void_p), ("n_pl", C.c_uint32),
                ("targets_obj", C.c_void_p), ("targets_sphere", C.c_void_p), ("n_tg", C.c_uint32),
                ("tex", C.c_void_p), ("tex_w", C.c_uint32), ("tex_h", C.c_uint32),
                ("tex_x0", C.c_float), ("tex_y0", C.c_float), ("tex_ext_u", C.c_float), ("tex_ext_v", C.c_float),
                ("recv_obj", C.c_uint32), ("recv_wc", C.c_uint32), ("recv_hc", C.c_uint32),
                ("recv_x0", C.c_float), ("recv_y0", C.c_float), ("recv_ext_u", C.c_float), ("recv_ext_v", C.c_float),
                ("tex_rgb", C.c_void_p)]


class BvhOpts(C.Structure):
    _fields_ = [("width", C.c_uint32), ("leaf_max", C.c_uint32)]


class BvhInfo(C.Structure):
    _fields_ = [("width", C.c_uint32), ("leaf_max", C.c_uint32), ("n_nodes", C.c_uint32), ("depth", C.c_uint32),
                ("node_bytes", C.c_uint64), ("tri_bytes", C.c_uint64), ("max_stack", C.c_uint32)]


class Camera(C.Structure):
    _fields_ = [("eye", C.c_float * 3), ("fwd", C.c_float * 3), ("right", C.c_float * 3), ("up", C.c_float * 3),
                ("w", C.c_uint32), ("h", C.c_uint32)]


class Wavelengths(C.Structure):
    _fields_ = [("mode", C.c_uint32), ("k", C.c_uint32), ("nm", C.c_float * 4), ("lo", C.c_float),
                ("hi", C.c_float), ("bins", C.c_uint32)]


class Aov(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("obj", C.c_void_p), ("trans", C.c_void_p), ("tri", C.c_void_p),
                ("depth", C.c_void_p), ("depthn", C.c_void_p), ("normal", C.c_void_p),
                ("normal_cam", C.c_void_p), ("albedo", C.c_void_p)]


class BatchItem(C.Structure):
    _fields_ = [("bvh", C.c_void_p), ("cam", Camera), ("spp", C.c_uint32), ("max_depth", C.c_uint32),
                ("wl", Wavelengths), ("seed", C.c_uint64), ("photon_seed", C.c_uint64), ("n_photons", C.c_uint64),
                ("caustic_map", C.c_void_p), ("out", Aov)]


class Tune(C.Structure):
    _fields_ = [("block_size", C.c_uint32), ("blocks_per_cu", C.c_uint32), ("px_per_item", C.c_uint32),
                ("use_graph", C.c_uint32), ("ph_per_item", C.c_uint32), ("bvh_width", C.c_uint32)]


class PhotonStats(C.Structure):
    _fields_ = [("flux", C.c_double * 9), ("count", C.c_uint64 * 9), ("segments", C.c_uint64)]


class PmapInfo(C.Structure):
    _fields_ = [("n_stored", C.c_uint64), ("radius", C.c_float), ("channels", C.c_uint32), ("scale", C.c_double),
                ("buckets", C.c_uint32), ("bytes", C.c_uint64)]


def _quiet_close(obj):
    """Release a handle from __del__; at interpreter shutdown (module globals
    may already be gone) the process exit frees it instead."""
    try:
        if sys is None or sys.is_finalizing():
            return
        obj.close()
    except Exception:
        pass


class Counters(C.Structure):
    _fields_ = [("rays_closest", C.c_uint64), ("rays_shadow", C.c_uint64), ("node_visits", C.c_uint64),
                ("tri_tests", C.c_uint64), ("closest_launches", C.c_uint64), ("closest_ms", C.c_double),
                ("closest_rays_timed", C.c_uint64), ("finish_launches", C.c_uint64), ("finish_ms", C.c_double),
                ("finish_paths", C.c_uint64), ("finish_rays", C.c_uint64), ("finish_node_visits", C.c_uint64),
                ("finish_tri_tests", C.c_uint64), ("anyhit_launches", C.c_uint64), ("anyhit_ms", C.c_double),
                ("anyhit_rays", C.c_uint64), ("anyhit_node_visits", C.c_uint64), ("anyhit_tri_tests", C.c_uint64),
                ("cam_finish_launches", C.c_uint64), ("cam_finish_ms", C.c_double),
                ("cam_finish_paths", C.c_uint64), ("cam_finish_rays", C.c_uint64),
                ("cam_finish_shadow_rays", C.c_uint64), ("cam_finish_node_visits", C.c_uint64),
                ("cam_finish_tri_tests", C.c_uint64)]


NODE_DTYPE = np.dtype([("lox", "<f4", 8), ("hix", "<f4", 8), ("loy", "<f4", 8), ("hiy", "<f4", 8),
                       ("loz", "<f4", 8), ("hiz", "<f4", 8), ("child", "<u4", 8), ("pad", "<u4", 8)])

PH_OUTCOMES = ("deposited", "outside", "direct", "elsewhere", "escaped", "absorbed", "truncated", "lost",
               "emit_dead")

EXPORTS = ["sc_abi_version", "sc_last_error", "sc_create", "sc_destroy", "sc_set_stream", "sc_set_option",
           "sc_sync", "sc_get_counters", "sc_reset_counters", "sc_build_bvh", "sc_bvh_rebuild", "sc_bvh_get_info",
           "sc_bvh_free", "sc_bvh_export",
           "sc_trace_rays", "sc_trace_rays_noalloc", "sc_trace_rays_noalloc_max", "sc_occluded", "sc_trace_photons",
           "sc_render", "sc_render_overlap",
           "sc_unet_create", "sc_unet_free", "sc_unet_num_params", "sc_unet_set_params", "sc_unet_get_params",
           "sc_unet_forward", "sc_unet_backward", "sc_unet_train_step", "sc_unet_features",
           "sc_unet_layer_forward", "sc_unet_layer_backward", "sc_denoise",
           "sc_batch_create", "sc_batch_run", "sc_batch_free", "sc_render_batch", "sc_autotune",
           "sc_caustic_mask", "sc_outline", "sc_occlusion_boundary",
           "sc_pmap_trace", "sc_pmap_retrace", "sc_pmap_get_info", "sc_pmap_export", "sc_pmap_gather",
           "sc_pmap_free", "sc_render_pmap"]


def load(path: str = LIB_PATH):
    """Load libsc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ScError(f"{path} is missing: build it with paper_2107_11008_amd/build.py (no CPU fallback exists)")
    L = C.CDLL(path)
    vp, u32, u64, i32 = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int32
    L.sc_abi_version.restype = u32
    L.sc_last_error.restype = C.c_char_p
    L.sc_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    L.sc_destroy.argtypes = [vp]
    L.sc_set_stream.argtypes = [vp, vp]
    L.sc_set_option.argtypes = [vp, i32, C.c_int64]
    L.sc_sync.argtypes = [vp]
    L.sc_get_counters.argtypes = [vp, C.POINTER(Counters)]
    L.sc_reset_counters.argtypes = [vp]
    L.sc_build_bvh.argtypes = [vp, C.POINTER(Scene), C.POINTER(BvhOpts), C.POINTER(vp)]
    L.sc_bvh_rebuild.argtypes = [vp, vp, C.POINTER(Scene)]
    L.sc_bvh_get_info.argtypes = [vp, C.POINTER(BvhInfo)]
    L.sc_bvh_free.argtypes = [vp]
    L.sc_bvh_export.argtypes = [vp, vp, vp]
    L.sc_trace_rays.argtypes = [vp, vp, u32, vp, vp, vp, vp, vp, vp]
    L.sc_occluded.argtypes = [vp, vp, u32, vp, vp, vp, vp, vp]
    L.sc_trace_rays_noalloc.argtypes = [vp, vp, u32, vp, vp, vp, vp, vp, vp]
    L.sc_trace_rays_noalloc_max.restype = u32
    L.sc_trace_photons.argtypes = [vp, vp, u64, u32, C.POINTER(Wavelengths), u64, vp, vp, C.POINTER(PhotonStats)]
    L.sc_render.argtypes = [vp, vp, C.POINTER(Camera), u32, u32, C.POINTER(Wavelengths), u64, vp, C.POINTER(Aov)]
    L.sc_render_overlap.argtypes = [vp, vp, C.POINTER(Camera), u32, u32, C.POINTER(Wavelengths), u64, vp, vp,
                                    C.POINTER(Aov)]
    L.sc_pmap_trace.argtypes = [vp, vp, u64, u32, C.POINTER(Wavelengths), u64, C.c_float, C.POINTER(vp),
                                C.POINTER(PhotonStats)]
    L.sc_pmap_retrace.argtypes = [vp, vp, u64, u32, C.POINTER(Wavelengths), u64, C.c_float, vp,
                                  C.POINTER(PhotonStats)]
    L.sc_pmap_get_info.argtypes = [vp, C.POINTER(PmapInfo)]
    L.sc_pmap_export.argtypes = [vp, vp, vp, vp, vp, vp]
    L.sc_pmap_gather.argtypes = [vp, vp, u32, vp, vp, vp, vp]
    L.sc_pmap_free.argtypes = [vp]
    L.sc_render_pmap.argtypes = [vp, vp, C.POINTER(Camera), u32, u32, C.POINTER(Wavelengths), u64, vp, C.POINTER(Aov)]
    L.sc_caustic_mask.argtypes = [vp, vp, vp, vp, u32, u32, C.c_float, vp]
    L.sc_outline.argtypes = [vp, vp, u32, u32, u32, vp]
    L.sc_occlusion_boundary.argtypes = [vp, vp, u32, u32, C.c_float, vp]
    L.sc_batch_create.argtypes = [vp, u32, vp, C.POINTER(Tune), C.POINTER(vp)]
    L.sc_batch_run.argtypes = [vp, vp]
    L.sc_batch_free.argtypes = [vp]
    L.sc_render_batch.argtypes = [vp, u32, vp, C.POINTER(Tune)]
    L.sc_autotune.argtypes = [vp, u32, vp, C.POINTER(Tune)]
    L.sc_unet_create.argtypes = [vp, vp, u32, C.POINTER(vp)]
    L.sc_unet_free.argtypes = [vp]
    L.sc_unet_num_params.argtypes = [vp, C.POINTER(u64)]
    L.sc_unet_set_params.argtypes = [vp, vp]
    L.sc_unet_get_params.argtypes = [vp, vp]
    L.sc_unet_forward.argtypes = [vp, vp, vp, u32, u32, u32, vp]
    L.sc_unet_backward.argtypes = [vp, vp, vp, vp]
    L.sc_unet_train_step.argtypes = [vp, vp, vp, vp, u32, u32, u32, C.c_float, C.POINTER(C.c_float)]
    L.sc_denoise.argtypes = [vp, vp, C.POINTER(Aov), u32, u32, vp]
    L.sc_unet_features.argtypes = [vp, C.POINTER(Aov), u32, u32, vp]
    L.sc_unet_layer_forward.argtypes = [vp, vp, u32, vp, u32, u32, u32, i32, vp]
    L.sc_unet_layer_backward.argtypes = [vp, vp, u32, vp, vp, u32, u32, u32, vp, vp]
    for name in EXPORTS:
        fn = getattr(L, name)
        if name not in ("sc_abi_version", "sc_last_error", "sc_trace_rays_noalloc_max"):
            fn.restype = i32
    if L.sc_abi_version() != ABI_VERSION:
        raise ScError(f"{path} has ABI version {L.sc_abi_version()}, the binding expects {ABI_VERSION}: rebuild it")
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        msg = load().sc_last_error().decode(errors="replace")
        raise ScError(f"{what} failed ({rc}): {msg}")


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA (ROCm) tensors"
    return t.data_ptr()


def _dev(a: np.ndarray, device) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


def camera_struct(cam) -> Camera:
    c = Camera()
    c.eye[:] = [float(x) for x in cam.eye]
    c.fwd[:] = [float(x) for x in cam.fwd]
    c.right[:] = [float(x) for x in cam.right]
    c.up[:] = [float(x) for x in cam.up]
    c.w, c.h = int(cam.w), int(cam.h)
    return c


def wavelengths_struct(wl) -> Wavelengths:
    w = Wavelengths()
    w.mode, w.k = int(wl.mode), int(wl.k)
    nm = list(wl.nm) + [0.0] * (4 - len(wl.nm))
    w.nm[:] = [float(x) for x in nm[:4]]
    w.lo, w.hi, w.bins = float(wl.lo), float(wl.hi), int(wl.bins)
    return w


class Context:
    """A library context bound to a device and PyTorch's current stream."""

    def __init__(self, device: int = 0):
        L = load()
        self.device = torch.device("cuda", device)
        torch.cuda.set_device(self.device)
        stream = torch.cuda.current_stream(self.device).cuda_stream
        h = C.c_void_p()
        _check(L.sc_create(device, C.c_void_p(stream), C.byref(h)), "sc_create")
        self.h = h
        _live["ctx"].add(self)

    def close(self):
        if getattr(self, "h", None):
            load().sc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            _quiet_close(self)
        except Exception:   # module globals already cleared at shutdown
            pass

    def set_option(self, opt: int, value: int):
        _check(load().sc_set_option(self.h, opt, int(value)), "sc_set_option")

    def sync(self):
        _check(load().sc_sync(self.h), "sc_sync")

    def counters(self) -> dict:
        c = Counters()
        _check(load().sc_get_counters(self.h, C.byref(c)), "sc_get_counters")
        return {k: getattr(c, k) for k, _ in Counters._fields_}

    def reset_counters(self):
        _check(load().sc_reset_counters(self.h), "sc_reset_counters")

    # ------------------------------------------------------------ entry points
    def upload_scene(self, scene) -> "SceneDev":
        """Copy a host scene (scenegen.Scene) to the device once; the result
        can be passed to build_bvh any number of times."""
        return SceneDev(self, scene)

    def build_bvh(self, scene, width: int = 8, leaf_max: int = 4, out: Optional["Bvh"] = None) -> "Bvh":
        """Wide BVH of a scene (host scenegen.Scene, uploaded on the fly, or
        a SceneDev).  With out=, that handle is rebuilt in place (same
        width and leaf size) and returned."""
        if out is not None:
            out.rebuild(scene)
            return out
        return Bvh(self, scene, width, leaf_max)

    def trace_rays(self, bvh: "Bvh", O: torch.Tensor, D: torch.Tensor):
        n = O.shape[0]
        t = torch.empty(n, dtype=torch.float32, device=self.device)
        prim = torch.empty(n, dtype=torch.int32, device=self.device)
        u = torch.empty(n, dtype=torch.float32, device=self.device)
        v = torch.empty(n, dtype=torch.float32, device=self.device)
        _check(load().sc_trace_rays(self.h, bvh.h, n, _ptr(O), _ptr(D), _ptr(t), _ptr(prim), _ptr(u), _ptr(v)),
               "sc_trace_rays")
        return t, prim, u, v

    def unet_features(self, aov: dict, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """The denoiser's input features [h][w][9] of a render's buffers
        (sc_unet_features): the same function sc_denoise applies."""
        h, w = aov["rgb"].shape[:2]
        a = Aov()
        for k in ("rgb", "albedo", "normal", "depthn", "trans"):
            if k in aov and aov[k] is not None:
                setattr(a, k, _ptr(aov[k]))
        o = out if out is not None else torch.empty((h, w, 9), dtype=torch.float32, device=self.device)
        _check(load().sc_unet_features(self.h, C.byref(a), w, h, _ptr(o)), "sc_unet_features")
        return o

    def trace_rays_noalloc(self, bvh: "Bvh", O: torch.Tensor, D: torch.Tensor, t: torch.Tensor,
                           prim: torch.Tensor, u: Optional[torch.Tensor] = None, v: Optional[torch.Tensor] = None):
        """sc_trace_rays_noalloc: closest hits into caller-given outputs,
        with no device allocation by the library (at most
        sc_trace_rays_noalloc_max() rays)."""
        _check(load().sc_trace_rays_noalloc(self.h, bvh.h, O.shape[0], _ptr(O), _ptr(D), _ptr(t), _ptr(prim),
                                            _ptr(u), _ptr(v)), "sc_trace_rays_noalloc")

    def occluded(self, bvh: "Bvh", O, D, tmax, excl=None):
        n = O.shape[0]
        occ = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(load().sc_occluded(self.h, bvh.h, n, _ptr(O), _ptr(D), _ptr(tmax), _ptr(excl), _ptr(occ)),
               "sc_occluded")
        return occ

    def trace_photons(self, bvh: "Bvh", n_photons: int, max_depth: int, wl, seed: int, counts: bool = False,
                      stats: bool = False, out: Optional[torch.Tensor] = None):
        r = bvh.scene.receiver
        shape = (r.hc, r.wc, wl.channels)
        cmap = out if out is not None else torch.empty(shape, dtype=torch.float32, device=self.device)
        cnt = torch.empty(shape, dtype=torch.int32, device=self.device) if counts else None
        st = PhotonStats() if stats else None
        w = wavelengths_struct(wl)
        _check(load().sc_trace_photons(self.h, bvh.h, int(n_photons), int(max_depth), C.byref(w), int(seed),
                                       _ptr(cmap), _ptr(cnt), C.byref(st) if st is not None else None),
               "sc_trace_photons")
        res = {"map": cmap}
        if counts:
            res["count"] = cnt
        if stats:
            res["stats"] = {k: (st.flux[i], st.count[i]) for i, k in enumerate(PH_OUTCOMES)}
            res["stats"]["segments"] = st.segments
        return res

    def render(self, bvh: "Bvh", cam, spp: int, max_depth: int, wl, seed: int,
               caustic_map: Optional[torch.Tensor] = None, outputs=("rgb", "obj", "trans", "tri", "depth", "depthn",
                                                                      "normal", "normal_cam", "albedo"),
               out: Optional[dict] = None, pmap: Optional["PhotonMap"] = None,
               map_ready: Optional[torch.cuda.Event] = None):
        """Render (sc_render); with pmap= the caustic gather comes from a
        general photon map on every diffuse surface (sc_render_pmap); with
        map_ready= (an event recorded after the photon pass that writes
        caustic_map, on another stream) the render overlaps that pass and
        waits for the event only where it first reads the map
        (sc_render_overlap)."""
        H, W = cam.h, cam.w
        shapes = dict(rgb=((H, W, 3), torch.float32), obj=((H, W), torch.int32), trans=((H, W), torch.uint8),
                      tri=((H, W), torch.int32), depth=((H, W), torch.float32), depthn=((H, W), torch.float32),
                      normal=((H, W, 3), torch.float32), normal_cam=((H, W, 3), torch.float32),
                      albedo=((H, W), torch.float32))
        res = {} if out is None else dict(out)
        a = Aov()
        for k in outputs:
            if k not in res:
                shp, dt = shapes[k]
                res[k] = torch.empty(shp, dtype=dt, device=self.device)
            setattr(a, k, _ptr(res[k]))
        cs = camera_struct(cam)
        w = wavelengths_struct(wl)
        if pmap is not None:
            _check(load().sc_render_pmap(self.h, bvh.h, C.byref(cs), int(spp), int(max_depth), C.byref(w), int(seed),
                                         pmap.h, C.byref(a)), "sc_render_pmap")
        elif map_ready is not None:
            _check(load().sc_render_overlap(self.h, bvh.h, C.byref(cs), int(spp), int(max_depth), C.byref(w),
                                            int(seed), _ptr(caustic_map), C.c_void_p(map_ready.cuda_event),
                                            C.byref(a)), "sc_render_overlap")
        else:
            _check(load().sc_render(self.h, bvh.h, C.byref(cs), int(spp), int(max_depth), C.byref(w), int(seed),
                                    _ptr(caustic_map), C.byref(a)), "sc_render")
        return res

    def pmap_trace(self, bvh: "Bvh", n_photons: int, max_depth: int, wl, seed: int, radius: float,
                   stats: bool = False, out: Optional["PhotonMap"] = None) -> "PhotonMap":
        """General photon map: caustic photons stored on every diffuse surface
        (sc_pmap_trace; with out=, rebuilt in that handle's memory by
        sc_pmap_retrace).  With stats=True the outcome statistics are kept
        in the result's .stats."""
        st = PhotonStats() if stats else None
        w = wavelengths_struct(wl)
        pst = C.byref(st) if st is not None else None
        if out is not None:
            _check(load().sc_pmap_retrace(self.h, bvh.h, int(n_photons), int(max_depth), C.byref(w), int(seed),
                                          float(radius), out.h, pst), "sc_pmap_retrace")
            pm = out
        else:
            h = C.c_void_p()
            _check(load().sc_pmap_trace(self.h, bvh.h, int(n_photons), int(max_depth), C.byref(w), int(seed),
                                        float(radius), C.byref(h), pst), "sc_pmap_trace")
            pm = PhotonMap(self, h)
        if stats:
            pm.stats = {k: (st.flux[i], st.count[i]) for i, k in enumerate(PH_OUTCOMES)}
            pm.stats["segments"] = st.segments
        return pm


def _gt_methods():
    def caustic_mask(self, rgb_with, rgb_without, trans=None, threshold: float = 0.0):
        h, w = rgb_with.shape[:2]
        m = torch.empty((h, w), dtype=torch.uint8, device=self.device)
        _check(load().sc_caustic_mask(self.h, _ptr(rgb_with), _ptr(rgb_without), _ptr(trans), w, h,
                                      float(threshold), _ptr(m)), "sc_caustic_mask")
        return m

    def render_caustic_mask(self, bvh, cam, spp, max_depth, wl, seed, caustic_map, rel: float = 0.05):
        """Renders with and without the caustic gather (same seeds) and
        thresholds the luminance difference at rel x the mean luminance of
        the render with caustics."""
        a = self.render(bvh, cam, spp, max_depth, wl, seed, caustic_map=caustic_map, outputs=("rgb", "trans"))
        b = self.render(bvh, cam, spp, max_depth, wl, seed, caustic_map=None, outputs=("rgb",))
        lum = (0.2126 * a["rgb"][..., 0].double() + 0.7152 * a["rgb"][..., 1].double()
               + 0.0722 * a["rgb"][..., 2].double())
        thr = float(rel * float(lum.mean()))
        return self.caustic_mask(a["rgb"], b["rgb"], a["trans"], thr), a, b, thr

    def outline(self, obj, thickness: int = 1):
        h, w = obj.shape
        o = torch.empty((h, w), dtype=torch.uint8, device=self.device)
        _check(load().sc_outline(self.h, _ptr(obj), w, h, int(thickness), _ptr(o)), "sc_outline")
        return o

    def occlusion_boundary(self, depth, rel_jump: float = 0.1):
        h, w = depth.shape
        o = torch.empty((h, w), dtype=torch.uint8, device=self.device)
        _check(load().sc_occlusion_boundary(self.h, _ptr(depth), w, h, float(rel_jump), _ptr(o)),
               "sc_occlusion_boundary")
        return o

    Context.caustic_mask = caustic_mask
    Context.render_caustic_mask = render_caustic_mask
    Context.outline = outline
    Context.occlusion_boundary = occlusion_boundary


class SceneDev:
    """A scene's arrays on the device and the sc_scene describing them."""

    def __init__(self, ctx: Context, scene):
        if isinstance(scene, SceneDev):
            scene = scene.scene
        self.scene = scene
        dev = ctx.device
        self.V = _dev(scene.V, dev)
        self.I = _dev(scene.I.view(np.int32), dev)
        self.VN = _dev(scene.VN, dev) if scene.VN is not None else None
        self.tri_obj = _dev(scene.tri_obj.view(np.int32), dev)
        self.tex = _dev(scene.tex, dev) if scene.tex is not None else None
        self.tex_rgb = _dev(scene.tex_rgb, dev) if getattr(scene, "tex_rgb", None) is not None else None
        self._mat = np.ascontiguousarray(scene.materials)
        self._pl = np.ascontiguousarray(scene.point_lights, dtype=np.float32)
        self._tgo = np.ascontiguousarray(scene.targets_obj, dtype=np.uint32)
        self._tgs = np.ascontiguousarray(scene.targets_sphere, dtype=np.float32)
        s = Scene()
        s.V, s.I, s.VN, s.tri_obj = _ptr(self.V), _ptr(self.I), _ptr(self.VN), _ptr(self.tri_obj)
        s.nv, s.nt = scene.nv, scene.nt
        s.mat, s.n_mat = self._mat.ctypes.data, len(self._mat)
        s.point_lights, s.n_pl = (self._pl.ctypes.data if len(self._pl) else None), len(self._pl)
        s.targets_obj = self._tgo.ctypes.data if len(self._tgo) else None
        s.targets_sphere = self._tgs.ctypes.data if len(self._tgs) else None
        s.n_tg = len(self._tgo)
        if self.tex is not None:
            s.tex, s.tex_h, s.tex_w = _ptr(self.tex), scene.tex.shape[0], scene.tex.shape[1]
            s.tex_x0, s.tex_y0, s.tex_ext_u, s.tex_ext_v = scene.tex_rect
        if self.tex_rgb is not None:
            s.tex_rgb, s.tex_h, s.tex_w = _ptr(self.tex_rgb), scene.tex_rgb.shape[0], scene.tex_rgb.shape[1]
            s.tex_x0, s.tex_y0, s.tex_ext_u, s.tex_ext_v = scene.tex_rect
        r = scene.receiver
        if r is not None:
            s.recv_obj, s.recv_wc, s.recv_hc = r.obj, r.wc, r.hc
            s.recv_x0, s.recv_y0, s.recv_ext_u, s.recv_ext_v = r.x0, r.y0, r.ext_u, r.ext_v
        self.s = s

    # the scene's attributes (nt, nv, V, ...) as on the host scene
    def __getattr__(self, name):
        return getattr(self.__dict__["scene"], name)


class Bvh:
    """A scene on the device plus its wide BVH and tables.  Holds the
    SceneDev it was built from (the tree references its arrays)."""

    def __init__(self, ctx: Context, scene, width: int = 8, leaf_max: int = 4):
        self.ctx = ctx
        self.dev = scene if isinstance(scene, SceneDev) else SceneDev(ctx, scene)
        self.scene = self.dev.scene
        opts = BvhOpts(width, leaf_max)
        h = C.c_void_p()
        _check(load().sc_build_bvh(ctx.h, C.byref(self.dev.s), C.byref(opts), C.byref(h)), "sc_build_bvh")
        self.h = h
        _live["bvh"].add(self)

    def rebuild(self, scene):
        """Rebuild this handle's tree for scene (host scene or SceneDev),
        reusing its device memory."""
        dev = scene if isinstance(scene, SceneDev) else SceneDev(self.ctx, scene)
        _check(load().sc_bvh_rebuild(self.ctx.h, self.h, C.byref(dev.s)), "sc_bvh_rebuild")
        self.dev = dev
        self.scene = dev.scene

    def info(self) -> dict:
        i = BvhInfo()
        _check(load().sc_bvh_get_info(self.h, C.byref(i)), "sc_bvh_get_info")
        return {k: getattr(i, k) for k, _ in BvhInfo._fields_}

    def export(self):
        """Host copies of the wide nodes (structured array) and the
        leaf-ordered triangles ([nt, 3, 4] float32, index bits in [:, 0, 3])."""
        inf = self.info()
        nodes = np.zeros(inf["n_nodes"], dtype=NODE_DTYPE)
        tris = np.zeros((self.scene.nt, 3, 4), dtype=np.float32)
        _check(load().sc_bvh_export(self.h, nodes.ctypes.data, tris.ctypes.data), "sc_bvh_export")
        return nodes, tris

    def close(self):
        if getattr(self, "h", None):
            load().sc_bvh_free(self.h)
            self.h = None

    def __del__(self):
        try:
            _quiet_close(self)
        except Exception:   # module globals already cleared at shutdown
            pass


class PhotonMap:
    """A general photon map on the device (sc_pmap_*)."""

    def __init__(self, ctx: Context, h):
        self.ctx = ctx
        self.h = h
        self.stats = None
        _live["pmap"].add(self)

    def info(self) -> dict:
        i = PmapInfo()
        _check(load().sc_pmap_get_info(self.h, C.byref(i)), "sc_pmap_get_info")
        return {k: getattr(i, k) for k, _ in PmapInfo._fields_}

    def export(self) -> dict:
        """Host copies of the stored photons in photon-index order."""
        n = self.info()["n_stored"]
        out = dict(pos=np.zeros((n, 3), np.float32), nrm=np.zeros((n, 3), np.float32), phi=np.zeros(n, np.float32),
                   channel=np.zeros(n, np.uint32), photon=np.zeros(n, np.uint64))
        _check(load().sc_pmap_export(self.h, *[out[k].ctypes.data for k in ("pos", "nrm", "phi", "channel", "photon")]),
               "sc_pmap_export")
        return out

    def gather(self, P: torch.Tensor, N: torch.Tensor, ch: torch.Tensor) -> torch.Tensor:
        """Irradiance estimates at device points P [n, 3] with facing normals
        N [n, 3] for channels ch [n] (int32)."""
        n = P.shape[0]
        E = torch.empty(n, dtype=torch.float32, device=self.ctx.device)
        _check(load().sc_pmap_gather(self.ctx.h, self.h, n, _ptr(P), _ptr(N), _ptr(ch), _ptr(E)), "sc_pmap_gather")
        return E

    def close(self):
        if getattr(self, "h", None):
            load().sc_pmap_free(self.h)
            self.h = None

    def __del__(self):
        try:
            _quiet_close(self)
        except Exception:   # module globals already cleared at shutdown
            pass


class UNet:
    """The denoiser network on the device (sc_unet_*)."""

    def __init__(self, ctx: Context, widths=(32, 48, 64, 96, 128), params: Optional[np.ndarray] = None):
        self.ctx = ctx
        self.widths = tuple(int(w) for w in widths)
        arr = (C.c_uint32 * len(self.widths))(*self.widths)
        h = C.c_void_p()
        _check(load().sc_unet_create(ctx.h, arr, len(self.widths), C.byref(h)), "sc_unet_create")
        self.h = h
        _live["unet"].add(self)
        n = C.c_uint64()
        _check(load().sc_unet_num_params(self.h, C.byref(n)), "sc_unet_num_params")
        self.n_params = n.value
        # (cout, k, cin) of every convolution in parameter order
        L, cin = [], 9
        for w in self.widths:
            L += [(w, 3, cin), (w, 3, w)]
            cin = w
        for i in range(len(self.widths) - 2, -1, -1):
            L += [(self.widths[i], 3, cin + self.widths[i]), (self.widths[i], 3, self.widths[i])]
            cin = self.widths[i]
        L.append((3, 1, cin))
        self.layer_shapes = L
        if params is not None:
            self.set_params(params)

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == self.n_params
        _check(load().sc_unet_set_params(self.h, p.ctypes.data), "sc_unet_set_params")

    def get_params(self) -> np.ndarray:
        p = np.empty(self.n_params, np.float32)
        _check(load().sc_unet_get_params(self.h, p.ctypes.data), "sc_unet_get_params")
        return p

    def forward(self, feat: torch.Tensor) -> torch.Tensor:
        n, h, w, c = feat.shape
        assert c == 9
        pred = torch.empty((n, h, w, 3), dtype=torch.float32, device=self.ctx.device)
        _check(load().sc_unet_forward(self.ctx.h, self.h, _ptr(feat), n, w, h, _ptr(pred)), "sc_unet_forward")
        return pred

    def backward(self, dpred: torch.Tensor) -> torch.Tensor:
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.ctx.device)
        _check(load().sc_unet_backward(self.ctx.h, self.h, _ptr(dpred), _ptr(g)), "sc_unet_backward")
        return g

    def train_step(self, feat: torch.Tensor, target: torch.Tensor, lr: float, want_loss: bool = True):
        n, h, w, _ = feat.shape
        loss = C.c_float()
        _check(load().sc_unet_train_step(self.ctx.h, self.h, _ptr(feat), _ptr(target), n, w, h, float(lr),
                                         C.byref(loss) if want_loss else None), "sc_unet_train_step")
        return loss.value if want_loss else None

    def layer_forward(self, layer: int, x: torch.Tensor, relu: bool = True) -> torch.Tensor:
        """sc_unet_layer_forward: one convolution of the network alone;
        x float [n][h][w][cin] -> float [n][h][w][cout]."""
        n, h, w, _ = x.shape
        cout = self.layer_shapes[layer][0]
        y = torch.empty((n, h, w, cout), dtype=torch.float32, device=self.ctx.device)
        _check(load().sc_unet_layer_forward(self.ctx.h, self.h, layer, _ptr(x), n, h, w, int(relu), _ptr(y)),
               "sc_unet_layer_forward")
        return y

    def layer_backward(self, layer: int, x: torch.Tensor, dz: torch.Tensor):
        """sc_unet_layer_backward: (dX float [n][h][w][cin], dW float
        [cout*k*k*cin + cout]) of one convolution given dz."""
        n, h, w, cin = x.shape
        cout, k, _ = self.layer_shapes[layer]
        dx = torch.empty_like(x)
        dw = torch.empty(cout * k * k * cin + cout, dtype=torch.float32, device=self.ctx.device)
        _check(load().sc_unet_layer_backward(self.ctx.h, self.h, layer, _ptr(x), _ptr(dz), n, h, w, _ptr(dx), _ptr(dw)),
               "sc_unet_layer_backward")
        return dx, dw

    def denoise(self, aov: dict, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        h, w = aov["rgb"].shape[:2]
        a = Aov()
        for k in ("rgb", "albedo", "normal", "depthn", "trans"):
            if k in aov and aov[k] is not None:
                setattr(a, k, _ptr(aov[k]))
        o = out if out is not None else torch.empty((h, w, 3), dtype=torch.float32, device=self.ctx.device)
        _check(load().sc_denoise(self.ctx.h, self.h, C.byref(a), w, h, _ptr(o)), "sc_denoise")
        return o

    def close(self):
        if getattr(self, "h", None):
            load().sc_unet_free(self.h)
            self.h = None

    def __del__(self):
        try:
            _quiet_close(self)
        except Exception:   # module globals already cleared at shutdown
            pass


_gt_methods()


def _batch_items(ctx: "Context", items, outs_keep: list):
    """The sc_batch_item array for a list of item dicts (see Batch), with
    output tensors allocated here and appended to outs_keep."""
    arr = (BatchItem * len(items))()
    for i, it in enumerate(items):
        a = arr[i]
        a.bvh = it["bvh"].h
        a.cam = camera_struct(it["cam"])
        a.spp, a.max_depth = int(it["spp"]), int(it["max_depth"])
        a.wl = wavelengths_struct(it["wl"])
        a.seed, a.photon_seed, a.n_photons = int(it["seed"]), int(it.get("photon_seed", 0)), int(it.get("n_photons", 0))
        cm = it.get("caustic_map")
        if cm is None and a.n_photons:
            r = it["bvh"].scene.receiver
            cm = torch.empty((r.hc, r.wc, it["wl"].channels), dtype=torch.float32, device=ctx.device)
        a.caustic_map = _ptr(cm)
        H, W = it["cam"].h, it["cam"].w
        outs = {"caustic_map": cm}
        for k in it.get("outputs", ("rgb", "obj", "trans", "tri", "depth", "depthn", "normal", "normal_cam",
                                    "albedo")):
            c, dt = Batch._SHAPES[k]
            outs[k] = torch.empty((H, W) if c is None else (H, W, c), dtype=dt, device=ctx.device)
            setattr(a.out, k, _ptr(outs[k]))
        outs_keep.append(outs)
    return arr


def autotune_batch(ctx: "Context", items) -> dict:
    """sc_autotune: the fastest batch setting for these items (their output
    buffers, allocated here, are scratch)."""
    keep = []
    arr = _batch_items(ctx, items, keep)
    t = Tune()
    _check(load().sc_autotune(ctx.h, len(items), C.cast(arr, C.c_void_p), C.byref(t)), "sc_autotune")
    return {k: getattr(t, k) for k, _ in Tune._fields_}


class Batch:
    """Many scenes rendered by the persistent, graph-captured batch kernels.

    items: list of dicts with keys bvh, cam, spp, max_depth, wl, seed,
    photon_seed, n_photons and optionally caustic_map (tensor) and outputs
    (names as in Context.render).  Output tensors are allocated here and
    returned by outputs()."""

    _SHAPES = dict(rgb=(3, torch.float32), obj=(None, torch.int32), trans=(None, torch.uint8),
                   tri=(None, torch.int32), depth=(None, torch.float32), depthn=(None, torch.float32),
                   normal=(3, torch.float32), normal_cam=(3, torch.float32), albedo=(None, torch.float32))

    def __init__(self, ctx: Context, items, tune: Optional[dict] = None):
        self.ctx = ctx
        self.items = items
        self._outs = []
        self._keep = []
        arr = _batch_items(ctx, items, self._outs)
        self._arr = arr
        t = None
        if tune is not None:
            t = Tune(int(tune["block_size"]), int(tune["blocks_per_cu"]), int(tune["px_per_item"]),
                     int(tune.get("use_graph", 1)), int(tune.get("ph_per_item", 0)), int(tune.get("bvh_width", 8)))
        h = C.c_void_p()
        _check(load().sc_batch_create(ctx.h, len(items), C.cast(arr, C.c_void_p), C.byref(t) if t else None,
                                      C.byref(h)), "sc_batch_create")
        self.h = h
        _live["batch"].add(self)

    def run(self):
        _check(load().sc_batch_run(self.ctx.h, self.h), "sc_batch_run")

    def outputs(self):
        return self._outs

    def close(self):
        if getattr(self, "h", None):
            load().sc_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            _quiet_close(self)
        except Exception:   # module globals already cleared at shutdown
            pass
