"""Benchmark of the rendering hot path on one MI355X.

One step = the whole path over the large workload (1920x1080, 64 spp
spectral 380-720 nm, depth 16, 2^24 caustic photons into a 2048x2048x16
map; 40 overlapping glass meshes and diffuse clutter, 2,006,734 triangles,
two area lights): GPU BVH build, photon pass into the caustic map,
ground-truth pass (pixel-centre rays) and the spectral path-traced image
gathering the caustic map.  The scene arrays are resident in HBM before
anything is timed.

value = traced ray segments per second over the timed steps (camera and
ground-truth closest hits + shadow any hits + photon closest hits), in
Mrays/s.  The JSON line also carries the roofline of the traversal kernel
with the most time per step (HBM bandwidth, in algorithmic bytes per ray:
32 B ray in + 16 B hit out (4 B for a shadow ray) + node visits x 256 B +
triangle tests x 36 B, the visit counts from a counting pass of the same
kernels), its VALU fraction (14 operations per child box x 8 children per
node + 40 per triangle, against 39.3 T lane operations per second), the
same figures for the other traversal kernels, the medium workload's step,
the CPU oracle timed on the host (one core and all cores) on a bounded
sample of the same workload, and further workloads (richer glass, general
photon map, U-Net, ground truth, denoised vs plain 1080p frames, the
64-scene batch).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s; 1080p frames/s at relMSE≤0.01 vs 1024spp, denoised vs plain"
HBM_PEAK_GBS = 8000.0
# unpacked VALU lane operations per second: 256 CUs x 64 lanes x 2.4 GHz
VALU_PEAK_GOPS = 256 * 64 * 2.4
NODE_BYTES, TRI_BYTES = 256, 36          # uncompressed 8-wide node; a triangle's three vertices
RAY_IN, HIT_OUT, OCC_OUT = 32, 16, 4     # ray record read; closest hit written; occlusion written
OPS_PER_NODE, OPS_PER_TRI = 14 * 8, 40   # VALU operations per node visit (8 child boxes) and per triangle test
# what the traversal's loads request: 14 float4 of a node (its 32 pad bytes
# are not read) and a triangle's padded 48-byte record
NODE_FETCH, TRI_FETCH = 14 * 16, 48
TRAFFIC_FILES = {"large": os.path.join(ROOT, "profiles", "traversal_large_traffic.md"),
                 "medium": os.path.join(ROOT, "profiles", "traversal_medium_traffic.md")}


def _src_hash():
    h = hashlib.sha256()
    for f in ("trace.hip", "sc_path.h", "sc_device.h", "sc_kernels.h", "sc_types.h", "bvh.hip"):
        with open(os.path.join(ROOT, "paper_2107_11008_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_per_launch(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary, or None when absent or taken on different
    kernel sources."""
    path = TRAFFIC_FILES[workload]
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source_hash:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch " + re.escape(kernel) + r":\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != _src_hash():
        return None
    return float(b.group(1))


def _host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(cfg, rays_per_step, step_s):
    """The oracle (single-threaded C, unchanged) on a bounded sample of the
    workload.  One core: every 16th pixel of every 16th row (1/256 of the
    pixels) at full spp and depth, and photons [0, N/64).  All host cores:
    every 8th pixel of every 8th row (1/64) and photons [0, N/16), split
    over one thread per core, each a call of the same oracle on its own
    photon range or pixel slices (the oracle's own parallel driver)."""
    import numpy as np

    import oracle
    import oracle.parallel as op
    scene, wl, cam = cfg["scene"], cfg["wavelengths"], cfg["camera"]
    t0 = time.perf_counter()
    osc = oracle.OracleScene(scene)
    t_bvh = time.perf_counter() - t0
    n_ph, md = cfg["n_photons"], cfg["max_depth"]

    def run(step, photon_frac, threads):
        p1 = n_ph // photon_frac
        ys, xs = np.meshgrid(np.arange(0, cam.h, step), np.arange(0, cam.w, step), indexing="ij")
        pix = (ys * cam.w + xs).ravel().astype(np.uint32)
        t0 = time.perf_counter()
        if threads == 1:
            m, _, _, st = oracle.trace_photons(osc, n_ph, md, wl, cfg["photon_seed"], p0=0, p1=p1)
        else:
            m, _, _, st = op.trace_photons(osc, n_ph, md, wl, cfg["photon_seed"], p0=0, p1=p1, threads=threads)
        t_ph = time.perf_counter() - t0
        t0 = time.perf_counter()
        if threads == 1:
            out = oracle.render(osc, cam, cfg["spp"], md, wl, cfg["render_seed"], caustic_map=m, pixels=pix)
        else:
            out = op.render(osc, cam, cfg["spp"], md, wl, cfg["render_seed"], caustic_map=m, pixels=pix,
                            threads=threads)
        t_r = time.perf_counter() - t0
        rays = st["segments"] + out["segments"]
        secs = t_ph + t_r
        rate = rays / secs
        return {"value": round(rate / 1e6, 4), "unit": "Mrays/s", "cores": threads, "kind": "oracle",
                "sample": f"every {step}th pixel of every {step}th row ({len(pix)} px) at {cfg['spp']} spp, depth "
                          f"{md}, and photons [0, {p1}) of {n_ph}: {rays} ray segments in {secs:.2f} s "
                          f"(photons {t_ph:.2f} s, image {t_r:.2f} s)",
                "full_step_s": round(rays_per_step / rate, 1)}

    one = run(16, 64, 1)
    n = op.host_threads()
    allc = run(8, 16, n) if n > 1 else one
    res = dict(allc)
    res["host"] = _host_cpu()
    res["one_core"] = one
    res["oracle_bvh_build_s"] = round(t_bvh, 2)
    res["gpu_step_ms"] = round(step_s * 1e3, 2)
    res["note"] = ("all-cores figure: one thread per host core, each running the single-threaded oracle on its "
                   "own photon range or pixel slices; full_step_s extrapolates the step's ray count at each rate")
    return res


def _kernel_roofline(name, kernel_id, launches, ms, rays_cl, rays_sh, nodes, tris, steps, workload, extra=None):
    """Roofline of one traversal kernel from its launches' HIP-event time and
    its counted visits (counting pass, scaled to the timed launches by the
    ray counts)."""
    if not launches or ms <= 0:
        return None
    f_ms = ms / launches
    alg = (rays_cl * (RAY_IN + HIT_OUT) + rays_sh * (RAY_IN + OCC_OUT) + nodes * NODE_BYTES + tris * TRI_BYTES) \
        / launches
    ops = (nodes * OPS_PER_NODE + tris * OPS_PER_TRI) / launches
    fetched = (rays_cl * (RAY_IN + HIT_OUT) + rays_sh * (RAY_IN + OCC_OUT) + nodes * NODE_FETCH
               + tris * TRI_FETCH) / launches
    gbs = alg / (f_ms * 1e-3) / 1e9
    gops = ops / (f_ms * 1e-3) / 1e9
    r = {"bound": "hbm", "kernel": name, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": _traffic_per_launch(kernel_id, workload),
         "avg_launch_ms": round(f_ms, 5), "launches": launches, "alg_bytes_per_launch": round(alg),
         "rays_per_launch": round((rays_cl + rays_sh) / launches),
         "nodes_per_ray": round(nodes / max(rays_cl + rays_sh, 1), 3),
         "tris_per_ray": round(tris / max(rays_cl + rays_sh, 1), 3),
         "valu": {"achieved_Gops": round(gops, 1), "peak_Gops": VALU_PEAK_GOPS,
                  "frac": round(gops / VALU_PEAK_GOPS, 4), "ops_per_launch": round(ops)},
         "fetched": {"bytes_per_launch": round(fetched), "GB_s": round(fetched / (f_ms * 1e-3) / 1e9, 1),
                     "frac": round(fetched / (f_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "model": "224 B per node visit, 48 B per triangle test, ray and hit as above"},
         "kernel_Mrays_s": round((rays_cl + rays_sh) / (ms * 1e-3) / 1e6, 1),
         "ms_per_step": round(ms / steps, 4)}
    if extra:
        r.update(extra)
    return r


def scene_step(ctx, cfg, steps, warmup, workload):
    """Time `steps` full steps (BVH build + photon pass + ground truth +
    image) of one workload after `warmup` untimed ones; visit counts come
    from one untimed counting step of the same kernels."""
    import torch

    import paper_2107_11008_amd as sc
    scene, wl, cam = cfg["scene"], cfg["wavelengths"], cfg["camera"]
    outs = {}
    # the scene's arrays are resident in HBM before anything is timed; each
    # step rebuilds the BVH from them into the same handle's memory
    dscene = ctx.upload_scene(scene)

    def step():
        bvh = ctx.build_bvh(dscene, out=outs.get("bvh"))
        outs["bvh"] = bvh
        ph = ctx.trace_photons(bvh, cfg["n_photons"], cfg["max_depth"], wl, cfg["photon_seed"], out=outs.get("map"))
        outs["map"] = ph["map"]
        outs["img"] = ctx.render(bvh, cam, cfg["spp"], cfg["max_depth"], wl, cfg["render_seed"],
                                 caustic_map=ph["map"], out=outs.get("img"))
        return bvh

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()

    # visit counts (the same kernels' counting variants), untimed
    ctx.reset_counters()
    ctx.set_option(sc._sc.SC_OPT_COUNT_VISITS, 1)
    bvh = step()
    cnt = ctx.counters()
    ctx.set_option(sc._sc.SC_OPT_COUNT_VISITS, 0)
    rays_per_step = cnt["rays_closest"] + cnt["rays_shadow"]
    info = bvh.info()
    del bvh

    # timed region: HIP events around every traversal launch
    ctx.reset_counters()
    ctx.set_option(sc._sc.SC_OPT_PROFILE, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c = ctx.counters()
    ctx.set_option(sc._sc.SC_OPT_PROFILE, 0)
    secs = t1 - t0

    def per(key_rays, key_c):   # counted visits per ray of the counting step
        return cnt[key_c] / max(cnt[key_rays], 1)

    closest_any = max(c["closest_rays_timed"], 1)
    rl = []
    rl.append(_kernel_roofline(
        "k_closest (staged closest-hit traversal)", "k_closest<false>", c["closest_launches"], c["closest_ms"],
        c["closest_rays_timed"], 0, per("closest_rays_timed", "node_visits") * closest_any,
        per("closest_rays_timed", "tri_tests") * closest_any, steps, workload))
    rl.append(_kernel_roofline(
        "k_anyhit (staged shadow-ray traversal)", "k_anyhit<false>", c["anyhit_launches"], c["anyhit_ms"], 0,
        c["anyhit_rays"], per("anyhit_rays", "anyhit_node_visits") * c["anyhit_rays"],
        per("anyhit_rays", "anyhit_tri_tests") * c["anyhit_rays"], steps, workload))
    cf_all = c["cam_finish_rays"] + c["cam_finish_shadow_rays"]
    cnt_cf_all = max(cnt["cam_finish_rays"] + cnt["cam_finish_shadow_rays"], 1)
    rl.append(_kernel_roofline(
        "k_finish_camera (per-lane camera path finishing)", "k_finish_camera<false, false>",
        c["cam_finish_launches"], c["cam_finish_ms"], c["cam_finish_rays"], c["cam_finish_shadow_rays"],
        cnt["cam_finish_node_visits"] / cnt_cf_all * cf_all, cnt["cam_finish_tri_tests"] / cnt_cf_all * cf_all, steps,
        workload, {"paths_per_launch": round(c["cam_finish_paths"] / max(c["cam_finish_launches"], 1))}))
    rl.append(_kernel_roofline(
        "k_finish_photons (per-lane photon path finishing)", "k_finish_photons<false>", c["finish_launches"],
        c["finish_ms"], c["finish_rays"], 0, per("finish_rays", "finish_node_visits") * c["finish_rays"],
        per("finish_rays", "finish_tri_tests") * c["finish_rays"], steps, workload,
        {"paths_per_launch": round(c["finish_paths"] / max(c["finish_launches"], 1))}))
    rl = sorted([r for r in rl if r], key=lambda r: -r["ms_per_step"])

    # breakdown of one step (separately, untimed for the headline)
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    bvh = ctx.build_bvh(dscene, out=outs["bvh"])
    torch.cuda.synchronize()
    tb1 = time.perf_counter()
    ph = ctx.trace_photons(bvh, cfg["n_photons"], cfg["max_depth"], wl, cfg["photon_seed"], out=outs["map"])
    torch.cuda.synchronize()
    tb2 = time.perf_counter()
    ctx.render(bvh, cam, cfg["spp"], cfg["max_depth"], wl, cfg["render_seed"], caustic_map=ph["map"],
               out=outs["img"])
    torch.cuda.synchronize()
    tb3 = time.perf_counter()
    rays = c["rays_closest"] + c["rays_shadow"]
    res = {"secs": secs, "rays": rays, "rays_per_step": rays_per_step,
           "ms_per_step": round(secs / steps * 1e3, 3), "Mrays_s": round(rays / secs / 1e6, 2),
           "breakdown_ms": {"bvh_build": round((tb1 - tb0) * 1e3, 3), "photons": round((tb2 - tb1) * 1e3, 3),
                            "render": round((tb3 - tb2) * 1e3, 3)},
           "bvh": {"nodes": info["n_nodes"], "depth": info["depth"], "node_bytes": info["node_bytes"],
                   "tri_bytes": info["tri_bytes"]},
           "rooflines": rl}
    outs.clear()
    del dscene
    return res


# frame schedules of the frames/s protocol: (name, render contexts, blocks per CU of their traversal grids)
def progress(msg):
    """One progress line on stderr (the JSON result stays the only line on
    stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# (name, render contexts, persistent blocks per CU of the render contexts,
#  stream of the U-Net: "side" after the next frame's photons and ground
#  truth, or "render" right after its frame's render on that render stream)
DEN_SCHEDULES = (("one", 1, 8, "side"), ("two", 2, 8, "side"), ("two_5", 2, 5, "side"),
                 ("two_r", 2, 8, "render"), ("two_r5", 2, 5, "render"), ("three_r", 3, 8, "render"))
PLAIN_SCHEDULES = (("one", 1, 8, "side"), ("two", 2, 8, "side"))


def denoise_heldout(ctx, n_scenes=8, spp_ref=1024):
    """The second half of the metric: 1080p frames/s at relMSE <= 0.01
    against a 1024-spp reference, denoised vs plain rendering, on the
    held-out large scenes (seeds 200000..200000+n-1, ~2M triangles each,
    never trained on).  Per scene two references with independent seeds
    (1024 spp, 2^22 photons) give the reference's noise floor (their relMSE,
    halved).  Accuracy is the mean relMSE over the scenes.

    Both kinds of frame run as the same two-stage pipeline over two
    streams (frame rate, not latency, is the metric): the main stream
    renders frame k as soon as its caustic map is ready, while a second
    context on a second stream traces frame k+1's photons (and, for
    denoised frames, its ground-truth buffers) and then, once frame k's
    render is done, runs frame k's U-Net.  Every timed frame does all of
    its own work; the pipeline only overlaps work of neighbouring frames.
    Each setting is timed under each schedule of its kind and keeps the
    fastest: every render on the main stream ("one"); even and odd frames
    rendering on two contexts and streams, so one frame's first bounces
    overlap the previous frame's finishing tail ("two"); and, for denoised
    frames, the same with the render contexts' persistent traversal grids
    at 5 instead of 8 blocks per CU, leaving room for the side stream's
    photon pass, ground truth and U-Net ("two_5"); and both of these with
    each frame's U-Net on its render stream right after the render, so the
    next frame's photon pass does not queue behind it on the side stream
    ("two_r", "two_r5").  `schedules` counts the scenes each schedule won.
    Plain: photon pass + render; for each photon count in {2^16, 2^18,
    2^20, 2^22, 2^24} the smallest power-of-two spp from 4 whose mean
    relMSE meets the bar, then the cheapest of those.  Denoised: photon
    pass + ground truth + render + U-Net (the committed trained weights);
    the 4-spp input at the smallest photon count in {2^16, 2^18, 2^20}
    that meets the bar is the headline, the cheapest input over spp in
    {1, 2, 4} is reported beside it.  Frame times are means over the scenes
    (the steady-state frame period: after one frame that fills the
    pipeline, the time between the first and the last completion of the
    timed frames, from HIP events, over their number; fill and drain are
    not counted, for plain and denoised frames alike)."""
    import torch

    import paper_2107_11008_amd as sc
    import scenegen as sg
    from paper_2107_11008_amd import denoiser as D
    params, meta = D.load_weights()
    if params is None:
        return None
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    main2 = torch.cuda.Stream()
    main3 = torch.cuda.Stream()
    done = torch.cuda.Stream()   # frame completions, in frame order (timing only)
    with torch.cuda.stream(side):
        ctx_gt = sc.Context(0)
        net = sc.UNet(ctx_gt, tuple(meta["widths"]), params)
    net_main = sc.UNet(ctx, tuple(meta["widths"]), params)   # U-Nets on the render streams
    with torch.cuda.stream(main2):
        ctx2 = sc.Context(0)   # a second render context for the two-render schedule
        net_main2 = sc.UNet(ctx2, tuple(meta["widths"]), params)
    with torch.cuda.stream(main3):
        ctx3 = sc.Context(0)   # a third, for the three-render schedule
        net_main3 = sc.UNet(ctx3, tuple(meta["widths"]), params)
    aov = ("albedo", "normal", "depthn", "trans")

    class Pipeline:
        """Frames k = 0, 1, ... of one scene setting.  frame() issues frame
        k's render and, on the side stream, frame k+1's photons (+ ground
        truth) and frame k's U-Net; buffers alternate between even and odd
        frames.  renders = 1: every render on the main stream; renders = 2:
        even and odd frames render on two contexts and streams, so one
        frame's first bounces overlap the previous frame's finishing tail;
        renders = 3: the same over three.  Buffers: one set per frame in
        flight (max(2, renders)).  unet_on = "render": frame k's U-Net runs
        on frame k's render stream once its ground truth is there.  Each
        frame ends with a timing event on the completion stream, which waits
        for the frames in order, so completion times never go backwards."""

        def __init__(self, bvh, cam, wl, md, spp, photons, den, renders=1, blocks=8, unet_on="side"):
            self.a = (bvh, cam, wl, md, spp, photons)
            self.den = den
            self.unet_on = unet_on
            self.k = 0
            self.b = {}
            self.rs = [(ctx, main, net_main), (ctx2, main2, net_main2), (ctx3, main3, net_main3)][:renders]
            self.nb = max(2, renders)
            self.rec = None
            for rctx, _, _ in self.rs:   # persistent traversal grids of the render contexts
                rctx.set_option(sc._sc.SC_OPT_TRACE_BLOCKS, blocks)

        def _side_work(self, f):
            bvh, cam, wl, md, spp, photons = self.a
            b = self.b
            b[f"m{f}"] = ctx_gt.trace_photons(bvh, photons, md, wl, 11, out=b.get(f"m{f}"))["map"]
            ev = torch.cuda.Event()
            ev.record(side)
            b[f"map_ev{f}"] = ev
            if self.den:
                b[f"g{f}"] = ctx_gt.render(bvh, cam, 1, md, wl, 12, outputs=aov, out=b.get(f"g{f}"))
                ev = torch.cuda.Event()
                ev.record(side)
                b[f"gt_ev{f}"] = ev

        def frame(self):
            bvh, cam, wl, md, spp, photons = self.a
            b = self.b
            i, j = self.k % self.nb, (self.k + 1) % self.nb
            rctx, rst, rnet = self.rs[self.k % len(self.rs)]
            if self.k == 0:
                e0 = torch.cuda.Event()
                e0.record(main)
                side.wait_event(e0)
                main2.wait_event(e0)
                main3.wait_event(e0)
                self._side_work(i)
            self._side_work(j)                      # frame k+1's photons (+ ground truth)
            rst.wait_event(b[f"map_ev{i}"])         # frame k's map
            if f"done_ev{i}" in b:
                rst.wait_event(b[f"done_ev{i}"])    # frame k-2 is done with this render buffer
            with torch.cuda.stream(rst):
                b[f"r{i}"] = rctx.render(bvh, cam, spp, md, wl, 12, caustic_map=b[f"m{i}"], outputs=("rgb",),
                                         out=b.get(f"r{i}"))
            self.k += 1
            if self.den and self.unet_on == "render":
                rst.wait_event(b[f"gt_ev{i}"])      # frame k's ground truth
                with torch.cuda.stream(rst):
                    b[f"den{i}"] = rnet.denoise(dict(b[f"g{i}"], rgb=b[f"r{i}"]["rgb"]), out=b.get(f"den{i}"))
                ev = torch.cuda.Event()
                ev.record(rst)
                side.wait_event(ev)                 # frame k's map and ground truth are free after this
                out_ev = ev
            else:
                e_r = torch.cuda.Event()
                e_r.record(rst)
                side.wait_event(e_r)                # frame k's render is read (U-Net) or its map freed
                if self.den:
                    b[f"den{i}"] = net.denoise(dict(b[f"g{i}"], rgb=b[f"r{i}"]["rgb"]), out=b.get(f"den{i}"))
                ev = torch.cuda.Event()
                ev.record(side)
                out_ev = ev if self.den else e_r    # the frame's image is complete
            b[f"done_ev{i}"] = ev
            done.wait_event(out_ev)
            self.rec = torch.cuda.Event(enable_timing=True)
            self.rec.record(done)
            return b[f"den{i}"] if self.den else b[f"r{i}"]["rgb"]

    def timed(p, reps):
        """Steady-state frame period of pipeline p: one frame fills the
        pipeline, then reps + 1 frames; the period is the time between the
        first and the last of their completions over reps (no fill or drain
        counted)."""
        p.frame()
        recs = []
        for _ in range(reps + 1):
            img = p.frame()
            recs.append(p.rec)
        torch.cuda.synchronize()
        return img, recs[0].elapsed_time(recs[-1]) / 1e3 / reps

    den_inputs = [(spp, ph) for ph in (1 << 16, 1 << 18, 1 << 20) for spp in (1, 2, 4)]
    plain_photons = (1 << 16, 1 << 18, 1 << 20, 1 << 22, 1 << 24)
    plain_spp = (4, 8, 16, 32, 64, 128)
    scenes = []
    for j in range(n_scenes):
        cfg = sg.config3(seed=200000 + j)
        scene, wl, cam, md = cfg["scene"], cfg["wavelengths"], cfg["camera"], cfg["max_depth"]
        bvh = ctx.build_bvh(scene)
        refs = []
        for k in range(2):
            m = ctx.trace_photons(bvh, 1 << 22, md, wl, 902 + 10 * k)["map"]
            refs.append(ctx.render(bvh, cam, spp_ref, md, wl, 901 + 10 * k, caustic_map=m, outputs=("rgb",))["rgb"])
        ref = refs[0]
        row = {"seed": 200000 + j, "triangles": scene.nt, "ref_noise_floor": D.rel_mse(refs[1], ref) / 2,
               "den": {}, "plain": {}, "den_ms": {}, "plain_ms": {}, "den_sched": {}, "plain_sched": {}}
        del refs
        # every setting is timed under each schedule of its kind and keeps
        # the fastest (the images are the same under every schedule)
        for spp, ph in den_inputs:
            img, best = None, None
            for name, renders, blocks, unet_on in DEN_SCHEDULES:
                im, t = timed(Pipeline(bvh, cam, wl, md, spp, ph, True, renders, blocks, unet_on), 6)
                img = im if img is None else img
                if best is None or t < best[1]:
                    best = (name, t)
            row["den"][(spp, ph)] = D.rel_mse(img, ref)
            row["den_ms"][(spp, ph)] = best[1] * 1e3
            row["den_sched"][(spp, ph)] = best[0]
        for ph in plain_photons:
            for spp in plain_spp:
                reps = 2 if spp <= 16 else 1
                img, best = None, None
                for name, renders, blocks, unet_on in PLAIN_SCHEDULES:
                    im, t = timed(Pipeline(bvh, cam, wl, md, spp, ph, False, renders, blocks, unet_on),
                                  max(reps, renders))
                    img = im if img is None else img
                    if best is None or t < best[1]:
                        best = (name, t)
                row["plain"][(spp, ph)] = D.rel_mse(img, ref)
                row["plain_ms"][(spp, ph)] = best[1] * 1e3
                row["plain_sched"][(spp, ph)] = best[0]
        scenes.append(row)
        progress(f"denoise protocol: held-out scene {j + 1}/{n_scenes} done")
        del bvh, ref
        torch.cuda.empty_cache()

    def mean_over(key, cand):
        vals = [r[key].get(cand) for r in scenes]
        return None if any(v is None for v in vals) else sum(vals) / len(vals)

    den = [{"spp": spp, "photons": ph, "relmse": round(mean_over("den", (spp, ph)), 5),
            "ms": round(mean_over("den_ms", (spp, ph)), 2)} for spp, ph in den_inputs]
    plain_rows = []
    for ph in plain_photons:
        for spp in plain_spp:
            e = mean_over("plain", (spp, ph))
            if e is None:
                continue
            plain_rows.append({"spp": spp, "photons": ph, "relmse": round(e, 5),
                               "ms": round(mean_over("plain_ms", (spp, ph)), 2)})
            if e <= 0.01:
                break
    d_pass = [d for d in den if d["relmse"] <= 0.01]
    four = [d for d in d_pass if d["spp"] == 4]
    d4 = min(four, key=lambda d: d["ms"]) if four else None
    dbest = min(d_pass, key=lambda d: d["ms"]) if d_pass else None
    p_pass = [d for d in plain_rows if d["relmse"] <= 0.01]
    pbest = min(p_pass, key=lambda d: d["ms"]) if p_pass else None
    res = {"scenes": f"{n_scenes} held-out large glass scenes (seeds 200000..{200000 + n_scenes - 1}), 1920x1080, "
                     f"{min(r['triangles'] for r in scenes)}..{max(r['triangles'] for r in scenes)} triangles",
           "ref_noise_floor_mean": round(sum(r["ref_noise_floor"] for r in scenes) / n_scenes, 5),
           "denoised_4spp": d4, "denoised_cheapest": dbest, "plain": pbest,
           "denoised_inputs": [(d["spp"], d["photons"], d["relmse"], d["ms"]) for d in den],
           "plain_inputs": [(d["spp"], d["photons"], d["relmse"], d["ms"]) for d in plain_rows],
           "per_scene": [{"seed": r["seed"], "ref_noise_floor": round(r["ref_noise_floor"], 5),
                          "raw_4spp_2^16": round(r["plain"].get((4, 1 << 16), float("nan")), 5),
                          "denoised_4spp_2^16": round(r["den"][(4, 1 << 16)], 5),
                          "plain_min_spp_2^20": min([s for (s, p), e in r["plain"].items()
                                                     if p == 1 << 20 and e <= 0.01], default=None)}
                         for r in scenes]}
    def schedules(key, cand):   # how many scenes each schedule won
        out = {}
        for r in scenes:
            out[r[key].get(cand)] = out.get(r[key].get(cand), 0) + 1
        return out

    if d4 is not None:
        d4["schedules"] = schedules("den_sched", (d4["spp"], d4["photons"]))
    if pbest is not None:
        pbest["schedules"] = schedules("plain_sched", (pbest["spp"], pbest["photons"]))
    if pbest is not None and d4 is not None:
        # the headline ratio: the 4-spp denoised frame against the cheapest
        # plain frame meeting the same bar
        res["fps_ratio"] = round(pbest["ms"] / d4["ms"], 2)
        # a frame's time grows about in proportion to its samples, so a
        # 4-spp input can beat an N-spp plain frame by at most about N/4
        res["fps_ratio_bound_at_4spp"] = round(pbest["spp"] / 4.0, 2)
    if pbest is not None and dbest is not None:
        res["fps_ratio_cheapest_input"] = round(pbest["ms"] / dbest["ms"], 2)
    ctx.set_option(sc._sc.SC_OPT_TRACE_BLOCKS, 8)   # the library's default, for the workloads after this one
    net.close()
    net_main.close()
    net_main2.close()
    net_main3.close()
    ctx_gt.close()
    ctx2.close()
    ctx3.close()
    return res


def batch_compare(ctx):
    """The batched form: 64 scenes of 1e3-5e5 triangles (log-uniform) at
    256^2-1024^2 pixels, 8 spp, depth 12, 2^18 photons each, rendered by the
    autotuned persistent graph launch vs one scene after another."""
    import scenegen as sg
    from paper_2107_11008_amd import autotune as A
    cfgs = [sg.config4_item(j) for j in range(64)]
    best = A.autotune(ctx, cfgs)
    res = A.compare(ctx, cfgs, best)
    res["tuning"] = {k: best[k] for k in ("width", "block_size", "blocks_per_cu", "px_per_item", "ph_per_item",
                                          "tuning_s", "cached") if k in best}
    return res


MFMA_BF16_PEAK_TFLOPS = 2500.0   # dense bf16 matrix-core peak of one MI355X


def unet_flops(widths, h, w, in_ch=9, out_ch=3):
    """2 x multiply-adds of the U-Net's convolutions on an h x w canvas (real
    channel counts, not the padded ones the kernels multiply)."""
    f, cin = 0, in_ch
    for i, c in enumerate(widths):
        p = (h >> i) * (w >> i)
        f += 2 * p * 9 * (cin * c + c * c)
        cin = c
    for i in range(len(widths) - 2, -1, -1):
        p = (h >> i) * (w >> i)
        c = widths[i]
        f += 2 * p * 9 * ((cin + c) * c + c * c)
        cin = c
    return f + 2 * h * w * cin * out_ch


def unet_1080p(ctx, reps=20):
    """U-Net inference alone on a 1920x1080 frame of synthetic buffers (the
    committed trained weights): ms per call from HIP events around `reps`
    calls, and the achieved fraction of the bf16 matrix-core peak."""
    import torch

    import paper_2107_11008_amd as sc
    from paper_2107_11008_amd import denoiser as D
    params, meta = D.load_weights()
    if params is None:
        return None
    widths = tuple(meta["widths"])
    net = sc.UNet(ctx, widths, params)
    h, w = 1080, 1920
    g = torch.Generator().manual_seed(1)
    aov = {"rgb": torch.rand((h, w, 3), generator=g), "albedo": torch.rand((h, w), generator=g),
           "normal": torch.rand((h, w, 3), generator=g) * 2 - 1, "depthn": torch.rand((h, w), generator=g),
           "trans": (torch.rand((h, w), generator=g) < 0.3).to(torch.uint8)}
    aov = {k: v.cuda() for k, v in aov.items()}   # the context runs on torch's current stream: events see it
    out = net.denoise(aov)
    for _ in range(3):
        net.denoise(aov, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        net.denoise(aov, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    hc = (h + 15) // 16 * 16            # the padded canvas the network runs on
    fl = unet_flops(widths, hc, w)
    tf = fl / (ms * 1e-3) / 1e12
    return {"widths": list(widths), "canvas": [w, hc], "ms": round(ms, 4), "gflop": round(fl / 1e9, 1),
            "achieved_tflops": round(tf, 1), "peak_tflops": MFMA_BF16_PEAK_TFLOPS,
            "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4)}


def _event_ms(fn, reps):
    """Mean ms per call of fn from HIP events on torch's current stream (the
    library context runs on it), after one untimed call."""
    import torch
    fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def unet_train_step(ctx, reps=10, batch=12, crop=128):
    """One U-Net training step (forward, loss, input and weight gradients,
    Adam) on a batch of 12 128x128 crops, the denoiser's training shape, with
    the committed network's widths: ms per step and the achieved fraction of
    the bf16 matrix-core peak, counting forward + input gradient + weight
    gradient as 3x the forward multiply-adds."""
    import torch

    import paper_2107_11008_amd as sc
    from paper_2107_11008_amd import denoiser as D
    params, meta = D.load_weights()
    if params is None:
        return None
    widths = tuple(meta["widths"])
    net = sc.UNet(ctx, widths, params)
    g = torch.Generator().manual_seed(2)
    feat = torch.rand((batch, crop, crop, 9), generator=g).cuda()
    target = torch.rand((batch, crop, crop, 3), generator=g).cuda()
    ms = _event_ms(lambda: net.train_step(feat, target, 1e-4, want_loss=False), reps)
    fl = 3 * batch * unet_flops(widths, crop, crop)
    tf = fl / (ms * 1e-3) / 1e12
    net.close()
    return {"batch": [batch, crop, crop], "ms": round(ms, 4), "gflop": round(fl / 1e9, 1),
            "achieved_tflops": round(tf, 1), "peak_tflops": MFMA_BF16_PEAK_TFLOPS,
            "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4)}


def ground_truth_1080p(ctx, reps=20):
    """Ground-truth post-processing at 1920x1080 on the held-out large
    scene's own buffers (a 1-spp render with and without the caustic gather:
    rgb, first-hit ids, transparency, depth): the local / non-local caustic
    mask, 3-pixel outlines and occlusion boundaries, each timed with HIP
    events; GB/s in algorithmic bytes (each input read once, each output
    written once) against the 8 TB/s HBM peak."""
    import scenegen as sg
    cfg = sg.config3(seed=200000)
    md, wl, cam = cfg["max_depth"], cfg["wavelengths"], cfg["camera"]
    bvh = ctx.build_bvh(cfg["scene"])
    m = ctx.trace_photons(bvh, 1 << 18, md, wl, 11)["map"]
    a = ctx.render(bvh, cam, 1, md, wl, 12, caustic_map=m, outputs=("rgb", "obj", "trans", "depth"))
    b = ctx.render(bvh, cam, 1, md, wl, 12, caustic_map=None, outputs=("rgb",))
    n = cam.w * cam.h
    legs = {"caustic_mask": (lambda: ctx.caustic_mask(a["rgb"], b["rgb"], a["trans"], 0.01), n * (12 + 12 + 1 + 1)),
            "outline_3px": (lambda: ctx.outline(a["obj"], 3), n * (4 + 1)),
            "occlusion_boundary": (lambda: ctx.occlusion_boundary(a["depth"], 0.1), n * (4 + 1))}
    res = {"pixels": n}
    for k, (fn, by) in legs.items():
        ms = _event_ms(fn, reps)
        gbs = by / (ms * 1e-3) / 1e9
        res[k] = {"us": round(ms * 1e3, 2), "alg_MB": round(by / 1e6, 1), "GB_s": round(gbs, 1),
                  "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    del bvh
    return res


def glass_variants(ctx, steps=5, warmup=2):
    """The same medium-scene step on the richer glass: every object tinted
    and every second one rough ("rich"), and the clear scene under a light
    twice the size at the same power ("soft_light_x2")."""
    import torch

    import scenegen as sg
    res = {}
    for name, kw in (("rich", dict(glass_style="rich")), ("soft_light_x2", dict(light_scale=2.0))):
        cfg = sg.config2(**kw)
        wl, cam = cfg["wavelengths"], cfg["camera"]
        dscene = ctx.upload_scene(cfg["scene"])
        outs = {}

        def step():
            outs["bvh"] = ctx.build_bvh(dscene, out=outs.get("bvh"))
            ph = ctx.trace_photons(outs["bvh"], cfg["n_photons"], cfg["max_depth"], wl, cfg["photon_seed"],
                                   out=outs.get("map"))
            outs["map"] = ph["map"]
            outs["img"] = ctx.render(outs["bvh"], cam, cfg["spp"], cfg["max_depth"], wl, cfg["render_seed"],
                                     caustic_map=ph["map"], out=outs.get("img"))

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        ctx.reset_counters()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        c = ctx.counters()
        rays = c["rays_closest"] + c["rays_shadow"]
        res[name] = {"ms_per_step": round(secs / steps * 1e3, 3), "Mrays_s": round(rays / secs / 1e6, 1),
                     "rays_per_step": rays // steps, "steps": steps}
        outs.clear()
        del dscene
    return res


def general_photon_map(ctx, reps=3):
    """The general photon map (caustic photons on every diffuse surface):
    photon pass plus hashed-grid build, and the render gathering from it,
    against the receiver map on the same scene.  Medium scene at its own
    settings (radius = one receiver cell, 3.9 mm); clutter scene = the
    large-scene generator at a quarter of its triangles, RGB floor,
    960x540, 4 spp, 2^22 photons, radius 4 mm."""
    import torch

    import scenegen as sg

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return out, (time.perf_counter() - t0) / reps * 1e3

    res = {}
    c3 = sg.config3(tri_scale=0.25, w=960, h=540, floor="rgb")
    c3.update(spp=4, n_photons=1 << 22)
    for name, cfg, radius in (("medium", sg.config2(), 4.0 / 1024), ("clutter", c3, 0.004)):
        wl, cam, md = cfg["wavelengths"], cfg["camera"], cfg["max_depth"]
        bvh = ctx.build_bvh(cfg["scene"])
        outs = {}
        ph, t_ph = timed(lambda: ctx.trace_photons(bvh, cfg["n_photons"], md, wl, cfg["photon_seed"],
                                                   out=outs.get("map")))
        outs["map"] = ph["map"]
        img, t_r = timed(lambda: ctx.render(bvh, cam, cfg["spp"], md, wl, cfg["render_seed"], caustic_map=ph["map"],
                                            outputs=("rgb",), out=outs.get("img")))
        outs["img"] = img
        holder = {}

        def pm_pass():
            holder["pm"] = ctx.pmap_trace(bvh, cfg["n_photons"], md, wl, cfg["photon_seed"], radius,
                                          out=holder.get("pm"))
            return holder["pm"]

        pm, t_pm = timed(pm_pass)
        _, t_rp = timed(lambda: ctx.render(bvh, cam, cfg["spp"], md, wl, cfg["render_seed"], pmap=pm,
                                           outputs=("rgb",), out=outs.get("img")))
        inf = pm.info()
        res[name] = {"triangles": cfg["scene"].nt, "pixels": cam.w * cam.h, "spp": cfg["spp"],
                     "photons": cfg["n_photons"], "radius_m": radius, "stored": inf["n_stored"],
                     "buckets": inf["buckets"], "map_MB": round(inf["bytes"] / 2 ** 20, 1),
                     "receiver_map": {"photons_ms": round(t_ph, 3), "render_ms": round(t_r, 3)},
                     "general_map": {"photons_and_build_ms": round(t_pm, 3), "render_ms": round(t_rp, 3)}}
        pm.close()
        del bvh, outs
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=("large", "medium"), default="large",
                    help="the step timed as the headline (medium: for profiling the medium scene alone)")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-medium", action="store_true")
    ap.add_argument("--no-denoise", action="store_true")
    ap.add_argument("--staged-depth", type=int, default=None,
                    help="bounces run as one launch per stage before per-lane path finishing "
                         "(library default if omitted; 0 = none, max depth or more = all bounces staged)")
    ap.add_argument("--photon-staged-depth", type=int, default=None,
                    help="the same for photon paths (library default if omitted)")
    ap.add_argument("--queue-cap", type=int, default=None, help="camera paths per wavefront chunk")
    ap.add_argument("--photon-cap", type=int, default=None, help="photons per photon-pass chunk")
    ap.add_argument("--trace-blocks", type=int, default=None,
                    help="blocks of 128 threads per CU in the persistent traversal grids (library default 8)")
    ap.add_argument("--builder", type=int, choices=(0, 1, 2), default=None,
                    help="BVH builder: 0 radix tree over Morton codes, 1 locally-ordered clustering, 2 by size "
                         "(the library's default)")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-glass-variants", action="store_true")
    ap.add_argument("--no-pmap", action="store_true")
    ap.add_argument("--no-unet", action="store_true")
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--no-gt", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1 "
                                   "(the multi-GPU sharding is described in the design notes, not run)"}))
        sys.exit(2)

    import torch

    import paper_2107_11008_amd as sc
    import scenegen as sg

    cfg = sg.config3() if args.workload == "large" else sg.config2()
    scene = cfg["scene"]
    ctx = sc.Context(0)
    if args.staged_depth is not None:
        ctx.set_option(sc._sc.SC_OPT_STAGED_DEPTH, args.staged_depth)
    if args.photon_staged_depth is not None:
        ctx.set_option(sc._sc.SC_OPT_PHOTON_STAGED_DEPTH, args.photon_staged_depth)
    if args.queue_cap is not None:
        ctx.set_option(sc._sc.SC_OPT_QUEUE_CAP, args.queue_cap)
    if args.photon_cap is not None:
        ctx.set_option(sc._sc.SC_OPT_PHOTON_CAP, args.photon_cap)
    if args.builder is not None:
        ctx.set_option(sc._sc.SC_OPT_BVH_BUILDER, args.builder)
    if args.trace_blocks is not None:
        ctx.set_option(sc._sc.SC_OPT_TRACE_BLOCKS, args.trace_blocks)

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    big = scene_step(ctx, cfg, args.steps, args.warmup, args.workload)
    secs = big["secs"]
    cam = cfg["camera"]
    line = {
        "metric": METRIC,
        "value": round(big["rays"] / secs / 1e6, 2),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(secs / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"large glass scene: {cam.w}x{cam.h}, {cfg['spp']} spp, wavelengths uniform 380-720 "
                                f"nm, max depth {cfg['max_depth']}, 2^24 caustic photons into a 2048x2048x16 map, "
                                f"40 overlapping glass meshes and diffuse clutter ({scene.nt} triangles), two area "
                                "lights; step = BVH build + photon pass + ground truth + image")
                   if args.workload == "large" else
                   (f"medium glass scene: {cam.w}x{cam.h}, {cfg['spp']} spp, depth {cfg['max_depth']}, 2^22 photons "
                    f"into 1024x1024x16, {scene.nt} triangles, one area light; step = BVH build + photon pass + "
                    "ground truth + image"),
                   "triangles": scene.nt, "width": cam.w, "height": cam.h, "spp": cfg["spp"],
                   "max_depth": cfg["max_depth"], "photons": cfg["n_photons"]},
        "frames_per_s": round(args.steps / secs, 3),
        "rays_per_step": big["rays_per_step"],
        "breakdown_ms": big["breakdown_ms"],
        "bvh": big["bvh"],
        "roofline": big["rooflines"][0],
        "roofline_other_traversal_kernels": big["rooflines"][1:],
        "paper": "no published renderer numbers (the paper renders with a game engine's hardware ray tracing on "
                 "2x GTX 1080 Ti and quotes no frame rates)",
    }
    progress(f"headline workload done: {line['ms_per_step']} ms per step")
    if not args.no_medium and args.workload == "large":
        c2 = sg.config2()
        med = scene_step(ctx, c2, max(args.steps, 20), args.warmup, "medium")
        line["medium_scene"] = {
            "workload": f"medium glass scene: 512x512, 16 spp, depth 12, 2^22 photons into 1024x1024x16, "
                        f"{c2['scene'].nt} triangles, one area light",
            "ms_per_step": med["ms_per_step"], "Mrays_s": med["Mrays_s"], "rays_per_step": med["rays_per_step"],
            "breakdown_ms": med["breakdown_ms"], "roofline": med["rooflines"][0],
            "roofline_other_traversal_kernels": med["rooflines"][1:]}
    if not args.no_glass_variants:
        line["glass_variants"] = glass_variants(ctx)
        progress("glass variants done")
    if not args.no_pmap:
        line["general_photon_map"] = general_photon_map(ctx)
        progress("general photon map done")
    if not args.no_unet:
        line["unet_1080p"] = unet_1080p(ctx)
    if not args.no_train:
        line["unet_train_step"] = unet_train_step(ctx)
    if not args.no_gt:
        line["ground_truth_1080p"] = ground_truth_1080p(ctx)
    progress("U-Net and ground-truth kernels done")
    if not args.no_denoise:
        line["denoise_1080p"] = denoise_heldout(ctx)
    if not args.no_batch:
        line["batch_64"] = batch_compare(ctx)
        progress("64-scene batch done")
    if not args.no_cpu_baseline:
        if args.workload == "large":
            line["cpu_baseline"] = cpu_baseline(cfg, big["rays_per_step"], secs / args.steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
