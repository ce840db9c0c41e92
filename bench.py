"""Benchmark of the rendering hot path on one MI355X.

One step = the whole path over the medium workload (512x512, 16 spp
spectral 380-720 nm, depth 12, 2^22 caustic photons, eight glass objects of
~198k triangles on a textured plane with an area light): GPU BVH build,
photon pass into the caustic map, ground-truth pass (pixel-centre rays)
and the spectral path-traced image gathering the caustic map.

value = traced ray segments per second over the timed steps (camera and
ground-truth closest hits + shadow any hits + photon closest hits), in
Mrays/s.  The JSON line also carries the roofline of the dominant kernel
(closest-hit traversal, bound by HBM bandwidth; algorithmic bytes per ray
= 24 B ray + 4 B queue entry + 16 B hit + node visits x 256 B + triangle
tests x 48 B, the visit counts taken from a counting pass of the same
kernel) and the CPU oracle timed on a bounded sample of the same workload.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traversal_c2_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2107_11008_amd", "csrc", "trace.hip")


def _src_hash():
    h = hashlib.sha256()
    for f in ("trace.hip", "sc_path.h", "sc_device.h", "sc_kernels.h", "sc_types.h", "bvh.hip"):
        with open(os.path.join(ROOT, "paper_2107_11008_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_per_launch(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when absent or taken on different kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"source_hash:\s*([0-9a-f]+)", txt)
    b = re.search(r"hbm_bytes_per_launch " + re.escape(kernel) + r":\s*([0-9.eE+]+)", txt)
    if not m or not b or m.group(1) != _src_hash():
        return None
    return float(b.group(1))


def cpu_baseline(cfg, rays_per_step, step_s):
    """The oracle (single-threaded C) on a bounded sample of the workload:
    every 2nd pixel of every 2nd row (1/4 of the pixels) at full spp and
    depth, and the first 1/8 of the photons (about 10 s of one core)."""
    import numpy as np

    import oracle
    scene, wl, cam = cfg["scene"], cfg["wavelengths"], cfg["camera"]
    t0 = time.perf_counter()
    osc = oracle.OracleScene(scene)
    t_bvh = time.perf_counter() - t0
    n_ph = cfg["n_photons"]
    p1 = n_ph // 8
    t0 = time.perf_counter()
    m, msum, cnt, st = oracle.trace_photons(osc, n_ph, cfg["max_depth"], wl, cfg["photon_seed"], p0=0, p1=p1)
    t_ph = time.perf_counter() - t0
    ys, xs = np.meshgrid(np.arange(0, cam.h, 2), np.arange(0, cam.w, 2), indexing="ij")
    pix = (ys * cam.w + xs).ravel().astype(np.uint32)
    t0 = time.perf_counter()
    out = oracle.render(osc, cam, cfg["spp"], cfg["max_depth"], wl, cfg["render_seed"], caustic_map=m, pixels=pix)
    t_r = time.perf_counter() - t0
    rays = st["segments"] + out["segments"]
    secs = t_ph + t_r
    return {"value": round(rays / secs / 1e6, 4), "unit": "Mrays/s", "cores": 1, "kind": "oracle",
            "sample": f"1/4 of the pixels (every 2nd row and column, {len(pix)} px at {cfg['spp']} spp) and "
                      f"photons [0, {p1}) of {n_ph}; {rays} ray segments in {secs:.2f} s (oracle BVH build "
                      f"{t_bvh:.2f} s not counted); full step would take ~{rays_per_step / (rays / secs):.0f} s "
                      f"on one core vs {step_s * 1e3:.1f} ms on the GPU"}


def denoise_fps(ctx):
    """The second half of the metric: 1080p frames/s at relMSE <= 0.01
    against a 1024-spp reference, denoised vs plain rendering, on the
    held-out large scene (seed 200000, ~2M triangles).  Plain: photon pass
    + render, at the cheapest (spp, photons) whose render meets the bar
    (photons in {2^16, 2^18, 2^20, 2^22, 2^24}, for each the smallest
    power-of-two spp from 4).  Denoised: photon pass + render, the
    ground-truth buffers (a second context on a second stream, overlapping
    the photon pass) + the U-Net with the committed trained weights, at the
    cheapest input
    (spp in {1, 2, 4}, photons in {2^16, 2^18, 2^20}) whose denoised image
    meets the same bar; the 4-spp, 2^20-photon input is reported beside
    it."""
    import torch

    import paper_2107_11008_amd as sc
    import scenegen as sg
    from paper_2107_11008_amd import denoiser as D
    params, meta = D.load_weights()
    if params is None:
        return None
    net = sc.UNet(ctx, tuple(meta["widths"]), params)
    cfg = sg.config3(seed=200000)
    scene, wl, cam, md = cfg["scene"], cfg["wavelengths"], cfg["camera"], cfg["max_depth"]
    bvh = ctx.build_bvh(scene)
    ref = ctx.render(bvh, cam, 1024, md, wl, 901, caustic_map=ctx.trace_photons(bvh, cfg["n_photons"], md, wl,
                                                                               902)["map"], outputs=("rgb",))["rgb"]
    outs = {}
    # the denoiser's ground-truth inputs (one pixel-centre ray per pixel,
    # independent of the paths) come from a second context on a second
    # stream, overlapping the photon pass; the U-Net waits for both streams
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ctx_gt = sc.Context(0)

    def denoised(spp, photons):
        e0 = torch.cuda.Event()
        e0.record(main)
        side.wait_event(e0)            # the previous frame's U-Net has read the buffers
        g = ctx_gt.render(bvh, cam, 1, md, wl, 12, outputs=("albedo", "normal", "depthn", "trans"),
                          out=outs.get("g_d"))
        outs["g_d"] = g
        e1 = torch.cuda.Event()
        e1.record(side)
        m = ctx.trace_photons(bvh, photons, md, wl, 11, out=outs.get("m_d"))["map"]
        outs["m_d"] = m
        r = ctx.render(bvh, cam, spp, md, wl, 12, caustic_map=m, outputs=("rgb",), out=outs.get("r_d"))
        outs["r_d"] = r
        main.wait_event(e1)
        outs["den"] = net.denoise(dict(g, rgb=r["rgb"]), out=outs.get("den"))
        return outs["den"]

    def plain(spp, photons):
        m = ctx.trace_photons(bvh, photons, md, wl, 11, out=outs.get("m_p"))["map"]
        outs["m_p"] = m
        r = ctx.render(bvh, cam, spp, md, wl, 12, caustic_map=m, outputs=("rgb",), out=outs.get("r_p"))
        outs["r_p"] = r
        return r["rgb"]

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            img = fn()
        torch.cuda.synchronize()
        return img, (time.perf_counter() - t) / reps

    tried = []
    for photons in (1 << 16, 1 << 18, 1 << 20):
        for spp in (1, 2, 4):
            img_d, t_d = timed(lambda: denoised(spp, photons), 5)
            tried.append({"spp": spp, "photons": photons, "relmse": round(D.rel_mse(img_d, ref), 5),
                          "ms": round(t_d * 1e3, 2), "fps": round(1.0 / t_d, 2)})
    passing = [d for d in tried if d["relmse"] <= 0.01]
    best = min(passing, key=lambda d: d["ms"]) if passing else None
    fixed = [d for d in tried if d["spp"] == 4 and d["photons"] == 1 << 20][0]
    # plain: for each photon count the smallest power-of-two spp from 4 that
    # meets the bar, then the cheapest of those
    plain_tried = []
    for photons in (1 << 16, 1 << 18, 1 << 20, 1 << 22, cfg["n_photons"]):
        spp = 4
        while spp <= 1024:
            img_p, t = timed(lambda: plain(spp, photons), 2)
            e = D.rel_mse(img_p, ref)
            plain_tried.append({"spp": spp, "photons": photons, "relmse": round(e, 5), "ms": round(t * 1e3, 2),
                                "fps": round(1.0 / t, 2)})
            if e <= 0.01:
                break
            spp *= 2
    plain_pass = [d for d in plain_tried if d["relmse"] <= 0.01]
    pbest = min(plain_pass, key=lambda d: d["ms"]) if plain_pass else None
    res = {"scene": "large glass scene, seed 200000, 1920x1080, %d triangles" % scene.nt,
           "denoised": best, "denoised_4spp": fixed, "plain": pbest,
           "denoised_inputs_tried": [(d["spp"], d["photons"], d["relmse"], d["ms"]) for d in tried],
           "plain_inputs_tried": [(d["spp"], d["photons"], d["relmse"], d["ms"]) for d in plain_tried]}
    if pbest is not None and best is not None:
        res["fps_ratio"] = round(pbest["ms"] / best["ms"], 2)
        res["fps_ratio_4spp"] = round(pbest["ms"] / fixed["ms"], 2) if fixed["relmse"] <= 0.01 else None
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
    res["tuning"] = {k: best[k] for k in ("width", "block_size", "blocks_per_cu", "px_per_item")}
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
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-denoise", action="store_true")
    ap.add_argument("--staged-depth", type=int, default=None,
                    help="bounces run as one launch per stage before per-lane path finishing "
                         "(library default if omitted; 0 = all bounces staged)")
    ap.add_argument("--photon-staged-depth", type=int, default=None,
                    help="the same for photon paths (library default if omitted)")
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

    cfg = sg.config2()
    scene, wl, cam = cfg["scene"], cfg["wavelengths"], cfg["camera"]
    ctx = sc.Context(0)
    if args.staged_depth is not None:
        ctx.set_option(sc._sc.SC_OPT_STAGED_DEPTH, args.staged_depth)
    if args.photon_staged_depth is not None:
        ctx.set_option(sc._sc.SC_OPT_PHOTON_STAGED_DEPTH, args.photon_staged_depth)
    stream = torch.cuda.current_stream()

    if args.calib_copy_mib:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    outs = {}
    # the scene's arrays are resident in HBM before anything is timed; each
    # step rebuilds the BVH from them into the same handle's memory
    dscene = ctx.upload_scene(scene)

    def step():
        bvh = ctx.build_bvh(dscene, out=outs.get("bvh"))
        outs["bvh"] = bvh
        ph = ctx.trace_photons(bvh, cfg["n_photons"], cfg["max_depth"], wl, cfg["photon_seed"],
                               out=outs.get("map"))
        outs["map"] = ph["map"]
        r = ctx.render(bvh, cam, cfg["spp"], cfg["max_depth"], wl, cfg["render_seed"], caustic_map=ph["map"],
                       out=outs.get("img"))
        outs["img"] = r
        return bvh

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # visit counts of the traversal kernels (same kernels, counting variants), untimed
    ctx.reset_counters()
    ctx.set_option(sc._sc.SC_OPT_COUNT_VISITS, 1)
    bvh = step()
    cnt = ctx.counters()
    ctx.set_option(sc._sc.SC_OPT_COUNT_VISITS, 0)
    # visits are counted by the staged closest-hit kernel, over its own rays
    nodes_per_ray = cnt["node_visits"] / cnt["closest_rays_timed"]
    tris_per_ray = cnt["tri_tests"] / cnt["closest_rays_timed"]
    # and by the photon path finishing kernel, over its own segments
    fin_nodes_per_ray = cnt["finish_node_visits"] / max(cnt["finish_rays"], 1)
    fin_tris_per_ray = cnt["finish_tri_tests"] / max(cnt["finish_rays"], 1)
    rays_per_step = cnt["rays_closest"] + cnt["rays_shadow"]
    info = bvh.info()
    del bvh

    # timed region
    ctx.reset_counters()
    ctx.set_option(sc._sc.SC_OPT_PROFILE, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    c = ctx.counters()
    ctx.set_option(sc._sc.SC_OPT_PROFILE, 0)

    secs = t1 - t0
    rays = c["rays_closest"] + c["rays_shadow"]
    value = rays / secs / 1e6
    bytes_per_ray = 24 + 4 + 16 + nodes_per_ray * 256 + tris_per_ray * 48
    launches = c["closest_launches"]
    avg_ms = c["closest_ms"] / max(launches, 1)
    alg_bytes_per_launch = bytes_per_ray * c["closest_rays_timed"] / max(launches, 1)
    achieved = alg_bytes_per_launch / (avg_ms * 1e-3) / 1e9
    roof_closest = {"bound": "hbm", "kernel": "k_closest (staged closest-hit traversal)",
                    "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": _traffic_per_launch("k_closest<false>"),
                    "avg_launch_ms": round(avg_ms, 5), "launches": launches,
                    "alg_bytes_per_launch": round(alg_bytes_per_launch),
                    "bytes_per_ray": round(bytes_per_ray, 1), "nodes_per_ray": round(nodes_per_ray, 3),
                    "tris_per_ray": round(tris_per_ray, 3),
                    "kernel_Mrays_s": round(c["closest_rays_timed"] / (c["closest_ms"] * 1e-3) / 1e6, 1),
                    "ms_per_step": round(c["closest_ms"] / args.steps, 4)}
    # photon path finishing: per path its state (48 B) and queue entry (4 B)
    # are read once; per closest-hit segment the nodes and triangles fetched
    f_launches = c["finish_launches"]
    roof_finish = None
    if f_launches:
        f_ms = c["finish_ms"] / f_launches
        f_bytes = (c["finish_paths"] * 52 + c["finish_rays"] * (fin_nodes_per_ray * 256 + fin_tris_per_ray * 48)) \
            / f_launches
        f_ach = f_bytes / (f_ms * 1e-3) / 1e9
        roof_finish = {"bound": "hbm", "kernel": "k_finish_photons (per-lane photon path finishing)",
                       "achieved": round(f_ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(f_ach / HBM_PEAK_GBS, 4),
                       "traffic": _traffic_per_launch("k_finish_photons<false>"),
                       "avg_launch_ms": round(f_ms, 5), "launches": f_launches, "alg_bytes_per_launch": round(f_bytes),
                       "paths_per_launch": round(c["finish_paths"] / f_launches),
                       "rays_per_launch": round(c["finish_rays"] / f_launches),
                       "nodes_per_ray": round(fin_nodes_per_ray, 3), "tris_per_ray": round(fin_tris_per_ray, 3),
                       "kernel_Mrays_s": round(c["finish_rays"] / (c["finish_ms"] * 1e-3) / 1e6, 1),
                       "ms_per_step": round(c["finish_ms"] / args.steps, 4)}
    # the roofline object is the kernel with the most time per step; the
    # other traversal kernel is reported beside it
    if roof_finish and roof_finish["ms_per_step"] > roof_closest["ms_per_step"]:
        roofline, roofline_other = roof_finish, roof_closest
    else:
        roofline, roofline_other = roof_closest, roof_finish

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

    line = {
        "metric": METRIC,
        "value": round(value, 2),
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
        "config": {"workload": "medium glass scene: 512x512, 16 spp, wavelengths uniform 380-720 nm, max depth 12, "
                               "2^22 caustic photons into a 1024x1024x16 map, 8 procedural glass objects "
                               f"({scene.nt} triangles) on a textured plane, one area light; step = BVH build + "
                               "photon pass + ground truth + image",
                   "triangles": scene.nt, "width": cam.w, "height": cam.h, "spp": cfg["spp"],
                   "max_depth": cfg["max_depth"], "photons": cfg["n_photons"]},
        "rays_per_step": rays_per_step,
        "breakdown_ms": {"bvh_build": round((tb1 - tb0) * 1e3, 3), "photons": round((tb2 - tb1) * 1e3, 3),
                         "render": round((tb3 - tb2) * 1e3, 3)},
        "bvh": {"nodes": info["n_nodes"], "depth": info["depth"], "node_bytes": info["node_bytes"],
                "tri_bytes": info["tri_bytes"]},
        "roofline": roofline,
        "roofline_other_traversal_kernel": roofline_other,
    }
    if not args.no_glass_variants:
        line["glass_variants"] = glass_variants(ctx)
    if not args.no_pmap:
        line["general_photon_map"] = general_photon_map(ctx)
    if not args.no_unet:
        line["unet_1080p"] = unet_1080p(ctx)
    if not args.no_train:
        line["unet_train_step"] = unet_train_step(ctx)
    if not args.no_gt:
        line["ground_truth_1080p"] = ground_truth_1080p(ctx)
    if not args.no_denoise:
        line["denoise_1080p"] = denoise_fps(ctx)
    if not args.no_batch:
        line["batch_64"] = batch_compare(ctx)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, rays_per_step, secs / args.steps)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
