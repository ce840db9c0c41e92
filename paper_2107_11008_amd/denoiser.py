"""Training and evaluation of the learned denoiser on the renderer's output.

Training pairs come from the renderer itself: seeded medium-type scenes
(glass lathes and superquadrics on a textured plane, one area light)
rendered at low sample count with the ground-truth buffers (the network
input) and at 1024 samples per pixel with independent seeds (the target).
The network is trained on the GPU by the library's own forward, backward and
Adam kernels (sc_unet_train_step).  Evaluation renders held-out large-type
scenes at 1920x1080 and reports relMSE = mean (x - ref)^2 / (ref^2 + 0.01)
against a 1024-spp reference, for the raw low-spp render, the denoised
render, and plain renders at increasing sample counts; the reference's own
noise floor is estimated from a second independent 1024-spp reference.

Usage (on a GPU):
    python -m paper_2107_11008_amd.denoiser --out weights_dir
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import _sc as sc

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
WEIGHTS_NAME = "unet_denoiser"
WIDTHS = (32, 48, 64, 96, 128)


def rel_mse(x: torch.Tensor, ref: torch.Tensor, eps: float = 0.01) -> float:
    x = x.double()
    ref = ref.double()
    return float(((x - ref) ** 2 / (ref * ref + eps)).mean())


def features(ctx, r: dict) -> torch.Tensor:
    """[H,W,9] float: log1p(rgb), albedo, normal, depth/10, transparent,
    built by the library (sc_unet_features), the function sc_denoise uses."""
    return ctx.unet_features(r)


def render_pair(ctx, cfg, spp_in: int, spp_ref: int, ph_in: int, ph_ref: int, seed: int, cam=None, bvh=None):
    scene, wl = cfg["scene"], cfg["wavelengths"]
    cam = cfg["camera"] if cam is None else cam
    bvh = ctx.build_bvh(scene) if bvh is None else bvh
    m_in = ctx.trace_photons(bvh, ph_in, cfg["max_depth"], wl, seed + 11)["map"]
    r_in = ctx.render(bvh, cam, spp_in, cfg["max_depth"], wl, seed + 12, caustic_map=m_in,
                      outputs=("rgb", "albedo", "normal", "depthn", "trans"))
    m_ref = ctx.trace_photons(bvh, ph_ref, cfg["max_depth"], wl, seed + 21)["map"]
    r_ref = ctx.render(bvh, cam, spp_ref, cfg["max_depth"], wl, seed + 22, caustic_map=m_ref, outputs=("rgb",))
    return features(ctx, r_in), r_ref["rgb"].contiguous()


def crop_camera(cam, x0: int, y0: int, w: int, h: int):
    """Camera whose w x h film is the window [x0, x0+w) x [y0, y0+h) of cam's
    film: same pixel footprint, so crops of a full-resolution frame."""
    import scenegen as sg
    W, H = cam.w, cam.h
    f = cam.fwd.astype(np.float64) + ((2.0 * x0 + w) / W - 1.0) * cam.right.astype(np.float64) \
        + (1.0 - (2.0 * y0 + h) / H) * cam.up.astype(np.float64)
    return sg.Camera(cam.eye.copy(), f.astype(np.float32), (cam.right.astype(np.float64) * (w / W)).astype(np.float32),
                     (cam.up.astype(np.float64) * (h / H)).astype(np.float32), int(w), int(h))


def layer_shapes(widths=WIDTHS, in_ch: int = 9, out_ch: int = 3):
    """(cout, ksize, cin) of every convolution in the library's parameter
    order: encoder levels shallow to deep (two 3x3 each), decoder levels
    deep to shallow (3x3 over [upsampled | skip], then 3x3), 1x1 output."""
    L = []
    cin = in_ch
    for w in widths:
        L += [(w, 3, cin), (w, 3, w)]
        cin = w
    for i in range(len(widths) - 2, -1, -1):
        L += [(widths[i], 3, cin + widths[i]), (widths[i], 3, widths[i])]
        cin = widths[i]
    L.append((out_ch, 1, cin))
    return L


def he_init(net, seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for co, k, ci in layer_shapes(net.widths):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / (k * k * ci)), size=co * k * k * ci))
        parts.append(np.zeros(co))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == net.n_params
    return p


def save_weights(params: np.ndarray, meta: dict, d: str = WEIGHTS_DIR, name: str = WEIGHTS_NAME):
    os.makedirs(d, exist_ok=True)
    np.ascontiguousarray(params, dtype="<f4").tofile(os.path.join(d, name + ".bin"))
    with open(os.path.join(d, name + ".json"), "w") as f:
        json.dump(meta, f, indent=1)


def load_weights(d: str = WEIGHTS_DIR, name: str = WEIGHTS_NAME):
    """(params float32, meta) or (None, None) if no trained weights exist."""
    pb, pj = os.path.join(d, name + ".bin"), os.path.join(d, name + ".json")
    if not (os.path.exists(pb) and os.path.exists(pj)):
        return None, None
    with open(pj) as f:
        meta = json.load(f)
    return np.fromfile(pb, dtype="<f4"), meta


def train(ctx, net, pairs, steps: int, batch: int, crop: int, lr: float, seed: int = 0, log=print):
    rng = np.random.default_rng(seed)
    feats = torch.stack([p[0] for p in pairs])
    tgts = torch.stack([p[1] for p in pairs])
    n, H, W, _ = feats.shape
    losses = []
    t0 = time.time()
    for it in range(steps):
        idx = rng.integers(0, n, size=batch)
        ys = rng.integers(0, H - crop + 1, size=batch)
        xs = rng.integers(0, W - crop + 1, size=batch)
        fb = torch.stack([feats[i, y:y + crop, x:x + crop] for i, y, x in zip(idx, ys, xs)]).contiguous()
        tb = torch.stack([tgts[i, y:y + crop, x:x + crop] for i, y, x in zip(idx, ys, xs)]).contiguous()
        cur_lr = lr if it < 0.7 * steps else lr * 0.3
        want = (it % 50 == 0) or it == steps - 1
        loss = net.train_step(fb, tb, cur_lr, want_loss=want)
        if want:
            losses.append((it, loss))
            log(f"train step {it} loss {loss:.5f} ({time.time() - t0:.1f} s)")
    return losses


def c5_pairs(ctx, n_scenes: int, size: int, spp_in: int, spp_ref: int, seed0: int = 100000, log=print):
    """The training set of the denoiser's data protocol: n_scenes medium-type
    scenes (seeds seed0..seed0+n-1, full triangle count) at size x size;
    inputs are spp_in-sample renders with their ground-truth buffers and a
    caustic map of 2^16, 2^18 or 2^20 photons (seeded per scene), targets
    spp_ref-sample renders with 2^22 photons and independent seeds.  Kept
    in device memory: features [n][size][size][9] and targets
    [n][size][size][3] float (12.6 MB per scene at 512^2).  Scenes are
    generated on a host thread while the GPU renders the previous one."""
    import queue
    import threading

    import scenegen as sg
    feats = torch.empty((n_scenes, size, size, 9), dtype=torch.float32, device=ctx.device)
    tgts = torch.empty((n_scenes, size, size, 3), dtype=torch.float32, device=ctx.device)
    q = queue.Queue(maxsize=4)

    def produce():
        for j in range(n_scenes):
            q.put(sg.config2(seed=seed0 + j, w=size, h=size))

    th = threading.Thread(target=produce, daemon=True)
    th.start()
    rng = np.random.default_rng(seed0)
    t0 = time.time()
    for j in range(n_scenes):
        cfg = q.get()
        ph_in = int(rng.choice([1 << 16, 1 << 18, 1 << 20]))
        f, t = render_pair(ctx, cfg, spp_in, spp_ref, ph_in, 1 << 22, 7000 + 100 * j)
        feats[j].copy_(f)
        tgts[j].copy_(t)
        if j % 25 == 0 or j == n_scenes - 1:
            torch.cuda.synchronize()
            log(f"c5 pair {j + 1}/{n_scenes} ({time.time() - t0:.1f} s)")
    th.join()
    return feats, tgts


def train_tensors(ctx, net, feats, tgts, steps: int, batch: int, crop: int, lr: float, seed: int = 0, log=print):
    """train() over device tensors of whole frames (random crops)."""
    rng = np.random.default_rng(seed)
    n, H, W, _ = feats.shape
    losses = []
    t0 = time.time()
    for it in range(steps):
        idx = rng.integers(0, n, size=batch)
        ys = rng.integers(0, H - crop + 1, size=batch)
        xs = rng.integers(0, W - crop + 1, size=batch)
        fb = torch.stack([feats[i, y:y + crop, x:x + crop] for i, y, x in zip(idx, ys, xs)]).contiguous()
        tb = torch.stack([tgts[i, y:y + crop, x:x + crop] for i, y, x in zip(idx, ys, xs)]).contiguous()
        cur_lr = lr if it < 0.7 * steps else lr * 0.3
        want = (it % 500 == 0) or it == steps - 1
        loss = net.train_step(fb, tb, cur_lr, want_loss=want)
        if want:
            losses.append((it, loss))
            log(f"train step {it} loss {loss:.5f} ({time.time() - t0:.1f} s)")
    return losses


def main_c5(args, log):
    """Training on the data protocol's set (--c5): 2000 medium-type scenes at
    512^2, 4 spp in, 1024 spp targets."""
    ctx = sc.Context(0)
    t0 = time.time()
    feats, tgts = c5_pairs(ctx, args.scenes, args.size, args.spp_in, args.spp_ref, log=log)
    log(f"c5 set ready: {args.scenes} scenes in {time.time() - t0:.1f} s")
    net = sc.UNet(ctx, WIDTHS)
    net.set_params(he_init(net, 12345))
    losses = train_tensors(ctx, net, feats, tgts, args.steps, args.batch, args.crop, args.lr, log=log)
    params = net.get_params()
    meta = {"widths": list(WIDTHS), "n_params": int(net.n_params), "protocol": "c5",
            "train_scenes": args.scenes, "train_size": args.size, "spp_in": args.spp_in, "spp_ref": args.spp_ref,
            "photons_in": [1 << 16, 1 << 18, 1 << 20], "photons_ref": 1 << 22, "steps": args.steps,
            "batch": args.batch, "crop": args.crop, "lr": args.lr,
            "medium_scene_seeds": [100000, 100000 + args.scenes - 1], "large_scene_seeds": None,
            "data_s": round(time.time() - t0, 1), "loss_curve": losses}
    save_weights(params, meta, args.out)
    log(f"saved to {args.out} ({time.time() - t0:.1f} s)")


def main(argv=None):
    import scenegen as sg

    ap = argparse.ArgumentParser()
    ap.add_argument("--scenes", type=int, default=64)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--steps", type=int, default=8000)
    ap.add_argument("--batch", type=int, default=12)
    ap.add_argument("--crop", type=int, default=128)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--spp-in", type=int, default=4)
    ap.add_argument("--spp-ref", type=int, default=1024)
    ap.add_argument("--eval-scenes", type=int, default=2)
    ap.add_argument("--large-scenes", type=int, default=32)
    ap.add_argument("--crops", type=int, default=3)
    ap.add_argument("--photons-in", type=int, default=1 << 22)
    ap.add_argument("--out", default=WEIGHTS_DIR)
    ap.add_argument("--report", default=None)
    ap.add_argument("--c5", action="store_true", help="the data protocol's training set (see main_c5)")
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    if args.c5:
        return main_c5(args, log)

    ctx = sc.Context(0)
    t0 = time.time()
    pairs = []
    rng = np.random.default_rng(77)
    # medium-type scenes, whole frames at args.size^2
    for j in range(args.scenes):
        cfg = sg.config2(seed=100000 + j, tri_scale=0.5, w=args.size, h=args.size)
        pairs.append(render_pair(ctx, cfg, args.spp_in, args.spp_ref, 1 << 22, 1 << 22, 7000 + 100 * j))
        if j % 10 == 0:
            log(f"pair {j}/{args.scenes} ({time.time() - t0:.1f} s)")
    # large-type scenes: crops of the 1920x1080 frame at full pixel footprint
    for j in range(args.large_scenes):
        cfg = sg.config3(seed=150000 + j)
        bvh = ctx.build_bvh(cfg["scene"])
        for c in range(args.crops):
            x0 = int(rng.integers(0, 1920 - args.size + 1))
            y0 = int(rng.integers(0, 1080 - args.size + 1))
            cam = crop_camera(cfg["camera"], x0, y0, args.size, args.size)
            pairs.append(render_pair(ctx, cfg, args.spp_in, args.spp_ref, args.photons_in, cfg["n_photons"],
                                     9000 + 100 * j + 10 * c, cam=cam, bvh=bvh))
        del bvh
        log(f"large scene {j}/{args.large_scenes} ({time.time() - t0:.1f} s)")
    net = sc.UNet(ctx, WIDTHS)
    net.set_params(he_init(net, 12345))
    losses = train(ctx, net, pairs, args.steps, args.batch, args.crop, args.lr, log=log)
    params = net.get_params()
    meta = {"widths": list(WIDTHS), "n_params": int(net.n_params), "train_scenes": args.scenes,
            "train_size": args.size, "spp_in": args.spp_in, "spp_ref": args.spp_ref, "steps": args.steps,
            "batch": args.batch, "crop": args.crop, "lr": args.lr, "photons_in": args.photons_in,
            "medium_scene_seeds": [100000, 100000 + args.scenes - 1],
            "large_scene_seeds": [150000, 150000 + args.large_scenes - 1], "crops_per_large_scene": args.crops,
            "loss_curve": losses}
    save_weights(params, meta, args.out)
    del pairs
    torch.cuda.empty_cache()
    report = {"train": meta, "eval": evaluate(ctx, net, args.eval_scenes, ph_in=args.photons_in, log=log)}
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    log(json.dumps(report["eval"]))


def evaluate(ctx, net, n_scenes: int = 2, spp_in: int = 4, ph_in: int = 1 << 22, log=print, max_plain: int = 1024):
    """Held-out large scenes at 1920x1080: relMSE of raw, denoised and plain
    renders against a 1024-spp reference; frame times of each."""
    import scenegen as sg
    out = []
    for j in range(n_scenes):
        cfg = sg.config3(seed=200000 + j)
        scene, wl, cam = cfg["scene"], cfg["wavelengths"], cfg["camera"]
        bvh = ctx.build_bvh(scene)
        md = cfg["max_depth"]
        ph_ref = cfg["n_photons"]
        ref = ctx.render(bvh, cam, 1024, md, wl, 901, caustic_map=ctx.trace_photons(bvh, ph_ref, md, wl, 902)["map"],
                         outputs=("rgb",))["rgb"]
        ref2 = ctx.render(bvh, cam, 1024, md, wl, 903, caustic_map=ctx.trace_photons(bvh, ph_ref, md, wl, 904)["map"],
                          outputs=("rgb",))["rgb"]
        floor = rel_mse(ref2, ref) / 2
        log(f"eval scene {j}: reference noise floor {floor:.5f}")

        def timed(fn, reps=3, warm=True):
            if warm:
                fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                r = fn()
            torch.cuda.synchronize()
            return r, (time.perf_counter() - t) / reps

        def denoised():
            m = ctx.trace_photons(bvh, ph_in, md, wl, 11)["map"]
            r = ctx.render(bvh, cam, spp_in, md, wl, 12, caustic_map=m,
                           outputs=("rgb", "albedo", "normal", "depthn", "trans"))
            return r, net.denoise(r)

        (raw, den), t_den = timed(denoised)
        rm_raw, rm_den = rel_mse(raw["rgb"], ref), rel_mse(den, ref)
        plain = []
        n_star = None
        spp = 4
        while spp <= max_plain:
            def plain_fn(spp=spp):
                m = ctx.trace_photons(bvh, ph_ref, md, wl, 11)["map"]
                return ctx.render(bvh, cam, spp, md, wl, 12, caustic_map=m, outputs=("rgb",))["rgb"]
            img, t_plain = timed(plain_fn, reps=1, warm=False)
            rm = rel_mse(img, ref)
            plain.append({"spp": spp, "relmse": rm, "ms": t_plain * 1e3})
            log(f"  plain {spp} spp relMSE {rm:.5f} {t_plain * 1e3:.1f} ms")
            if rm <= 0.01 and n_star is None:
                n_star = spp
                break
            spp *= 2
        res = {"scene_seed": 200000 + j, "triangles": scene.nt, "reference_floor": floor,
               "raw_spp": spp_in, "raw_relmse": rm_raw, "denoised_relmse": rm_den, "denoised_ms": t_den * 1e3,
               "denoised_photons": ph_in, "plain": plain, "plain_n_star": n_star}
        if n_star is not None:
            t_plain = plain[-1]["ms"]
            res["fps_plain"] = 1e3 / t_plain
            res["fps_denoised"] = 1e3 / (t_den * 1e3)
            res["speedup"] = t_plain / (t_den * 1e3)
        log(f"eval scene {j}: raw {rm_raw:.5f} denoised {rm_den:.5f} ({t_den * 1e3:.1f} ms) N* {n_star}")
        out.append(res)
    return out


if __name__ == "__main__":
    sys.exit(main())
