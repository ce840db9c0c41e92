"""Autotuner of the batched persistent launch: a thin wrapper over
sc_autotune (the library's C autotuner, which times candidate settings of
the persistent grid, pixel tile, photon queue grain and BVH width on
reduced copies of the batch).  No choice changes any output: the batch
result is bit-identical for every setting.  Results are cached in a JSON
file keyed by the batch's shape.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import torch

from . import _sc as sc

CACHE = os.path.join(os.path.expanduser("~"), ".cache", "sc_autotune.json")
KEYS = ("width", "block_size", "blocks_per_cu", "px_per_item", "ph_per_item", "use_graph")


def signature(cfgs) -> str:
    h = hashlib.sha256()
    for c in cfgs:
        h.update(f"{c['scene'].nt}:{c['camera'].w}x{c['camera'].h}:{c['spp']}:{c['max_depth']}:"
                 f"{c.get('n_photons', 0)};".encode())
    return h.hexdigest()[:20]


def _items(cfgs, bvhs, spp=None, photon_div=1):
    return [dict(bvh=b, cam=c["camera"], spp=spp or c["spp"], max_depth=c["max_depth"], wl=c["wavelengths"],
                 seed=c["render_seed"], photon_seed=c["photon_seed"],
                 n_photons=max(64, c.get("n_photons", 0) // photon_div) if c.get("n_photons", 0) else 0)
            for c, b in zip(cfgs, bvhs)]


def autotune(ctx, cfgs, cache_path: str = CACHE, log=None) -> dict:
    """Best {width, block_size, blocks_per_cu, px_per_item, ph_per_item,
    use_graph} for the batch described by cfgs (scenegen configs), from
    sc_autotune on the batch built with 8-wide trees."""
    sig = signature(cfgs)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if sig in cache and all(k in cache[sig] for k in KEYS):
        return dict(cache[sig], cached=True)
    bvhs = [ctx.build_bvh(c["scene"], width=8) for c in cfgs]
    t0 = time.perf_counter()
    t = sc.autotune_batch(ctx, _items(cfgs, bvhs))
    secs = time.perf_counter() - t0
    for b in bvhs:
        b.close()
    best = dict(width=t["bvh_width"], block_size=t["block_size"], blocks_per_cu=t["blocks_per_cu"],
                px_per_item=t["px_per_item"], ph_per_item=t["ph_per_item"], use_graph=t["use_graph"],
                tuning_s=round(secs, 2))
    if log:
        log(f"autotune: {best}")
    if cache_path:
        cache[sig] = best
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return dict(best, cached=False)


def compare(ctx, cfgs, tuned: dict, reps: int = 2, log=None) -> dict:
    """Frame time of the whole batch: the tuned persistent graph launch vs
    the same scenes rendered one after another (photon pass + wavefront
    render per scene).  BVH builds are done before either is timed."""
    bvhs = [ctx.build_bvh(c["scene"], width=tuned["width"]) for c in cfgs]
    items = _items(cfgs, bvhs)
    b = sc.Batch(ctx, items, {k: tuned[k] for k in ("block_size", "blocks_per_cu", "px_per_item", "ph_per_item",
                                                     "use_graph")})
    b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.run()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    maps = [None] * len(cfgs)
    imgs = [None] * len(cfgs)

    def sequential():
        for i, (c, bv) in enumerate(zip(cfgs, bvhs)):
            m = None
            if c.get("n_photons", 0):
                maps[i] = ctx.trace_photons(bv, c["n_photons"], c["max_depth"], c["wavelengths"], c["photon_seed"],
                                            out=maps[i])["map"]
                m = maps[i]
            imgs[i] = ctx.render(bv, c["camera"], c["spp"], c["max_depth"], c["wavelengths"], c["render_seed"],
                                 caustic_map=m, out=imgs[i])

    sequential()
    torch.cuda.synchronize()
    ctx.reset_counters()
    t0 = time.perf_counter()
    for _ in range(reps):
        sequential()
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / reps
    cnt = ctx.counters()
    rays = (cnt["rays_closest"] + cnt["rays_shadow"]) / reps
    # the two must agree bit for bit
    same = all(torch.equal(o["rgb"], im["rgb"]) and torch.equal(o["tri"], im["tri"])
               for o, im in zip(b.outputs(), imgs))
    res = dict(scenes=len(cfgs), triangles=int(sum(c["scene"].nt for c in cfgs)),
               pixels=int(sum(c["camera"].w * c["camera"].h for c in cfgs)), batched_ms=round(t_batch * 1e3, 2),
               sequential_ms=round(t_seq * 1e3, 2), speedup=round(t_seq / t_batch, 3),
               batched_Mrays_s=round(rays / t_batch / 1e6, 1), sequential_Mrays_s=round(rays / t_seq / 1e6, 1),
               identical_outputs=bool(same))
    if log:
        log(json.dumps(res))
    return res
