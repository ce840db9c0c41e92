"""The batched persistent launch against one-scene-at-a-time rendering:
every image, ground-truth buffer and caustic map is bit-identical (the
same per-path code runs; caustic sums are exact fixed point), for every
tuning the autotuner may pick, and across replays of the captured graph."""
import numpy as np
import pytest
import torch

import scenegen as sg

pytestmark = pytest.mark.gpu

KEYS = ("rgb", "obj", "trans", "tri", "depth", "depthn", "normal", "normal_cam", "albedo")


def _bits(t):
    a = t.cpu().numpy()
    return a.view(np.uint32) if a.dtype in (np.float32, np.int32) else a


@pytest.fixture(scope="module")
def setup():
    import paper_2107_11008_amd as sc
    ctx = sc.Context(0)
    cfgs = [sg.config1(), sg.config2(tri_scale=0.05, w=96, h=64), sg.config4_item(3), sg.config4_item(7)]
    # keep the large batch scenes small for the test
    for c in cfgs[2:]:
        c["camera"] = sg.look_at((0.0, -1.8, 1.5), (0.0, 0.0, 0.05), (0, 0, 1), 40.0, 80, 48)
        c["spp"] = 2
    items, refs = [], []
    for i, c in enumerate(cfgs):
        bvh = ctx.build_bvh(c["scene"])
        n_ph = min(c["n_photons"], 1 << 15)
        it = dict(bvh=bvh, cam=c["camera"], spp=c["spp"], max_depth=c["max_depth"], wl=c["wavelengths"],
                  seed=c["render_seed"], photon_seed=c["photon_seed"], n_photons=n_ph)
        items.append(it)
        m = ctx.trace_photons(bvh, n_ph, c["max_depth"], c["wavelengths"], c["photon_seed"])["map"]
        r = ctx.render(bvh, c["camera"], c["spp"], c["max_depth"], c["wavelengths"], c["render_seed"], caustic_map=m)
        r["caustic_map"] = m
        refs.append(r)
    return ctx, items, refs


def _check(batch, refs):
    for outs, ref in zip(batch.outputs(), refs):
        for k in KEYS + ("caustic_map",):
            assert np.array_equal(_bits(outs[k]), _bits(ref[k])), k


@pytest.mark.parametrize("tune", [None, dict(block_size=64, blocks_per_cu=4, px_per_item=64, use_graph=0),
                                  dict(block_size=256, blocks_per_cu=2, px_per_item=256, use_graph=1),
                                  dict(block_size=128, blocks_per_cu=16, px_per_item=128, use_graph=1),
                                  dict(block_size=128, blocks_per_cu=8, px_per_item=64, ph_per_item=4096,
                                       use_graph=1),
                                  dict(block_size=256, blocks_per_cu=4, px_per_item=512, ph_per_item=64,
                                       use_graph=0)])
def test_batch_equals_sequential(setup, tune):
    import paper_2107_11008_amd as sc
    ctx, items, refs = setup
    b = sc.Batch(ctx, items, tune)
    b.run()
    torch.cuda.synchronize()
    _check(b, refs)


def test_graph_replays(setup):
    """Replays of the captured graph, with other work and synchronisation in
    between, reproduce the result every time."""
    import paper_2107_11008_amd as sc
    ctx, items, refs = setup
    b = sc.Batch(ctx, items, dict(block_size=128, blocks_per_cu=8, px_per_item=64, use_graph=1))
    for rep in range(3):
        b.run()
        torch.cuda.synchronize()
        _check(b, refs)
        x = torch.randn(1000, device="cuda").sum()   # unrelated eager work
        torch.cuda.synchronize()
        for outs in b.outputs():
            for k in KEYS:
                outs[k].zero_()
        torch.cuda.synchronize()


def test_bvh_width_does_not_change_batch(setup):
    import paper_2107_11008_amd as sc
    ctx, items, refs = setup
    items4 = [dict(it, bvh=ctx.build_bvh(it["bvh"].scene, width=4, leaf_max=2)) for it in items]
    b = sc.Batch(ctx, items4, None)
    b.run()
    torch.cuda.synchronize()
    _check(b, refs)


def test_autotune_picks_a_valid_setting(setup):
    """sc_autotune returns a setting inside its candidate sets; the batch
    run with it (and its BVH width) equals the one-scene outputs."""
    import paper_2107_11008_amd as sc
    ctx, items, refs = setup
    t = sc.autotune_batch(ctx, items)
    assert t["block_size"] in (64, 128, 256) and t["blocks_per_cu"] in (2, 4, 8)
    assert t["px_per_item"] in (64, 128, 256, 512) and t["ph_per_item"] in (64, 256, 1024, 4096)
    assert t["bvh_width"] in (4, 8) and t["use_graph"] == 1
    its = items
    if t["bvh_width"] != 8:
        its = [dict(it, bvh=ctx.build_bvh(it["bvh"].scene, width=t["bvh_width"])) for it in items]
    b = sc.Batch(ctx, its, t)
    b.run()
    torch.cuda.synchronize()
    _check(b, refs)
    bad = [dict(items[0], spp=0)]
    with pytest.raises(sc.ScError):
        sc.autotune_batch(ctx, bad)


def test_batch_rejects_bad_tuning(setup):
    import paper_2107_11008_amd as sc
    ctx, items, _ = setup
    with pytest.raises(sc.ScError):
        sc.Batch(ctx, items, dict(block_size=96, blocks_per_cu=4, px_per_item=64))
    with pytest.raises(sc.ScError):
        sc.Batch(ctx, items, dict(block_size=64, blocks_per_cu=4, px_per_item=100))
    with pytest.raises(sc.ScError):
        sc.Batch(ctx, items, dict(block_size=64, blocks_per_cu=4, px_per_item=64, ph_per_item=96))


def test_batch_with_richer_glass_and_rgb_texture():
    """Absorbing, rough, nested and overlapping glass and an RGB-textured
    floor in the batched form: still the single-scene outputs, bit for bit
    (the per-path functions carry the media set and the weights)."""
    import paper_2107_11008_amd as sc
    ctx = sc.Context(0)
    cfgs = [sg.tinted_nested(w=40, h=32), sg.config3(tri_scale=0.01, w=48, h=32, floor="rgb"),
            sg.config2(tri_scale=0.03, w=40, h=32, glass_style="rich")]
    items, refs = [], []
    for c in cfgs:
        bvh = ctx.build_bvh(c["scene"])
        n_ph, spp = 1 << 14, 2
        items.append(dict(bvh=bvh, cam=c["camera"], spp=spp, max_depth=c["max_depth"], wl=c["wavelengths"],
                          seed=c["render_seed"], photon_seed=c["photon_seed"], n_photons=n_ph))
        m = ctx.trace_photons(bvh, n_ph, c["max_depth"], c["wavelengths"], c["photon_seed"])["map"]
        r = ctx.render(bvh, c["camera"], spp, c["max_depth"], c["wavelengths"], c["render_seed"], caustic_map=m)
        r["caustic_map"] = m
        refs.append(r)
    b = sc.Batch(ctx, items, dict(block_size=128, blocks_per_cu=4, px_per_item=64, use_graph=1))
    b.run()
    torch.cuda.synchronize()
    _check(b, refs)
