"""The hybrid schedule: the first bounces as one launch per stage, the
remaining paths finished by one lane each.  Any switch depth must give the
same images, caustic maps, photon counts and photon outcome statistics, bit
for bit (the per-path functions are the same; only the schedule changes)."""
import numpy as np
import pytest
import torch

import scenegen as sg

pytestmark = pytest.mark.gpu

# (camera, photon) switch depths, the number of staged bounces (0: none, every
# path finished per lane; max depth or more: all staged); the first, every
# bounce staged, is the reference
DEPTHS = ((99, 99), (0, 0), (1, 1), (2, 5), (3, 2), (5, 1), (1, 3), (0, 2), (2, 0))


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_11008_amd as sc
    return sc.Context(0)


def _run(ctx, cfg, staged, spp):
    import paper_2107_11008_amd as sc
    ctx.set_option(sc._sc.SC_OPT_STAGED_DEPTH, staged[0])
    ctx.set_option(sc._sc.SC_OPT_PHOTON_STAGED_DEPTH, staged[1])
    try:
        bvh = ctx.build_bvh(cfg["scene"])
        md, wl = cfg["max_depth"], cfg["wavelengths"]
        ph = ctx.trace_photons(bvh, cfg["n_photons"], md, wl, cfg["photon_seed"], counts=True, stats=True)
        img = ctx.render(bvh, cfg["camera"], spp, md, wl, cfg["render_seed"], caustic_map=ph["map"],
                         outputs=("rgb", "obj", "depth"))
        torch.cuda.synchronize()
        return ({k: v.cpu().numpy().copy() for k, v in img.items()}, ph["map"].cpu().numpy().copy(),
                ph["count"].cpu().numpy().copy(), ph["stats"])
    finally:
        ctx.set_option(sc._sc.SC_OPT_STAGED_DEPTH, 2)      # the library's defaults
        ctx.set_option(sc._sc.SC_OPT_PHOTON_STAGED_DEPTH, 0)


@pytest.mark.parametrize("which", ["c1", "c2s", "glass"])
def test_switch_depth_does_not_change_outputs(ctx, which):
    if which == "c1":
        cfg, spp = sg.config1(), 2
    elif which == "glass":
        cfg, spp = sg.tinted_nested(), 3
    else:
        cfg, spp = sg.config2(tri_scale=0.05, w=48, h=40), 3
        cfg["n_photons"] = 1 << 17
    base = _run(ctx, cfg, DEPTHS[0], spp)
    assert np.isfinite(base[0]["rgb"]).all() and base[0]["rgb"].max() > 0
    for staged in DEPTHS[1:]:
        other = _run(ctx, cfg, staged, spp)
        for k in base[0]:
            assert base[0][k].tobytes() == other[0][k].tobytes(), (staged, k)
        assert base[1].tobytes() == other[1].tobytes(), staged
        assert np.array_equal(base[2], other[2]), staged
        for k, v in base[3].items():
            if k == "segments":
                assert v == other[3][k]
            else:
                assert v[1] == other[3][k][1], (staged, k)          # photon counts per outcome
                assert v[0] == pytest.approx(other[3][k][0], rel=1e-12)   # flux sums (float atomics)


def test_bad_staged_depth_rejected(ctx):
    import paper_2107_11008_amd as sc
    for opt in (sc._sc.SC_OPT_STAGED_DEPTH, sc._sc.SC_OPT_PHOTON_STAGED_DEPTH):
        with pytest.raises(sc.ScError):
            ctx.set_option(opt, -1)


@pytest.mark.parametrize("psd", [1, 0])
def test_finishing_counters(ctx, psd):
    """The counters behind the photon finishing kernel's roofline: with
    profiling and visit counting on, one timed launch per photon pass; it
    takes over the photons still alive after the staged bounce (every
    photon when no bounce is staged) and traces at least one segment each;
    every photon segment is counted once, by the staged kernel or by the
    finishing kernel (equal to the pass's segment statistic); counting does
    not change the map."""
    import paper_2107_11008_amd as sc
    c = sg.config2(tri_scale=0.05, w=32, h=24)
    md, wl = c["max_depth"], c["wavelengths"]
    n = 1 << 16
    bvh = ctx.build_bvh(c["scene"])
    plain = ctx.trace_photons(bvh, n, md, wl, c["photon_seed"])["map"].cpu().numpy()
    ctx.reset_counters()
    ctx.set_option(sc._sc.SC_OPT_PROFILE, 1)
    ctx.set_option(sc._sc.SC_OPT_COUNT_VISITS, 1)
    ctx.set_option(sc._sc.SC_OPT_PHOTON_STAGED_DEPTH, psd)
    try:
        r = ctx.trace_photons(bvh, n, md, wl, c["photon_seed"], stats=True)
        k = ctx.counters()
    finally:
        ctx.set_option(sc._sc.SC_OPT_PROFILE, 0)
        ctx.set_option(sc._sc.SC_OPT_COUNT_VISITS, 0)
        ctx.set_option(sc._sc.SC_OPT_PHOTON_STAGED_DEPTH, 0)
    assert r["map"].cpu().numpy().tobytes() == plain.tobytes()
    assert k["finish_launches"] == 1 and k["finish_ms"] > 0.0
    if psd:
        assert 0 < k["finish_paths"] < n
    else:
        assert k["finish_paths"] == n and k["closest_rays_timed"] == 0
    assert k["finish_rays"] >= k["finish_paths"]
    assert k["closest_rays_timed"] + k["finish_rays"] == k["rays_closest"] == r["stats"]["segments"]
    assert k["finish_node_visits"] >= k["finish_rays"] and k["finish_tri_tests"] > 0
    ctx.reset_counters()
    k = ctx.counters()
    assert k["finish_launches"] == 0 and k["finish_rays"] == 0 and k["finish_ms"] == 0.0


def test_trace_blocks_do_not_change_outputs(ctx):
    """Fewer blocks per CU in the persistent traversal grids (room for
    another stream's work) give the same images, maps and photon counts bit
    for bit."""
    import paper_2107_11008_amd as sc
    cfg = sg.config2(tri_scale=0.05, w=64, h=64)
    base = _run(ctx, cfg, (2, 0), 4)
    try:
        for tb in (3, 5, 16):
            ctx.set_option(sc._sc.SC_OPT_TRACE_BLOCKS, tb)
            other = _run(ctx, cfg, (2, 0), 4)
            for k in base[0]:
                assert base[0][k].tobytes() == other[0][k].tobytes(), (tb, k)
            assert base[1].tobytes() == other[1].tobytes(), tb
            assert np.array_equal(base[2], other[2]), tb
    finally:
        ctx.set_option(sc._sc.SC_OPT_TRACE_BLOCKS, 8)
    with pytest.raises(sc.ScError):
        ctx.set_option(sc._sc.SC_OPT_TRACE_BLOCKS, 0)
    with pytest.raises(sc.ScError):
        ctx.set_option(sc._sc.SC_OPT_TRACE_BLOCKS, 17)
