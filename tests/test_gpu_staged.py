"""The hybrid schedule: the first bounces as one launch per stage, the
remaining paths finished by one lane each.  Any switch depth must give the
same images, caustic maps, photon counts and photon outcome statistics, bit
for bit (the per-path functions are the same; only the schedule changes)."""
import numpy as np
import pytest
import torch

import scenegen as sg

pytestmark = pytest.mark.gpu

# (camera, photon) switch depths; the first is the reference
DEPTHS = ((0, 0), (1, 1), (2, 5), (3, 2), (5, 1), (1, 3))


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
        ctx.set_option(sc._sc.SC_OPT_STAGED_DEPTH, 4)      # the library's defaults
        ctx.set_option(sc._sc.SC_OPT_PHOTON_STAGED_DEPTH, 1)


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
