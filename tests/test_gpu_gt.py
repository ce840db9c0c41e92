"""Ground-truth passes on the GPU against the oracle's definitions, on the
tiny scene's own renders: masks bit-exact."""
import numpy as np
import pytest
import torch

import scenegen as sg
from oracle import gt

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rendered():
    import paper_2107_11008_amd as sc
    ctx = sc.Context(0)
    c = sg.config1()
    bvh = ctx.build_bvh(c["scene"])
    m = ctx.trace_photons(bvh, c["n_photons"], c["max_depth"], c["wavelengths"], c["photon_seed"])["map"]
    return ctx, c, bvh, m


def test_caustic_mask_matches_definition(rendered):
    ctx, c, bvh, m = rendered
    mask, a, b, thr = ctx.render_caustic_mask(bvh, c["camera"], 4, c["max_depth"], c["wavelengths"], 7, m, rel=0.05)
    ref = gt.caustic_mask(a["rgb"].cpu().numpy(), b["rgb"].cpu().numpy(), a["trans"].cpu().numpy(), thr)
    got = mask.cpu().numpy()
    assert np.array_equal(got, ref)
    # the focused caustic under the sphere is non-local; glass pixels show local caustics
    assert (got == 2).sum() > 5 and (got == 1).sum() > 5
    # without the gather nothing differs
    n = ctx.caustic_mask(b["rgb"], b["rgb"], None, 0.0)
    assert int(n.sum()) == 0


@pytest.mark.parametrize("t", [1, 3, 8])
def test_outline_matches_definition(rendered, t):
    ctx, c, bvh, _ = rendered
    r = ctx.render(bvh, c["camera"], 1, 1, c["wavelengths"], 1, outputs=("obj",))
    got = ctx.outline(r["obj"], t).cpu().numpy()
    ref = gt.outline(r["obj"].cpu().numpy().view(np.uint32), t)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("t", [1, 3, 8, 12])
@pytest.mark.parametrize("w,h", [(131, 37), (64, 16), (1, 5), (200, 1)])
def test_outline_ragged_images(rendered, w, h, t):
    """Object-id images whose sides are not multiples of the 64 x 16 tile
    (and single rows or columns), thicknesses inside the one-launch tile
    path (<= 8) and past it (the two-pass path): equal to the definition."""
    import torch
    ctx = rendered[0]
    rng = np.random.default_rng(w * 1000 + h + t)
    ids = rng.integers(0, 4, size=(h, w)).astype(np.uint32)
    ids = np.where(rng.uniform(size=(h, w)) < 0.8, np.repeat(ids[:, :1], w, 1), ids)   # runs of one id
    got = ctx.outline(torch.from_numpy(ids.view(np.int32)).cuda(), t).cpu().numpy()
    ref = gt.outline(ids, t)
    assert np.array_equal(got, ref)


def test_occlusion_matches_definition(rendered):
    ctx, c, bvh, _ = rendered
    r = ctx.render(bvh, c["camera"], 1, 1, c["wavelengths"], 1, outputs=("depth",))
    for rel in (0.02, 0.1):
        got = ctx.occlusion_boundary(r["depth"], rel).cpu().numpy()
        ref = gt.occlusion_boundary(r["depth"].cpu().numpy(), rel)
        assert np.array_equal(got, ref)
        assert got.sum() > 20
