"""Parity of the HIP path with the oracle on absorbing, rough, nested and
overlapping glass, through the C ABI.

Bar, as for clear glass: photon counts per cell exact, caustic-map cells
within 1e-5 relative (floor 1e-3 of the largest cell), outcome counts
exact; with the oracle's caustic map fed to both sides the image and the
ground-truth outputs are bit-exact (both sides take every decision, and
compute every weight, in the same float operations).  At full photon
counts the slab transmittance is checked against the incoherent
multilayer closed form instead of the oracle.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu

AOV_KEYS = ("obj", "trans", "tri", "depth", "depthn", "normal", "normal_cam", "albedo")


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_11008_amd as sc
    return sc.Context(0)


def _bits(x):
    return np.ascontiguousarray(x).view(np.uint32)


def _photons_match(r, msum, ocnt, ost):
    assert np.array_equal(r["count"].cpu().numpy().view(np.uint32), ocnt)
    g = r["map"].cpu().numpy().astype(np.float64)
    floor = 1e-3 * float(np.abs(msum).max())
    assert np.all(np.abs(g - msum) <= 1e-5 * np.maximum(np.abs(msum), floor))
    for k in oracle.PH_OUTCOMES:
        assert r["stats"][k][1] == ost[k][1], k
        assert abs(r["stats"][k][0] - ost[k][0]) <= 1e-9 * max(1.0, ost[k][0]), k
    assert r["stats"]["segments"] == ost["segments"]


def _parity(ctx, c, spp):
    scene, wl, cam, md = c["scene"], c["wavelengths"], c["camera"], c["max_depth"]
    osc = oracle.OracleScene(scene)
    om, msum, ocnt, ost = oracle.trace_photons(osc, c["n_photons"], md, wl, c["photon_seed"])
    o = oracle.render(osc, cam, spp, md, wl, c["render_seed"], caustic_map=om)
    bvh = ctx.build_bvh(scene)
    r = ctx.trace_photons(bvh, c["n_photons"], md, wl, c["photon_seed"], counts=True, stats=True)
    _photons_match(r, msum, ocnt, ost)
    g = ctx.render(bvh, cam, spp, md, wl, c["render_seed"], caustic_map=torch.from_numpy(om).cuda(),
                   outputs=("rgb",) + AOV_KEYS)
    assert np.array_equal(_bits(g["rgb"].cpu().numpy()), _bits(o["rgb"]))
    for k in AOV_KEYS:
        gv = g[k].cpu().numpy()
        if k in ("obj", "tri"):
            gv = gv.view(np.uint32)
        if gv.dtype == np.float32:
            assert np.array_equal(_bits(gv), _bits(o[k])), k
        else:
            assert np.array_equal(gv, o[k]), k
    return o


def test_tinted_nested_parity(ctx):
    o = _parity(ctx, sg.tinted_nested(), 2)
    assert o["rgb"].max() > 0


def test_soft_light_parity(ctx):
    """The caustic-softness knob: the point light as a square emitter."""
    c = sg.config1(light_size=0.6)
    c["n_photons"] = 1 << 15
    _parity(ctx, c, 1)


def test_rich_medium_scene_parity(ctx):
    """The medium scene with tinted and rough glass, shrunk."""
    c = sg.config2(tri_scale=0.03, w=40, h=32, glass_style="rich")
    c["n_photons"] = 1 << 14
    _parity(ctx, c, 2)


def test_overlapping_glass_parity():
    """The large scene's 40 overlapping glass meshes, shrunk: surfaces
    inside other glass are crossed by priority on both sides."""
    import paper_2107_11008_amd as sc
    c = sg.config3(tri_scale=0.01, w=40, h=24)
    c["n_photons"] = 1 << 14
    _parity(sc.Context(0), c, 1)


def _gpu_transmittance(ctx, layers, lam, n_photons, max_depth=32, seed=21):
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (lam,))
    r = ctx.trace_photons(ctx.build_bvh(sg.slab_stack(layers)), n_photons, max_depth, wl, seed, stats=True)
    clear = [(sz, zc, dict(m, sigma=np.zeros(3, np.float32))) for sz, zc, m in layers]
    r0 = ctx.trace_photons(ctx.build_bvh(sg.slab_stack(clear)), n_photons, max_depth, wl, seed, stats=True)
    total = sum(v[0] for k, v in r0["stats"].items() if k != "segments")
    assert r["stats"]["truncated"][1] < n_photons * 1e-4
    return r["stats"]["deposited"][0] / total


def _interface(n1, n2):
    rr = ((n1 - n2) / (n1 + n2)) ** 2
    return (rr, rr, 1.0 - rr)


def _stack(*elems):
    acc = elems[0]
    for b in elems[1:]:
        ra, rab, ta = acc
        rb, rbb, tb = b
        den = 1.0 - rab * rb
        acc = (ra + ta * ta * rb / den, rbb + tb * tb * rab / den, ta * tb / den)
    return acc[2]


def test_nested_absorbing_slab_closed_form_at_scale(ctx):
    n = 1 << 22
    outer = ((1.0, 1.0, 0.4), 0.7, sg.glass(1.5, sigma=(0.2, 0.5, 3.0), priority=1))
    inner = ((0.6, 0.6, 0.1), 0.7, sg.glass(1.9, sigma=(2.0, 2.0, 2.0), priority=2))
    got = _gpu_transmittance(ctx, [outer, inner], 600.0, n)   # sigma_outer(600) = 1.75
    want = _stack(_interface(1.0, 1.5), (0.0, 0.0, math.exp(-1.75 * 0.15)), _interface(1.5, 1.9),
                  (0.0, 0.0, math.exp(-0.2)), _interface(1.9, 1.5), (0.0, 0.0, math.exp(-1.75 * 0.15)),
                  _interface(1.5, 1.0))
    assert abs(got - want) < 2.5 / math.sqrt(n), (got, want)


@pytest.mark.parametrize("field,value", [("sigma", (-1.0, 0.0, 0.0)), ("sigma", (0.0, float("nan"), 0.0)),
                                         ("sigma", (0.0, 0.0, float("inf"))), ("roughness", 1.5),
                                         ("roughness", -0.1), ("roughness", float("nan"))])
def test_bad_glass_parameters_rejected(ctx, field, value):
    import paper_2107_11008_amd as sc
    c = sg.config1()
    s = c["scene"]
    m = s.materials.copy()
    m[2][field] = value
    bad = sg.Scene(V=s.V, I=s.I, VN=s.VN, tri_obj=s.tri_obj, materials=m, point_lights=s.point_lights,
                   targets_obj=s.targets_obj, targets_sphere=s.targets_sphere, receiver=s.receiver)
    with pytest.raises(sc.ScError):
        ctx.build_bvh(bad)
