"""Parity of the HIP path with the CPU oracle, through the C ABI.

Bar (from the method's outputs): triangle id, object id, mask and depth
bit-exact; the traced paths are bit-identical, so radiance is bit-exact
when both sides gather from the same caustic map, and within 1e-4
relative (99.9% of pixels, mean within 1e-5) with each side's own map;
caustic-map cells within 1e-5 relative (floor 1e-3 of the largest cell),
per-cell photon counts exact.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import scenegen as sg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2107_11008_amd as sc
    return sc.Context(0)


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bits(x):
    return np.ascontiguousarray(x).view(np.uint32)


def _rays(rng, n, center, spread, targets=None):
    O = (center + rng.normal(size=(n, 3)) * spread).astype(np.float32)
    if targets is None:
        D = rng.normal(size=(n, 3))
    else:
        D = targets[rng.integers(0, len(targets), size=n)] - O
    D = (D / np.linalg.norm(D, axis=1, keepdims=True)).astype(np.float32)
    return O, D


def _scene_c2_small(seed=2000, scale=0.03):
    c = sg.config2(seed=seed, tri_scale=scale, w=64, h=64)
    return c


@pytest.mark.parametrize("which", ["c1", "c2s", "soup"])
@pytest.mark.parametrize("n", [1, 63, 65, 5000])
def test_closest_hit_bitexact(ctx, which, n):
    rng = np.random.default_rng(n)
    if which == "c1":
        scene = sg.config1()["scene"]
        center, spread = np.array([0, 0, 1.5]), 3.0
    elif which == "c2s":
        scene = _scene_c2_small()["scene"]
        center, spread = np.array([0, 0, 0.2]), 0.8
    else:
        b = sg.SceneBuilder()
        V = rng.uniform(-1, 1, size=(600, 3))
        b.add(sg.Mesh(V, np.arange(600).reshape(200, 3), np.tile([0, 0, 1.0], (600, 1))),
              dict(type=sg.MAT_DIFFUSE, rho_a=0.5))
        scene = b.build(None)
        center, spread = np.zeros(3), 2.0
    V = scene.V.astype(np.float64)
    I = scene.I
    targets = np.concatenate([V, 0.5 * (V[I[:, 0]] + V[I[:, 1]])])
    O1, D1 = _rays(rng, n // 2 + 1, center, spread)
    O2, D2 = _rays(rng, n - n // 2 - 1, center, spread, targets)
    O, D = np.concatenate([O1, O2])[:n], np.concatenate([D1, D2])[:n]
    osc = oracle.OracleScene(scene)
    to, po, uo, vo = oracle.closest(osc, O, D)
    bvh = ctx.build_bvh(scene)
    t, p, u, v = [x.cpu().numpy() for x in ctx.trace_rays(bvh, _t(O), _t(D))]
    assert np.array_equal(p.view(np.uint32), po)
    assert np.array_equal(_bits(t), _bits(to))
    assert np.array_equal(_bits(u), _bits(uo))
    assert np.array_equal(_bits(v), _bits(vo))


@pytest.mark.parametrize("width,leaf", [(8, 4), (4, 1), (8, 8), (4, 3)])
def test_bvh_shape_does_not_change_hits(ctx, width, leaf):
    """Width and leaf size change only the traversal, never the result."""
    c = _scene_c2_small(scale=0.05)
    scene = c["scene"]
    rng = np.random.default_rng(5)
    O, D = _rays(rng, 4000, np.array([0, 0, 0.2]), 0.8)
    ref = oracle.closest(oracle.OracleScene(scene), O, D)
    bvh = ctx.build_bvh(scene, width=width, leaf_max=leaf)
    info = bvh.info()
    assert info["width"] == width and info["leaf_max"] == leaf
    t, p, u, v = [x.cpu().numpy() for x in ctx.trace_rays(bvh, _t(O), _t(D))]
    assert np.array_equal(p.view(np.uint32), ref[1])
    assert np.array_equal(_bits(t), _bits(ref[0]))


def test_any_hit_exact(ctx):
    c = sg.config1()
    scene = c["scene"]
    rng = np.random.default_rng(9)
    O, D = _rays(rng, 7000, np.array([0, 0, 1.5]), 2.5)
    tmax = rng.uniform(0.05, 8.0, size=len(O)).astype(np.float32)
    osc = oracle.OracleScene(scene)
    t, p, _, _ = oracle.closest(osc, O, D)
    excl = np.where(rng.uniform(size=len(O)) < 0.5, p, 0xFFFFFFFF).astype(np.uint32)
    ref = oracle.any_hit(osc, O, D, tmax, excl)
    bvh = ctx.build_bvh(scene)
    occ = ctx.occluded(bvh, _t(O), _t(D), _t(tmax), _t(excl.view(np.int32))).cpu().numpy().astype(bool)
    assert np.array_equal(occ, ref)


@pytest.mark.parametrize("offset", [(0.0, 0.0, 0.0), (3000.0, -2000.0, 500.0), (-40000.0, 25000.0, 0.0)])
def test_hits_far_from_the_origin(ctx, offset):
    """A triangle soup placed far from the world origin, rays starting on
    its triangles (as secondary rays do) or within a millimetre of them.
    The box test crosses a plane at p * inv + c with c = -o * inv, whose
    rounding grows with |o| while the distances stay small; its per-ray
    margins must keep every box that holds a hit, so closest hits
    (triangle, t, barycentrics) and occlusion equal the oracle's bit for
    bit.  The oracle's own traversal shares none of that arithmetic."""
    rng = np.random.default_rng(17)
    off = np.array(offset)
    b = sg.SceneBuilder()
    C = rng.uniform(-1, 1, size=(300, 3))
    V = np.repeat(C, 3, axis=0) + rng.normal(scale=0.05, size=(900, 3)) + off
    b.add(sg.Mesh(V, np.arange(900).reshape(300, 3), np.tile([0, 0, 1.0], (900, 1))),
          dict(type=sg.MAT_DIFFUSE, rho_a=0.5))
    scene = b.build(None)
    V = scene.V.astype(np.float64)
    I = scene.I
    k = rng.integers(0, len(I), size=3000)
    w = rng.dirichlet([1.0, 1.0, 1.0], size=3000)
    P = w[:, :1] * V[I[k, 0]] + w[:, 1:2] * V[I[k, 1]] + w[:, 2:] * V[I[k, 2]]
    O = np.concatenate([P, P + rng.normal(scale=1e-3, size=P.shape)]).astype(np.float32)
    D = rng.normal(size=O.shape)
    D = (D / np.linalg.norm(D, axis=1, keepdims=True)).astype(np.float32)
    osc = oracle.OracleScene(scene)
    to, po, uo, vo = oracle.closest(osc, O, D)
    bvh = ctx.build_bvh(scene)
    t, p, u, v = [x.cpu().numpy() for x in ctx.trace_rays(bvh, _t(O), _t(D))]
    assert np.array_equal(p.view(np.uint32), po)
    assert np.array_equal(_bits(t), _bits(to))
    assert np.array_equal(_bits(u), _bits(uo))
    assert np.array_equal(_bits(v), _bits(vo))
    hit = po != 0xFFFFFFFF
    assert hit.sum() > len(O) // 4   # most rays meet another triangle
    tmax = rng.uniform(0.01, 2.0, size=len(O)).astype(np.float32)
    excl = np.where(rng.uniform(size=len(O)) < 0.5, po, 0xFFFFFFFF).astype(np.uint32)
    ref = oracle.any_hit(osc, O, D, tmax, excl)
    occ = ctx.occluded(bvh, _t(O), _t(D), _t(tmax), _t(excl.view(np.int32))).cpu().numpy().astype(bool)
    assert np.array_equal(occ, ref)


def _oracle_aov(scene, cam, wl, spp=1, depth=1, seed=1, cmap=None, pixels=None):
    return oracle.render(oracle.OracleScene(scene), cam, spp, depth, wl, seed, caustic_map=cmap, pixels=pixels,
                         want_tie=True)


AOV_KEYS = ("obj", "trans", "tri", "depth", "depthn", "normal", "normal_cam", "albedo")


def _cmp_aov(g, o, mask=None):
    for k in AOV_KEYS:
        gv = g[k].cpu().numpy()
        ov = o[k]
        if k in ("obj", "tri"):
            gv = gv.view(np.uint32)
        if mask is not None:
            gv, ov = gv[mask], ov[mask]
        if gv.dtype == np.float32:
            assert np.array_equal(_bits(gv), _bits(ov)), k
        else:
            assert np.array_equal(gv, ov), k


def test_ground_truth_c1_bitexact(ctx):
    c = sg.config1()
    o = _oracle_aov(c["scene"], c["camera"], c["wavelengths"])
    bvh = ctx.build_bvh(c["scene"])
    g = ctx.render(bvh, c["camera"], 1, 1, c["wavelengths"], 1, outputs=AOV_KEYS)
    assert o["tie"].sum() == 0
    _cmp_aov(g, o)


def _photon_cmp(g_map, g_cnt, o_map64, o_cnt):
    o32 = o_map64.astype(np.float32)
    assert np.array_equal(g_cnt.view(np.uint32), o_cnt)
    floor = 1e-3 * float(np.abs(o_map64).max())
    err = np.abs(g_map.astype(np.float64) - o_map64)
    assert np.all(err <= 1e-5 * np.maximum(np.abs(o_map64), floor))
    return o32


def test_photons_c1(ctx):
    c = sg.config1()
    scene, wl = c["scene"], c["wavelengths"]
    osc = oracle.OracleScene(scene)
    om, msum, ocnt, ost = oracle.trace_photons(osc, c["n_photons"], c["max_depth"], wl, c["photon_seed"])
    bvh = ctx.build_bvh(scene)
    r = ctx.trace_photons(bvh, c["n_photons"], c["max_depth"], wl, c["photon_seed"], counts=True, stats=True)
    _photon_cmp(r["map"].cpu().numpy(), r["count"].cpu().numpy(), msum, ocnt)
    for k in oracle.PH_OUTCOMES:
        assert r["stats"][k][1] == ost[k][1], k
        assert abs(r["stats"][k][0] - ost[k][0]) <= 1e-9 * max(1.0, ost[k][0]), k
    assert r["stats"]["segments"] == ost["segments"]


def test_radiance_c1_same_map_bitexact(ctx):
    """With the oracle's caustic map fed to both sides every path is traced
    identically, so the image is bit-exact."""
    c = sg.config1()
    scene, wl = c["scene"], c["wavelengths"]
    osc = oracle.OracleScene(scene)
    om, _, _, _ = oracle.trace_photons(osc, c["n_photons"], c["max_depth"], wl, c["photon_seed"])
    o = oracle.render(osc, c["camera"], c["spp"], c["max_depth"], wl, c["render_seed"], caustic_map=om)
    bvh = ctx.build_bvh(scene)
    g = ctx.render(bvh, c["camera"], c["spp"], c["max_depth"], wl, c["render_seed"], caustic_map=_t(om))
    assert np.array_equal(_bits(g["rgb"].cpu().numpy()), _bits(o["rgb"]))
    _cmp_aov(g, o)


def _radiance_ok(g, o):
    g = g.astype(np.float64)
    o = o.astype(np.float64)
    for ch in range(3):
        gc, oc = g[..., ch], o[..., ch]
        floor = 1e-3 * oc.mean()
        ok = np.abs(gc - oc) <= 1e-4 * np.maximum(np.abs(oc), floor)
        assert ok.mean() >= 0.999, (ch, ok.mean())
        assert abs(gc.mean() - oc.mean()) <= 1e-5 * oc.mean(), ch


def test_radiance_c1_own_maps(ctx):
    """Each side gathers from its own photon map."""
    c = sg.config1()
    scene, wl = c["scene"], c["wavelengths"]
    osc = oracle.OracleScene(scene)
    om, _, _, _ = oracle.trace_photons(osc, c["n_photons"], c["max_depth"], wl, c["photon_seed"])
    o = oracle.render(osc, c["camera"], c["spp"], c["max_depth"], wl, c["render_seed"], caustic_map=om)
    bvh = ctx.build_bvh(scene)
    gm = ctx.trace_photons(bvh, c["n_photons"], c["max_depth"], wl, c["photon_seed"])["map"]
    g = ctx.render(bvh, c["camera"], c["spp"], c["max_depth"], wl, c["render_seed"], caustic_map=gm)
    _radiance_ok(g["rgb"].cpu().numpy(), o["rgb"])


@pytest.mark.parametrize("spp,cap", [(3, None), (5, 4096)])
def test_radiance_c2_small_spectral(ctx, spp, cap):
    """Spectral sampling, area light, texture, several objects; with a tiny
    queue capacity the image is processed in many sample chunks, and with a
    tiny photon chunk the photon pass in many chunks, and neither output
    may change."""
    c = _scene_c2_small()
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    osc = oracle.OracleScene(scene)
    n_ph = 1 << 15
    om, msum, ocnt, _ = oracle.trace_photons(osc, n_ph, c["max_depth"], wl, c["photon_seed"])
    o = oracle.render(osc, cam, spp, c["max_depth"], wl, c["render_seed"], caustic_map=om)
    if cap:
        ctx.set_option(3, cap)
        ctx.set_option(7, cap)
    try:
        bvh = ctx.build_bvh(scene)
        r = ctx.trace_photons(bvh, n_ph, c["max_depth"], wl, c["photon_seed"], counts=True)
        _photon_cmp(r["map"].cpu().numpy(), r["count"].cpu().numpy(), msum, ocnt)
        g = ctx.render(bvh, cam, spp, c["max_depth"], wl, c["render_seed"], caustic_map=_t(om))
    finally:
        ctx.set_option(3, 1 << 27)
        ctx.set_option(7, 1 << 24)
    assert np.array_equal(_bits(g["rgb"].cpu().numpy()), _bits(o["rgb"]))
    _cmp_aov(g, o)


@pytest.mark.parametrize("w,h", [(1, 1), (37, 23), (65, 3)])
def test_radiance_ragged_image_sizes(ctx, w, h):
    """Images whose pixel counts fill no wave or block evenly (one pixel;
    37 x 23; a 65-pixel-wide strip): with the oracle's caustic map on both
    sides the image and every ground-truth buffer are bit-exact."""
    c = sg.config2(seed=2001, tri_scale=0.03, w=w, h=h)
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    osc = oracle.OracleScene(scene)
    om, _, _, _ = oracle.trace_photons(osc, 1 << 14, c["max_depth"], wl, c["photon_seed"])
    o = oracle.render(osc, cam, 2, c["max_depth"], wl, c["render_seed"], caustic_map=om)
    bvh = ctx.build_bvh(scene)
    g = ctx.render(bvh, cam, 2, c["max_depth"], wl, c["render_seed"], caustic_map=_t(om))
    assert g["rgb"].shape == (h, w, 3)
    assert np.array_equal(_bits(g["rgb"].cpu().numpy()), _bits(o["rgb"]))
    _cmp_aov(g, o)


def test_determinism(ctx):
    c = sg.config1()
    bvh = ctx.build_bvh(c["scene"])
    a = ctx.trace_photons(bvh, 1 << 14, 8, c["wavelengths"], 3)["map"].cpu().numpy()
    b = ctx.trace_photons(bvh, 1 << 14, 8, c["wavelengths"], 3)["map"].cpu().numpy()
    assert np.array_equal(_bits(a), _bits(b))
    g1 = ctx.render(bvh, c["camera"], 2, 8, c["wavelengths"], 5, caustic_map=torch.from_numpy(a).cuda())
    g2 = ctx.render(bvh, c["camera"], 2, 8, c["wavelengths"], 5, caustic_map=torch.from_numpy(a).cuda())
    assert np.array_equal(_bits(g1["rgb"].cpu().numpy()), _bits(g2["rgb"].cpu().numpy()))


def test_empty_inputs(ctx):
    """Zero rays through each ray entry point return at once with nothing
    written; a pass of zero photons leaves an all-zero map and counts; a
    render of zero samples per pixel is refused (documented EINVAL)."""
    import paper_2107_11008_amd as sc
    c = sg.config1()
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    bvh = ctx.build_bvh(scene)
    O = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    D = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    t, p, u, v = ctx.trace_rays(bvh, O, D)
    assert t.numel() == 0 and p.numel() == 0 and u.numel() == 0 and v.numel() == 0
    occ = ctx.occluded(bvh, O, D, torch.empty(0, dtype=torch.float32, device="cuda"))
    assert occ.numel() == 0
    t0 = torch.full((4,), 7.0, dtype=torch.float32, device="cuda")
    p0 = torch.full((4,), 5, dtype=torch.int32, device="cuda")
    ctx.trace_rays_noalloc(bvh, O, D, t0, p0)
    assert torch.all(t0 == 7.0) and torch.all(p0 == 5)   # nothing written
    m = torch.full((scene.receiver.hc, scene.receiver.wc, wl.channels), 3.0, dtype=torch.float32, device="cuda")
    r = ctx.trace_photons(bvh, 0, c["max_depth"], wl, 1, counts=True, out=m)
    assert torch.count_nonzero(r["map"]).item() == 0
    assert torch.count_nonzero(r["count"]).item() == 0
    with pytest.raises(sc.ScError):
        ctx.render(bvh, cam, 0, c["max_depth"], wl, 1)


def test_single_triangle_and_degenerate(ctx):
    """One triangle, plus degenerate and non-finite triangles that never hit."""
    b = sg.SceneBuilder()
    V = np.array([[-1, -1, 0], [1, -1, 0], [0, 1, 0]], np.float64)
    b.add(sg.Mesh(V, np.array([[0, 1, 2]]), np.tile([0, 0, 1.0], (3, 1))), dict(type=sg.MAT_DIFFUSE, rho_a=0.5))
    one = b.build(None)
    b2 = sg.SceneBuilder()
    b2.add(sg.Mesh(V, np.array([[0, 1, 2]]), np.tile([0, 0, 1.0], (3, 1))), dict(type=sg.MAT_DIFFUSE, rho_a=0.5))
    Vd = np.array([[0, 0, 0.5], [0, 0, 0.5], [0.1, 0, 0.5], [np.nan, 0, 1], [0, 1, 1], [1, 0, 1]], np.float64)
    b2.add(sg.Mesh(Vd, np.array([[0, 1, 2], [3, 4, 5]]), np.tile([0, 0, 1.0], (6, 1))),
           dict(type=sg.MAT_DIFFUSE, rho_a=0.5))
    bad = b2.build(None)
    rng = np.random.default_rng(1)
    O = np.tile(np.array([0, 0, 3], np.float32), (500, 1))
    D = np.concatenate([rng.uniform(-0.3, 0.3, size=(500, 2)), -np.ones((500, 1))], 1)
    D = (D / np.linalg.norm(D, axis=1, keepdims=True)).astype(np.float32)
    for scene in (one, bad):
        ref = oracle.closest(oracle.OracleScene(scene), O, D)
        bvh = ctx.build_bvh(scene)
        t, p, u, v = [x.cpu().numpy() for x in ctx.trace_rays(bvh, _t(O), _t(D))]
        assert np.array_equal(p.view(np.uint32), ref[1])
        assert np.array_equal(_bits(t), _bits(ref[0]))
        assert (ref[1] != 0xFFFFFFFF).sum() > 100


def test_invalid_arguments_raise(ctx):
    import paper_2107_11008_amd as sc
    c = sg.config1()
    bvh = ctx.build_bvh(c["scene"])
    with pytest.raises(sc.ScError):
        ctx.render(bvh, c["camera"], 0, 8, c["wavelengths"], 1)
    with pytest.raises(sc.ScError):
        ctx.render(bvh, c["camera"], 1, 0, c["wavelengths"], 1)
    bad = sg.Wavelengths(sg.WL_FIXED, 2, (500.0, 600.0))
    with pytest.raises(sc.ScError):
        ctx.render(bvh, c["camera"], 1, 1, bad, 1)
    s = c["scene"]
    s2 = sg.Scene(V=s.V, I=s.I, VN=s.VN, tri_obj=np.full_like(s.tri_obj, 9), materials=s.materials,
                  point_lights=s.point_lights, targets_obj=s.targets_obj, targets_sphere=s.targets_sphere,
                  receiver=s.receiver)
    with pytest.raises(sc.ScError):
        ctx.build_bvh(s2)


def _full_size_sampled(ctx, c, n_map_photons=1 << 16, n_pix=96):
    """Render the full-size image on the GPU in the benchmark's launch
    configuration and a seeded sample of its pixels with the oracle, both
    gathering from one caustic map the oracle builds (full map resolution,
    fewer photons than the benchmark so that the oracle finishes quickly)."""
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    osc = oracle.OracleScene(scene)
    om, _, _, _ = oracle.trace_photons(osc, n_map_photons, c["max_depth"], wl, c["photon_seed"])
    bvh = ctx.build_bvh(scene)
    g = ctx.render(bvh, cam, c["spp"], c["max_depth"], wl, c["render_seed"], caustic_map=_t(om))
    rng = np.random.default_rng(11)
    pix = np.sort(rng.choice(cam.w * cam.h, size=n_pix, replace=False)).astype(np.uint32)
    o = oracle.render(osc, cam, c["spp"], c["max_depth"], wl, c["render_seed"], caustic_map=om, pixels=pix)
    m = np.zeros(cam.w * cam.h, bool)
    m[pix] = True
    m = m.reshape(cam.h, cam.w)
    assert np.array_equal(_bits(g["rgb"].cpu().numpy()[m]), _bits(o["rgb"][m]))
    _cmp_aov(g, o, mask=m)
    return g, osc


def test_c2_rich_glass_full_size_sampled_pixels(ctx):
    """The medium scene with tinted and rough glass (a benchmark leg) at
    full size, on sampled pixels."""
    _full_size_sampled(ctx, sg.config2(glass_style="rich"))


def test_c2_general_map_full_size_sampled_pixels(ctx):
    """The full-size medium scene rendered with the general photon map (a
    benchmark leg), on sampled pixels; each side builds its map from its own
    photon pass of 2^16 photons (the stored photons are equal bit for bit)."""
    c = sg.config2()
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    radius, n_ph = 4.0 / 1024, 1 << 16
    osc = oracle.OracleScene(scene)
    recs, _ = oracle.pm_trace(osc, n_ph, c["max_depth"], wl, c["photon_seed"])
    bvh = ctx.build_bvh(scene)
    pm = ctx.pmap_trace(bvh, n_ph, c["max_depth"], wl, c["photon_seed"], radius)
    g = ctx.render(bvh, cam, c["spp"], c["max_depth"], wl, c["render_seed"], pmap=pm, outputs=("rgb",))
    rng = np.random.default_rng(12)
    pix = np.sort(rng.choice(cam.w * cam.h, size=96, replace=False)).astype(np.uint32)
    o = oracle.render_pm(osc, cam, c["spp"], c["max_depth"], wl, c["render_seed"], recs, radius, pixels=pix)
    m = np.zeros(cam.w * cam.h, bool)
    m[pix] = True
    m = m.reshape(cam.h, cam.w)
    assert np.array_equal(_bits(g["rgb"].cpu().numpy()[m]), _bits(o["rgb"][m]))
    assert o["rgb"][m].max() > 0


def test_c2_full_size_sampled_pixels(ctx):
    """The full 512x512, 16 spp medium scene in the launch configuration the
    benchmark times, checked on a seeded sample of pixels the oracle
    renders one by one (both gathering from one oracle-built caustic map),
    and its ground truth on every 7th pixel."""
    c = sg.config2()
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    g, osc = _full_size_sampled(ctx, c)
    # full-size ground truth: every 7th pixel
    ogt = oracle.render(osc, cam, 1, 1, wl, 1, pixels=np.arange(0, cam.w * cam.h, 7, dtype=np.uint32))
    m2 = np.zeros(cam.w * cam.h, bool)
    m2[::7] = True
    _cmp_aov(g, ogt, mask=m2.reshape(cam.h, cam.w))


def test_photon_map_independent_of_earlier_passes(ctx):
    """The fixed-point accumulator is cleared cell by cell after each pass:
    a receiver map equals itself bit for bit when passes over other scenes,
    receiver sizes and photon counts, and a general photon map pass, ran in
    between on the same context."""
    c1 = sg.config1()
    c2 = _scene_c2_small()
    wl1, wl2 = c1["wavelengths"], c2["wavelengths"]
    b1, b2 = ctx.build_bvh(c1["scene"]), ctx.build_bvh(c2["scene"])
    first = ctx.trace_photons(b1, 1 << 14, c1["max_depth"], wl1, 5)["map"].cpu().numpy().copy()
    ctx.trace_photons(b2, 1 << 15, c2["max_depth"], wl2, 6)
    ctx.pmap_trace(b2, 1 << 13, c2["max_depth"], wl2, 7, 0.05)
    ctx.trace_photons(b1, 1 << 12, c1["max_depth"], wl1, 8)
    again = ctx.trace_photons(b1, 1 << 14, c1["max_depth"], wl1, 5)["map"].cpu().numpy()
    assert first.tobytes() == again.tobytes()
    assert first.max() > 0


def test_second_context_renders_from_shared_bvh(ctx):
    """A BVH is only read by rendering: a second context bound to another
    stream renders the same ground truth from it, bit for bit, while the
    first context traces photons on its own stream."""
    import paper_2107_11008_amd as sc
    c = sg.config1()
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    bvh = ctx.build_bvh(scene)
    keys = ("obj", "trans", "tri", "depth", "depthn", "normal", "albedo")
    ref = ctx.render(bvh, cam, 1, c["max_depth"], wl, 3, outputs=keys)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ctx2 = sc.Context(0)
    e = torch.cuda.Event()
    e.record(torch.cuda.current_stream())
    side.wait_event(e)
    g = ctx2.render(bvh, cam, 1, c["max_depth"], wl, 3, outputs=keys)
    ctx.trace_photons(bvh, 1 << 14, c["max_depth"], wl, 4)
    torch.cuda.synchronize()
    for k in keys:
        a, b = ref[k].cpu().numpy(), g[k].cpu().numpy()
        assert a.tobytes() == b.tobytes(), k
    ctx2.close()


def test_render_overlap_equals_render(ctx):
    """sc_render_overlap with the photon pass on another context and stream
    (the render waits for its event only at the first diffuse shading)
    gives sc_render's output bit for bit, for every output."""
    import paper_2107_11008_amd as sc
    c = _scene_c2_small()
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    bvh = ctx.build_bvh(scene)
    ref_map = ctx.trace_photons(bvh, 1 << 15, c["max_depth"], wl, c["photon_seed"])["map"]
    ref = ctx.render(bvh, cam, 3, c["max_depth"], wl, c["render_seed"], caustic_map=ref_map)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ctx2 = sc.Context(0)
    main = torch.cuda.current_stream()
    for rep in range(3):
        e0 = torch.cuda.Event()
        e0.record(main)
        side.wait_event(e0)
        m = ctx2.trace_photons(bvh, 1 << 15, c["max_depth"], wl, c["photon_seed"])["map"]
        e_map = torch.cuda.Event()
        e_map.record(side)
        g = ctx.render(bvh, cam, 3, c["max_depth"], wl, c["render_seed"], caustic_map=m, map_ready=e_map)
        torch.cuda.synchronize()
        assert m.cpu().numpy().tobytes() == ref_map.cpu().numpy().tobytes()
        for k in ref:
            assert ref[k].cpu().numpy().tobytes() == g[k].cpu().numpy().tobytes(), k
    with pytest.raises(sc.ScError):
        ctx.render(bvh, cam, 1, c["max_depth"], wl, 1, caustic_map=None, map_ready=torch.cuda.Event())
    ctx2.close()


def test_handles_outlive_their_context(ctx):
    """Handles made on a context that is destroyed first: the BVH still
    renders from another context (bit for bit as before), the network's
    calls fail with an error instead of touching the freed context, and
    freeing both afterwards is safe."""
    import paper_2107_11008_amd as sc
    c = sg.config1()
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    ctx2 = sc.Context(0)
    bvh = ctx2.build_bvh(scene)
    keys = ("obj", "tri", "depth")
    ref = ctx2.render(bvh, cam, 1, c["max_depth"], wl, 3, outputs=keys)
    ref = {k: v.cpu().numpy().copy() for k, v in ref.items()}
    net = sc.UNet(ctx2, (16, 16), None)
    torch.cuda.synchronize()
    ctx2.close()
    g = ctx.render(bvh, cam, 1, c["max_depth"], wl, 3, outputs=keys)
    for k in keys:
        assert g[k].cpu().numpy().tobytes() == ref[k].tobytes(), k
    with pytest.raises(sc.ScError):
        net.get_params()
    with pytest.raises(sc.ScError):
        bvh.export()
    net.close()
    bvh.close()
