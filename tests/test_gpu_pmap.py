"""Parity of the HIP general photon map and RGB textures with the oracle,
through the C ABI.

Bar: stored photons bit-exact (position, normal, flux, channel, photon
index; same set, compared in photon order), the fixed-point scale equal,
every gather bit-exact (the disc sum is an exact integer on both sides),
images and ground truth bit-exact when both sides gather from their own
(identical) maps.  At the benchmark's photon count the stored set is
checked against the receiver-map pass's outcome counts and sampled
gathers against a brute-force sum over the exported photons.
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


def _same_records(g, o):
    assert len(g["phi"]) == len(o)
    assert np.array_equal(g["photon"], o["photon"])
    assert np.array_equal(_bits(g["pos"]), _bits(o["pos"]))
    assert np.array_equal(_bits(g["nrm"]), _bits(o["nrm"]))
    assert np.array_equal(_bits(g["phi"]), _bits(o["phi"]))
    assert np.array_equal(g["channel"], o["channel"])


def _clutter(n_photons=1 << 13, w=24, h=16):
    c = sg.config3(tri_scale=0.02, w=w, h=h, floor="rgb")
    c["n_photons"] = n_photons
    c["max_depth"] = 10
    return c


@pytest.mark.parametrize("which", ["c1", "clutter", "tinted"])
def test_stored_photons_equal_oracle(ctx, which):
    c = {"c1": sg.config1, "clutter": _clutter, "tinted": sg.tinted_nested}[which]()
    radius = 0.05
    scene, wl = c["scene"], c["wavelengths"]
    o, ost = oracle.pm_trace(oracle.OracleScene(scene), c["n_photons"], c["max_depth"], wl, c["photon_seed"])
    pm = ctx.pmap_trace(ctx.build_bvh(scene), c["n_photons"], c["max_depth"], wl, c["photon_seed"], radius, stats=True)
    _same_records(pm.export(), o)
    for k in oracle.PH_OUTCOMES:
        assert pm.stats[k][1] == ost[k][1], k
    inf = pm.info()
    assert inf["n_stored"] == len(o) and inf["scale"] == oracle.pm_scale(o)
    assert inf["channels"] == wl.channels and inf["radius"] == np.float32(radius)


def test_gathers_equal_oracle(ctx):
    c = _clutter()
    scene, wl = c["scene"], c["wavelengths"]
    o, _ = oracle.pm_trace(oracle.OracleScene(scene), c["n_photons"], c["max_depth"], wl, c["photon_seed"])
    rng = np.random.default_rng(4)
    k = rng.integers(0, len(o), 300)
    N = o["nrm"][k].copy()
    N[::7] = -N[::7]                           # some from the other side
    ch = o["channel"][k].astype(np.uint32)
    for radius in (0.004, 0.03):
        P = (o["pos"][k] + rng.normal(scale=0.4 * radius, size=(300, 3))).astype(np.float32)
        pm = ctx.pmap_trace(ctx.build_bvh(scene), c["n_photons"], c["max_depth"], wl, c["photon_seed"], radius)
        E = pm.gather(torch.from_numpy(P).cuda(), torch.from_numpy(N).cuda(),
                      torch.from_numpy(ch.view(np.int32)).cuda()).cpu().numpy()
        want = np.array([oracle.pm_gather(o, radius, P[i], N[i], int(ch[i])) for i in range(len(P))], np.float32)
        assert np.array_equal(_bits(E), _bits(want)), radius
        assert (want > 0).mean() > 0.5, radius


@pytest.mark.parametrize("which", ["clutter", "tinted"])
def test_render_with_general_map_bitexact(ctx, which):
    c = _clutter() if which == "clutter" else sg.tinted_nested(w=32, h=24)
    radius = 0.03
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    osc = oracle.OracleScene(scene)
    o_rec, _ = oracle.pm_trace(osc, c["n_photons"], c["max_depth"], wl, c["photon_seed"])
    o = oracle.render_pm(osc, cam, 1, c["max_depth"], wl, c["render_seed"], o_rec, radius)
    bvh = ctx.build_bvh(scene)
    pm = ctx.pmap_trace(bvh, c["n_photons"], c["max_depth"], wl, c["photon_seed"], radius)
    g = ctx.render(bvh, cam, 1, c["max_depth"], wl, c["render_seed"], pmap=pm, outputs=("rgb",) + AOV_KEYS)
    assert np.array_equal(_bits(g["rgb"].cpu().numpy()), _bits(o["rgb"]))
    for key in AOV_KEYS:
        gv = g[key].cpu().numpy()
        if key in ("obj", "tri"):
            gv = gv.view(np.uint32)
        if gv.dtype == np.float32:
            assert np.array_equal(_bits(gv), _bits(o[key])), key
        else:
            assert np.array_equal(gv, o[key]), key
    assert o["rgb"].max() > 0


def test_rgb_floor_with_receiver_map_bitexact(ctx):
    c = _clutter()
    scene, wl, cam = c["scene"], c["wavelengths"], c["camera"]
    osc = oracle.OracleScene(scene)
    om, _, _, _ = oracle.trace_photons(osc, c["n_photons"], c["max_depth"], wl, c["photon_seed"])
    o = oracle.render(osc, cam, 2, c["max_depth"], wl, c["render_seed"], caustic_map=om)
    g = ctx.render(ctx.build_bvh(scene), cam, 2, c["max_depth"], wl, c["render_seed"],
                   caustic_map=torch.from_numpy(om).cuda(), outputs=("rgb", "albedo"))
    assert np.array_equal(_bits(g["rgb"].cpu().numpy()), _bits(o["rgb"]))
    assert np.array_equal(_bits(g["albedo"].cpu().numpy()), _bits(o["albedo"]))


def test_medium_scene_general_map_at_scale(ctx):
    """The benchmark's medium scene at 2^22 photons: every caustic photon
    is stored (the receiver pass's deposited + elsewhere + outside), and
    sampled gathers equal a brute-force fixed-point sum over the export."""
    c = sg.config2()
    scene, wl = c["scene"], c["wavelengths"]
    bvh = ctx.build_bvh(scene)
    rm = ctx.trace_photons(bvh, c["n_photons"], c["max_depth"], wl, c["photon_seed"], stats=True)["stats"]
    radius = 0.004
    pm = ctx.pmap_trace(bvh, c["n_photons"], c["max_depth"], wl, c["photon_seed"], radius, stats=True)
    rec = pm.export()
    n = len(rec["phi"])
    assert n == rm["deposited"][1] + rm["elsewhere"][1] + rm["outside"][1]
    assert np.all(np.diff(rec["photon"].astype(np.int64)) > 0)
    scale = pm.info()["scale"]
    q = np.rint(rec["phi"].astype(np.float64) * scale).astype(np.uint64)
    assert float(q.astype(np.float64).sum()) <= 2.0 ** 62
    rng = np.random.default_rng(9)
    k = rng.integers(0, n, 64)
    P = (rec["pos"][k] + rng.normal(scale=0.002, size=(64, 3))).astype(np.float32)
    N = rec["nrm"][k].copy()
    ch = rec["channel"][k].astype(np.uint32)
    E = pm.gather(torch.from_numpy(P).cuda(), torch.from_numpy(N).cuda(),
                  torch.from_numpy(ch.view(np.int32)).cuda()).cpu().numpy()
    r2 = np.float32(radius) * np.float32(radius)
    cnorm = 1.0 / ((scale * 3.14159265358979323846) * (float(np.float32(radius)) * float(np.float32(radius))))
    for i in range(64):
        d = rec["pos"] - P[i]
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]          # float32, in order
        side = ((rec["nrm"][:, 0] * N[i, 0] + rec["nrm"][:, 1] * N[i, 1]) + rec["nrm"][:, 2] * N[i, 2]) > 0
        sel = (d2 < r2) & side & (rec["channel"] == ch[i])
        want = np.float32(float(int(q[sel].sum())) * cnorm)
        assert E[i] == want, (i, E[i], want)
    img = ctx.render(bvh, sg.look_at((0.0, -1.6, 1.6), (0.0, 0.0, 0.05), (0, 0, 1), 40.0, 128, 128), 2,
                     c["max_depth"], wl, 3, pmap=pm, outputs=("rgb",))["rgb"]
    assert torch.isfinite(img).all() and float(img.max()) > 0


def test_pmap_argument_errors(ctx):
    import paper_2107_11008_amd as sc
    c = sg.config1()
    bvh = ctx.build_bvh(c["scene"])
    for r in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(sc.ScError):
            ctx.pmap_trace(bvh, 1 << 10, 8, c["wavelengths"], 1, r)
    with pytest.raises(sc.ScError):
        ctx.pmap_trace(bvh, 1 << 12, 8, c["wavelengths"], 1, 1e-7)     # grid would exceed 2^16 cells
    pm = ctx.pmap_trace(bvh, 1 << 12, 8, c["wavelengths"], 1, 0.05)
    with pytest.raises(sc.ScError):
        ctx.render(bvh, c["camera"], 1, 8, sg.Wavelengths(sg.WL_UNIFORM, 1, (550.0,), 380.0, 720.0, 16), 1, pmap=pm)


def test_retrace_in_place(ctx):
    """A map rebuilt in an existing handle equals a fresh one; after a failed
    rebuild the handle refuses use until a rebuild succeeds."""
    import paper_2107_11008_amd as sc
    c = _clutter()
    wl = c["wavelengths"]
    bvh = ctx.build_bvh(c["scene"])
    pm = ctx.pmap_trace(bvh, 1 << 10, 6, wl, 1, 0.05)
    args = (bvh, c["n_photons"], c["max_depth"], wl, c["photon_seed"], 0.03)
    assert ctx.pmap_trace(*args, out=pm) is pm                      # grows the handle's memory
    fresh = ctx.pmap_trace(*args)
    a, b = pm.export(), fresh.export()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
    assert pm.info() == fresh.info()
    with pytest.raises(sc.ScError):
        ctx.pmap_trace(bvh, c["n_photons"], c["max_depth"], wl, c["photon_seed"], 0.0, out=pm)
    P = torch.zeros((1, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(sc.ScError):
        pm.gather(P, P, torch.zeros(1, dtype=torch.int32, device="cuda"))
    with pytest.raises(sc.ScError):
        ctx.render(bvh, c["camera"], 1, 4, wl, 1, pmap=pm, outputs=("rgb",))
    ctx.pmap_trace(*args, out=pm)
    a = pm.export()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
