"""Pins of the oracle's general photon map and RGB albedo textures.

The paper's caustics land on whatever surface lies behind the glass
(Sec. III-D-6: caustic light falling on another surface); the general
photon map stores every caustic photon at its first diffuse hit on any
object and estimates irradiance over a disc of radius r (Jensen's photon
map density estimate with a fixed radius).  What pins it:

* its deposits restricted to the receiver rectangle are exactly the
  receiver map's (same photons, same cells, same FP64 sums in photon
  order), and the photons the receiver map counts as landing elsewhere or
  outside are exactly the extra records;
* under a clear slab lit at normal incidence by a distant point light of
  intensity I at distance L, the irradiance behind it is uniform,
  E0 = T I / L^2 with T the slab's closed-form transmittance: the disc
  estimate averaged over interior points matches E0 per channel, and is
  zero for the other side of the surface;
* the fixed-point disc sum equals the plain double sum of the fluxes in
  the disc divided by pi r^2, to rounding.

RGB textures: a texel is reflectance B at 450 nm, G at 550 nm, R at
650 nm, linear in between and constant outside.  With the three fixed
wavelengths 650/550/450 nm each image channel equals a grey render with
that channel's reflectance, bit for bit; in spectral mode the per-path
radiance is proportional to the interpolated reflectance.
"""
import math

import numpy as np
import pytest

import oracle as orc
import scenegen as sg


# ---------------------------------------------------------------- deposits

def _cells(scene, recs):
    r = scene.receiver
    sx = np.float32(r.wc) / np.float32(r.ext_u)
    sy = np.float32(r.hc) / np.float32(r.ext_v)
    ix = np.floor((recs["pos"][:, 0] - np.float32(r.x0)) * sx).astype(np.int64)
    iy = np.floor((recs["pos"][:, 1] - np.float32(r.y0)) * sy).astype(np.int64)
    ix = np.minimum(ix, r.wc - 1)
    iy = np.minimum(iy, r.hc - 1)
    return ix, iy


def test_receiver_deposits_equal_the_receiver_map():
    c = sg.config1()
    osc = orc.OracleScene(c["scene"])
    n = 1 << 15
    recs, st = orc.pm_trace(osc, n, c["max_depth"], c["wavelengths"], c["photon_seed"])
    _, msum, cnt, st2 = orc.trace_photons(osc, n, c["max_depth"], c["wavelengths"], c["photon_seed"])
    assert len(recs) == st2["deposited"][1] == st["deposited"][1]
    assert np.all(np.diff(recs["photon"].astype(np.int64)) > 0)     # photon order
    ix, iy = _cells(c["scene"], recs)
    m = np.zeros_like(msum)
    k = np.zeros_like(cnt)
    for x, y, ch, phi in zip(ix, iy, recs["channel"], recs["phi"]):
        m[y, x, ch] += float(phi)
        k[y, x, ch] += 1
    assert np.array_equal(m, msum) and np.array_equal(k, cnt)


def test_clutter_records_are_the_photons_landing_elsewhere():
    c = sg.config3(tri_scale=0.03, w=8, h=8)
    osc = orc.OracleScene(c["scene"])
    n = 1 << 14
    recs, st = orc.pm_trace(osc, n, c["max_depth"], c["wavelengths"], c["photon_seed"])
    _, _, _, st2 = orc.trace_photons(osc, n, c["max_depth"], c["wavelengths"], c["photon_seed"])
    moved = st2["deposited"][1] + st2["elsewhere"][1] + st2["outside"][1]
    assert st2["elsewhere"][1] > 20                  # caustics on the clutter
    assert len(recs) == moved == st["deposited"][1]
    assert st["elsewhere"][1] == 0 and st["outside"][1] == 0
    flux = st2["deposited"][0] + st2["elsewhere"][0] + st2["outside"][0]
    assert st["deposited"][0] == pytest.approx(flux, rel=1e-12)
    for k in ("direct", "escaped", "absorbed", "truncated", "lost"):
        assert st[k] == st2[k], k


# ---------------------------------------------------------------- density estimate

def test_disc_estimate_matches_uniform_irradiance_under_a_slab():
    n_glass = 1.5
    scene = sg.slab_stack([((2.0, 2.0, 0.2), 0.6, sg.glass(n_glass))], aperture=0.35, ext=2.0)
    wl = sg.Wavelengths(sg.WL_FIXED, 3, (650.0, 550.0, 450.0))
    recs, st = orc.pm_trace(orc.OracleScene(scene), 1 << 16, 32, wl, 3)
    R = ((n_glass - 1.0) / (n_glass + 1.0)) ** 2
    T = (1.0 - R) / (1.0 + R)                      # clear slab, all inter-reflections
    L = 1.0e4                                      # light height above the receiver plane
    E0 = T * 1.0 / (L * L)
    r = 0.03
    up = np.array([0.0, 0.0, 1.0], np.float32)
    pts = [(x, y) for x in np.arange(-0.18, 0.19, 0.06) for y in np.arange(-0.18, 0.19, 0.06)]
    for ch in range(3):
        est = np.array([orc.pm_gather(recs, r, np.array([x, y, 0.0], np.float32), up, ch) for x, y in pts])
        # photons per disc ~ N/3 * (r / 0.35)^2; relative sd of the mean over discs
        per = len(recs) / 3 * (r / 0.35) ** 2
        tol = 4.0 / math.sqrt(per * len(pts))
        assert abs(est.mean() / E0 - 1.0) < tol, (ch, est.mean() / E0, tol)
        below = orc.pm_gather(recs, r, np.array([0.0, 0.0, 0.0], np.float32), -up, ch)
        assert below == 0.0


def test_fixed_point_sum_equals_plain_sum():
    c = sg.config1()
    recs, _ = orc.pm_trace(orc.OracleScene(c["scene"]), 1 << 14, c["max_depth"], c["wavelengths"], c["photon_seed"])
    rng = np.random.default_rng(5)
    checked = 0
    for k in rng.choice(len(recs), 40, replace=False):
        P = recs["pos"][k] + np.array([0.01, -0.02, 0.0], np.float32)
        N = recs["nrm"][k]
        ch = int(recs["channel"][k])
        for r in (0.02, 0.1):
            d = recs["pos"].astype(np.float64) - P.astype(np.float64)
            inside = ((d * d).sum(1) < r * r) & (recs["channel"] == ch) & ((recs["nrm"] @ N) > 0)
            want = recs["phi"][inside].astype(np.float64).sum() / (math.pi * r * r)
            got = orc.pm_gather(recs, r, P, N, ch)
            assert got == pytest.approx(want, rel=2e-6, abs=1e-30)
            checked += inside.sum() > 0
    assert checked > 40
    # the scale leaves room for the whole map
    s = orc.pm_scale(recs)
    q = np.rint(recs["phi"].astype(np.float64) * s)
    assert q.sum() <= 2.0 ** 62 and q.sum() > 2.0 ** 60


def test_render_with_general_map_matches_receiver_map_on_the_plane():
    """On the tiny scene every caustic photon lands on the plane, so both
    maps estimate the same irradiance: the images agree in the mean."""
    c = sg.config1()
    c["camera"] = sg.look_at((0.0, -7.0, 5.0), (0.0, 0.0, 0.8), (0, 0, 1), 40.0, 32, 32)
    osc = orc.OracleScene(c["scene"])
    recs, _ = orc.pm_trace(osc, 1 << 16, c["max_depth"], c["wavelengths"], c["photon_seed"])
    _, msum, _, _ = orc.trace_photons(osc, 1 << 16, c["max_depth"], c["wavelengths"], c["photon_seed"])
    a = orc.render_pm(osc, c["camera"], 2, c["max_depth"], c["wavelengths"], 7, recs, 0.05)["rgb"]
    b = orc.render(osc, c["camera"], 2, c["max_depth"], c["wavelengths"], 7, caustic_map=msum.astype(np.float32))["rgb"]
    assert a.mean() == pytest.approx(b.mean(), rel=0.02)


# ---------------------------------------------------------------- RGB albedo

def test_rgb_channels_equal_grey_renders():
    rho = (0.8, 0.6, 0.1)
    wl = sg.Wavelengths(sg.WL_FIXED, 3, (650.0, 550.0, 450.0))
    s_rgb, cam = sg.plane_only(rgb=np.full((4, 4, 3), rho, np.float32), w=16, h=16)
    a = orc.render(orc.OracleScene(s_rgb), cam, 2, 3, wl, 11)
    hit = a["obj"] == 1
    assert hit.mean() > 0.5
    grey = ((np.float32(0.8) + np.float32(0.6)) + np.float32(0.1)) / np.float32(3)   # the mean, not G
    assert np.all(a["albedo"][hit] == grey)
    for ch, v in enumerate(rho):
        s_g, _ = sg.plane_only(albedo=v, w=16, h=16)
        g = orc.render(orc.OracleScene(s_g), cam, 2, 3, wl, 11)
        assert np.array_equal(a["rgb"][..., ch], g["rgb"][..., ch]), ch


def test_rgb_spectral_reflectance_is_piecewise_linear():
    rho = (0.9, 0.4, 0.1)          # R, G, B
    wl = sg.Wavelengths(sg.WL_UNIFORM, 1, (550.0,), 380.0, 720.0, 8)
    s_rgb, cam = sg.plane_only(rgb=np.full((2, 2, 3), rho, np.float32), w=8, h=8)
    s_w, _ = sg.plane_only(albedo=1.0, w=8, h=8)
    pix = np.arange(64, dtype=np.uint32)
    L, lam = orc.path_samples(orc.OracleScene(s_rgb), cam, 4, 1, wl, 3, pix)
    L1, lam1 = orc.path_samples(orc.OracleScene(s_w), cam, 4, 1, wl, 3, pix)
    assert np.array_equal(lam, lam1)
    ok = L1 > 0
    assert ok.mean() > 0.7          # the rest of the film sees no plane
    r, g, b = rho
    lv = lam[ok].astype(np.float64)
    want = np.where(lv <= 450, b, np.where(lv >= 650, r, np.where(lv < 550, b + (g - b) * (lv - 450) / 100,
                                                                   g + (r - g) * (lv - 550) / 100)))
    assert np.allclose(L[ok] / L1[ok], want, rtol=2e-6)
