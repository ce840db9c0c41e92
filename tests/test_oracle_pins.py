"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks one part of the oracle against a published value, a closed
form, an independent textbook routine, brute force, or an invariant, chosen
so that a plausible slip (a dropped term, a wrong sign or index, a swapped
operand) fails.  Everything here runs on the CPU.
"""
import math
import os

import numpy as np
import pytest

import oracle
import scenegen as sg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


# ------------------------------------------------------------ generator

def test_philox_known_answers():
    """Philox4x32-10 reproduces the published known-answer vectors."""
    for r in _rows("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in r]
        out = oracle.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_sincos2pi_accuracy_and_quadrants():
    us = np.concatenate([np.linspace(0, 1, 20001, endpoint=False), [0.25, 0.5, 0.75, 1 - 2 ** -24]])
    err = 0.0
    for u in us:
        s, c = oracle.sincos2pi(float(np.float32(u)))
        uu = float(np.float32(u))
        err = max(err, abs(s - math.sin(2 * math.pi * uu)), abs(c - math.cos(2 * math.pi * uu)))
    assert err < 4e-7
    assert oracle.sincos2pi(0.0) == (0.0, 1.0)
    assert oracle.sincos2pi(0.25) == (1.0, -0.0) or oracle.sincos2pi(0.25) == (1.0, 0.0)
    assert oracle.sincos2pi(0.5)[1] == -1.0
    assert oracle.sincos2pi(0.75)[0] == -1.0


# ------------------------------------------------------------ closest hit

def _random_rays(rng, n, center, spread, targets=None):
    O = (center + rng.normal(size=(n, 3)) * spread).astype(np.float32)
    if targets is None:
        D = rng.normal(size=(n, 3))
    else:
        D = targets[rng.integers(0, len(targets), size=n)] - O
    D = (D / np.linalg.norm(D, axis=1, keepdims=True)).astype(np.float32)
    return O, D


def _mt_fp64(V, I, o, d):
    """Independent textbook ray/triangle test (Moller-Trumbore) in float64:
    nearest t and triangle over all triangles."""
    a, b, c = V[I[:, 0]].astype(np.float64), V[I[:, 1]].astype(np.float64), V[I[:, 2]].astype(np.float64)
    e1, e2 = b - a, c - a
    p = np.cross(d, e2)
    det = np.einsum("ij,ij->i", e1, p)
    with np.errstate(divide="ignore", invalid="ignore"):
        inv = 1.0 / det
        tv = o - a
        u = np.einsum("ij,ij->i", tv, p) * inv
        q = np.cross(tv, e1)
        v = (q @ d) * inv
        t = np.einsum("ij,ij->i", e2, q) * inv
    ok = (np.abs(det) > 0) & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
    t = np.where(ok, t, np.inf)
    k = int(np.argmin(t))
    return t[k], k, u[k], v[k]


@pytest.mark.parametrize("which", ["ico2", "soup", "box"])
def test_bvh_equals_brute_force(which):
    """The oracle's BVH returns the brute-force (t, prim, u, v) bit for bit,
    including rays aimed exactly at vertices and edge midpoints."""
    rng = np.random.default_rng(7)
    b = sg.SceneBuilder()
    if which == "ico2":
        b.add(sg.icosphere(2, 1.0, (0, 0, 0)), sg.GLASS_C1)
    elif which == "box":
        b.add(sg.box((1.0, 2.0, 0.5)), dict(type=sg.MAT_DIFFUSE, rho_a=0.5))
    else:
        V = rng.uniform(-1, 1, size=(300, 3))
        I = np.arange(300).reshape(100, 3)
        b.add(sg.Mesh(V, I, np.tile([0, 0, 1.0], (300, 1))), dict(type=sg.MAT_DIFFUSE, rho_a=0.5))
    scene = b.build(None)
    osc = oracle.OracleScene(scene)
    V, I = scene.V, scene.I
    mids = np.concatenate([V, 0.5 * (V[I[:, 0]] + V[I[:, 1]]), (V[I[:, 0]] + V[I[:, 1]] + V[I[:, 2]]) / 3])
    O1, D1 = _random_rays(rng, 4000, np.zeros(3), 3.0)
    O2, D2 = _random_rays(rng, 4000, np.zeros(3), 3.0, targets=mids.astype(np.float64))
    O3 = np.zeros((500, 3), np.float32)   # from the inside
    D3 = rng.normal(size=(500, 3))
    D3 = (D3 / np.linalg.norm(D3, axis=1, keepdims=True)).astype(np.float32)
    O = np.concatenate([O1, O2, O3])
    D = np.concatenate([D1, D2, D3])
    tb, pb, ub, vb = oracle.closest(osc, O, D, brute=True)
    tv, pv, uv, vv = oracle.closest(osc, O, D)
    assert np.array_equal(pb, pv)
    assert np.array_equal(tb.view(np.uint32), tv.view(np.uint32))
    assert np.array_equal(ub.view(np.uint32), uv.view(np.uint32))
    assert np.array_equal(vb.view(np.uint32), vv.view(np.uint32))
    # against an independent float64 test on rays that are not grazing an edge
    checked = 0
    for i in range(0, len(O), 37):
        t64, k64, u64, v64 = _mt_fp64(V, I, O[i].astype(np.float64), D[i].astype(np.float64))
        if not np.isfinite(t64):
            if pb[i] != 0xFFFFFFFF:
                # a hit the float64 test missed must lie on an edge
                bu, bv = float(ub[i]), float(vb[i])
                assert min(bu, bv, 1 - bu - bv) < 1e-4
            continue
        if min(u64, v64, 1 - u64 - v64) < 1e-4:
            continue
        assert pb[i] != 0xFFFFFFFF
        if float(tb[i]) < t64 - 1e-5 * max(1.0, t64):
            # a nearer hit that float64 rejects must graze that triangle's edge
            bu, bv = float(ub[i]), float(vb[i])
            assert min(bu, bv, 1 - bu - bv) < 1e-4
            continue
        assert abs(float(tb[i]) - t64) <= 1e-5 * max(1.0, t64)
        if abs(float(tb[i]) - t64) > 0 and pb[i] != k64:
            # a different triangle only when it lies at the same distance
            t_other = _mt_fp64(V, I[[pb[i]]], O[i].astype(np.float64), D[i].astype(np.float64))[0]
            assert abs(t_other - t64) <= 1e-5 * max(1.0, t64)
        checked += 1
    assert checked > 50


def test_watertight_closed_mesh():
    """Rays from inside a closed mesh always find a surface, also when aimed
    exactly at shared vertices and edges."""
    scene = sg.SceneBuilder()
    scene.add(sg.icosphere(3, 1.0, (0.1, -0.2, 0.05)), sg.GLASS_C1)
    s = scene.build(None)
    osc = oracle.OracleScene(s)
    V, I = s.V.astype(np.float64), s.I
    targets = np.concatenate([V, 0.5 * (V[I[:, 0]] + V[I[:, 1]]), 0.5 * (V[I[:, 1]] + V[I[:, 2]])])
    O = np.tile(np.array([0.1, -0.2, 0.05], np.float32), (len(targets), 1))
    D = targets - O
    D = (D / np.linalg.norm(D, axis=1, keepdims=True)).astype(np.float32)
    t, p, _, _ = oracle.closest(osc, O, D)
    assert (p != 0xFFFFFFFF).all()
    occ = oracle.any_hit(osc, O, D, np.full(len(O), 10.0, np.float32))
    assert occ.all()


def test_any_hit_matches_closest():
    c = sg.config1(level=2)
    osc = oracle.OracleScene(c["scene"])
    rng = np.random.default_rng(3)
    O, D = _random_rays(rng, 3000, np.array([0, 0, 1.5]), 2.0)
    t, p, _, _ = oracle.closest(osc, O, D)
    tmax = rng.uniform(0.1, 6.0, size=len(O)).astype(np.float32)
    occ = oracle.any_hit(osc, O, D, tmax)
    occ_b = oracle.any_hit(osc, O, D, tmax, brute=True)
    assert np.array_equal(occ, occ_b)
    assert np.array_equal(occ, (p != 0xFFFFFFFF) & (t < tmax))
    # excluding the nearest triangle can only remove that one occluder
    occ_x = oracle.any_hit(osc, O, D, tmax, excl=p)
    assert not (occ_x & ~occ).any()


# ------------------------------------------------------------ camera, depth, mask

def test_depth_on_plane_closed_form():
    """Depth of the pixel-centre ray on z = 0 equals -o_z/d_z (d from the
    camera definition evaluated in float64); normalised depth is t/10 capped
    at 1; the normal is +z in world space and its camera-space image is the
    camera basis applied to +z."""
    scene, cam = sg.plane_only(w=24, h=16)
    osc = oracle.OracleScene(scene)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    out = oracle.render(osc, cam, 1, 1, wl, 5)
    eye = cam.eye.astype(np.float64)
    R = cam.right.astype(np.float64)
    U = cam.up.astype(np.float64)
    F = cam.fwd.astype(np.float64)
    for y in range(cam.h):
        for x in range(cam.w):
            sx = 2 * (x + 0.5) / cam.w - 1
            sy = 1 - 2 * (y + 0.5) / cam.h
            d = F + sx * R + sy * U
            d /= np.linalg.norm(d)
            if d[2] >= 0:
                assert out["obj"][y, x] == 0
                continue
            t = -eye[2] / d[2]
            P = eye + t * d
            if abs(P[0]) > 4 or abs(P[1]) > 4:
                continue
            assert out["obj"][y, x] == 1
            assert abs(out["depth"][y, x] - t) <= 2e-6 * t
            assert abs(out["depthn"][y, x] - min(t / 10, 1)) <= 2e-6
    n = out["normal"][out["obj"] == 1]
    assert np.all(n == np.array([0, 0, 1], np.float32))
    Rh, Uh, Fh = R / np.linalg.norm(R), U / np.linalg.norm(U), F / np.linalg.norm(F)
    nc = np.array([Rh[2], Uh[2], -Fh[2]])
    assert np.allclose(out["normal_cam"][out["obj"] == 1], nc, atol=1e-6)


def test_mask_sphere_silhouette():
    """Glass pixels of the c1 icosphere (level 3) lie inside the silhouette
    cone of its circumsphere (radius 1) and include every pixel whose centre
    ray passes within its insphere (radius = distance from centre to the
    nearest face plane)."""
    c = sg.config1()
    s, cam = c["scene"], c["camera"]
    osc = oracle.OracleScene(s)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    out = oracle.render(osc, cam, 1, 1, wl, 1)
    V = s.V.astype(np.float64)
    I = s.I[s.tri_obj == 2]
    ctr = np.array([0, 0, 1.5])
    a, b, cc = V[I[:, 0]], V[I[:, 1]], V[I[:, 2]]
    n = np.cross(b - a, cc - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    r_in = float(np.min(np.einsum("ij,ij->i", a - ctr, n)))
    assert 0.99 < r_in < 1.0
    eye = cam.eye.astype(np.float64)
    inside = outside = 0
    for y in range(cam.h):
        for x in range(cam.w):
            o, d = oracle.camera_ray(cam, x, y)
            d = d.astype(np.float64)
            w = ctr - eye
            dist = np.linalg.norm(w - np.dot(w, d) * d)
            glass = out["trans"][y, x] == 1
            if glass:
                assert dist <= 1.0 + 1e-6
                inside += 1
            if dist < r_in - 1e-6:
                assert glass
                outside += 1
    assert inside > 500 and outside > 500


# ------------------------------------------------------------ optics

def _optics():
    rows = _rows("optics_closed_forms.txt")
    return [(float(r[0]), float(r[1]), float(r[2]), float(r[3]), float(r[4]), float(r[5])) for r in rows]


def _flat_hit(theta, entering=True, phi=0.3):
    """Direction at incidence angle theta onto z = 0 (normal +z)."""
    s, c = math.sin(theta), math.cos(theta)
    d = np.array([s * math.cos(phi), s * math.sin(phi), -c if entering else c], np.float64)
    return d.astype(np.float32)


@pytest.mark.parametrize("lam,n,R0,thc,brew,f", _optics())
def test_snell_and_cauchy(lam, n, R0, thc, brew, f):
    """Refraction obeys n1 sin(ti) = n2 sin(tt) with n from the two-term
    Cauchy law, stays in the plane of incidence, and reflection mirrors."""
    Ng = np.array([0, 0, 1], np.float32)
    P = np.zeros(3, np.float32)
    for th in np.linspace(0.01, 1.5, 40):
        d = _flat_hit(th)
        ok, o, t, refl, R = oracle.dielectric(d, Ng, Ng, P, lam, 1.5, 0.0042, 1.0)
        assert ok and not refl
        d64, t64 = d.astype(np.float64), t.astype(np.float64)
        si = np.linalg.norm(np.cross(d64, [0, 0, 1]))
        st = np.linalg.norm(np.cross(t64, [0, 0, 1]))
        assert abs(si / st - n) < 3e-6 * n
        assert abs(np.dot(t64, np.cross(d64, [0, 0, 1]))) < 1e-6
        assert t[2] < 0 and o[2] < 0
        ok, o, r, refl, R = oracle.dielectric(d, Ng, Ng, P, lam, 1.5, 0.0042, 0.0)
        assert ok and refl
        assert np.allclose(r, [d[0], d[1], -d[2]], atol=2e-7) and o[2] > 0


@pytest.mark.parametrize("lam,n,R0,thc,brew,f", _optics())
def test_total_internal_reflection(lam, n, R0, thc, brew, f):
    """From inside the glass, every ray beyond the critical angle asin(1/n)
    reflects (even when u is just below 1); below it, u = 1 refracts."""
    Ng = np.array([0, 0, 1], np.float32)   # outward normal; ray travels +z from inside
    P = np.zeros(3, np.float32)
    tc = math.radians(thc)
    for th in (tc + 1e-4, tc + 0.05, 1.2, 1.5):
        d = _flat_hit(th, entering=False)
        ok, o, r, refl, R = oracle.dielectric(d, Ng, Ng, P, lam, 1.5, 0.0042, 1.0 - 2 ** -24)
        assert ok and refl and R == 1.0
        assert o[2] < 0
    for th in (0.1, tc - 0.05, tc - 1e-4):
        d = _flat_hit(th, entering=False)
        ok, o, t, refl, R = oracle.dielectric(d, Ng, Ng, P, lam, 1.5, 0.0042, 1.0)
        assert ok and not refl and R < 1.0 and t[2] > 0


@pytest.mark.parametrize("lam,n,R0,thc,brew,f", _optics())
def test_fresnel_energy_and_special_angles(lam, n, R0, thc, brew, f):
    """R + T = 1 with T from the independent transmission coefficients;
    normal incidence gives ((n-1)/(n+1))^2; at Brewster's angle the p part
    vanishes; R is reciprocal between the two sides."""
    nf = float(np.float32(n))
    for th in np.linspace(0.0, math.radians(89.5), 60):
        ci = math.cos(th)
        st = math.sin(th) / nf
        ct = math.sqrt(1 - st * st)
        R = oracle.fresnel(1.0, nf, ci, ct)
        ts = 2 * ci / (ci + nf * ct)
        tp = 2 * ci / (ct + nf * ci)
        T = (nf * ct) / ci * (ts * ts + tp * tp) / 2
        assert abs(R + T - 1) < 1e-6
        R_back = oracle.fresnel(nf, 1.0, ct, ci)
        assert abs(R - R_back) < 1e-6
    assert abs(oracle.fresnel(1.0, nf, 1.0, 1.0) - R0) < 5e-7
    tb = math.radians(brew)
    ci, ctb = math.cos(tb), math.sqrt(1 - (math.sin(tb) / nf) ** 2)
    rs = (ci - nf * ctb) / (ci + nf * ctb)
    assert abs(oracle.fresnel(1.0, nf, ci, ctb) - 0.5 * rs * rs) < 2e-6
    # the event decision uses exactly this R
    d = _flat_hit(0.7)
    Ng = np.array([0, 0, 1], np.float32)
    ok, o, dd, refl, R = oracle.dielectric(d, Ng, Ng, np.zeros(3, np.float32), lam, 1.5, 0.0042, 0.5)
    assert ok and not refl and 0.04 < R < 0.1
    ok2, _, _, refl2, _ = oracle.dielectric(d, Ng, Ng, np.zeros(3, np.float32), lam, 1.5, 0.0042,
                                            float(np.nextafter(np.float32(R), np.float32(0))))
    assert ok2 and refl2


def test_shading_normal_fallback():
    """A shading normal facing away from the ray falls back to the
    geometric normal; the outgoing ray is always on the correct side."""
    Ng = np.array([0, 0, 1], np.float32)
    Ns = np.array([0.9, 0.0, 0.43589], np.float32)
    Ns /= np.linalg.norm(Ns)
    d = _flat_hit(1.3, phi=0.0)
    for u in (0.0, 1.0):
        ok, o, out, refl, R = oracle.dielectric(d, Ng, Ns, np.zeros(3, np.float32), 550, 1.5, 0.0042, u)
        assert ok
        assert (out[2] > 0) == refl


# ------------------------------------------------------------ radiance special cases

def test_lambert_point_light_closed_form():
    """Plane + point light, no occluder, depth 1: each pixel equals
    rho/pi * I * cos(theta)/r^2 at the hit point of its jittered ray (the
    jitter is the first two outputs of the camera stream at purpose 0)."""
    scene, cam = sg.plane_only(albedo=0.8, w=20, h=20)
    osc = oracle.OracleScene(scene)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    seed = 123456789012345
    out = oracle.render(osc, cam, 1, 1, wl, seed)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    L = np.array([2.0, 3.0, 6.0])
    eye = cam.eye.astype(np.float64)
    n = 0
    for y in range(cam.h):
        for x in range(cam.w):
            r = oracle.philox([y * cam.w + x, 0, 0, 0], key)
            jx, jy = (r[0] >> 8) * 2.0 ** -24, (r[1] >> 8) * 2.0 ** -24
            sx = 2 * (x + jx) / cam.w - 1
            sy = 1 - 2 * (y + jy) / cam.h
            d = cam.fwd.astype(np.float64) + sx * cam.right.astype(np.float64) + sy * cam.up.astype(np.float64)
            d /= np.linalg.norm(d)
            if d[2] >= 0:
                continue
            P = eye + (-eye[2] / d[2]) * d
            if abs(P[0]) > 3.9 or abs(P[1]) > 3.9:
                continue
            w = L - P
            r2 = w @ w
            val = 0.8 / math.pi * 50.0 * (w[2] / math.sqrt(r2)) / r2
            assert abs(out["rgb"][y, x, 0] - val) <= 2e-5 * val
            n += 1
    assert n > 100
    # the worked value under the light's foot print at the origin
    w = L
    E = 50.0 * (w[2] / np.linalg.norm(w)) / (w @ w)
    assert abs(E - 0.87464) < 5e-5 and abs(0.8 / math.pi * E - 0.22272) < 5e-5


def test_caustic_gather_adds_rho_over_pi_E():
    """A constant caustic map of value m adds exactly rho/pi * m / A_cell to
    every receiver pixel (depth 1, no bounce)."""
    scene, _ = sg.plane_only(albedo=0.5)
    cam = sg.look_at((0.3, 0.2, 5.0), (0.3, 0.2, 0.0), (0, 1, 0), 40.0, 16, 16)
    osc = oracle.OracleScene(scene)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    m = np.full((64, 64, 1), 0.01, np.float32)
    m[:, :32] = 0.0   # left half of the receiver empty
    a = oracle.render(osc, cam, 1, 1, wl, 9)
    b = oracle.render(osc, cam, 1, 1, wl, 9, caustic_map=m)
    A_cell = (8.0 / 64) ** 2
    assert np.all(a["obj"] == 1)
    o, d = np.array(cam.eye, np.float64), None
    diff = (b["rgb"] - a["rgb"])[..., 0]
    lit = np.zeros(diff.shape, bool)
    for y in range(cam.h):
        for x in range(cam.w):
            _, d = oracle.camera_ray(cam, x, y)
            px = o[0] + (-o[2] / d[2]) * d[0]
            lit[y, x] = px > 0.0
    # pixels well inside either half (the jittered ray stays on that side)
    away = np.abs(np.arange(cam.w) - (cam.w / 2 - 0.5 - 0.3 / (5 * 0.364) * cam.w / 2)) > 1.5
    assert np.allclose(diff[:, away][lit[:, away]], 0.5 / math.pi * 0.01 / A_cell, rtol=2e-6)
    assert np.all(diff[:, away][~lit[:, away]] == 0)


def test_uniform_spectrum_is_white():
    """With wavelengths drawn uniformly, a flat-spectrum Lambert plane
    averages to the grey closed form in every channel (sensor curves
    normalised to mean 1)."""
    scene, cam = sg.plane_only(albedo=0.8, w=8, h=8)
    osc = oracle.OracleScene(scene)
    wl_u = sg.Wavelengths(sg.WL_UNIFORM, 1, (550.0,), 380.0, 720.0, 16)
    wl_f = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    u = oracle.render(osc, cam, 2048, 1, wl_u, 4)
    f = oracle.render(osc, cam, 2048, 1, wl_f, 4)
    m = u["obj"] == 1
    grey = f["rgb"][m][:, 0].mean()
    for c in range(3):
        assert abs(u["rgb"][m][:, c].mean() / grey - 1) < 0.03


def test_white_furnace_glass():
    """Inside an inward-emitting enclosure of radiance 1 every camera path
    through smooth glass carries weight 1: each pixel is exactly 1 unless
    its path is cut at max_depth."""
    scene, cam = sg.furnace("glass", w=24, h=24)
    osc = oracle.OracleScene(scene)
    wl = sg.Wavelengths(sg.WL_FIXED, 3, (650.0, 550.0, 450.0))
    out = oracle.render(osc, cam, 4, 64, wl, 11)
    v = out["rgb"] * 4
    assert np.all(np.isin(np.round(v, 5), [0, 1, 2, 3, 4]))
    assert out["rgb"].mean() >= 0.999


def test_white_furnace_diffuse():
    """A white Lambert sphere inside the same enclosure reflects radiance 1:
    next-event estimation over the emitting triangles has mean 1."""
    scene, cam = sg.furnace("diffuse", w=24, h=24)
    osc = oracle.OracleScene(scene)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    out = oracle.render(osc, cam, 16, 4, wl, 12)
    v = out["rgb"][..., 0]
    sph = out["obj"] == 1
    assert sph.sum() > 50
    # enclosure pixels away from the silhouette see the emitter directly
    near = sph.copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            near |= np.roll(np.roll(sph, dy, 0), dx, 1)
    assert np.all(v[~near] == 1.0)
    mean = v[sph].mean()
    # per-pixel variance estimated from the data; 4 sigma of the mean
    sig = v[sph].std() / math.sqrt(sph.sum())
    assert abs(mean - 1.0) < 4 * sig + 2e-3


# ------------------------------------------------------------ photons

def test_photon_energy_accounting_c1():
    """Every emitted photon ends in exactly one outcome; the flux of a
    wavelength slot sums to I * Omega with Omega = 2 pi (1 - cos theta) the
    solid angle of the target sphere seen from the light."""
    c = sg.config1()
    osc = oracle.OracleScene(c["scene"])
    N = 6000
    m, msum, cnt, st = oracle.trace_photons(osc, N, 8, c["wavelengths"], 77)
    tot_count = sum(v[1] for k, v in st.items() if k != "segments")
    assert tot_count == N
    sp = c["scene"].targets_sphere[0].astype(np.float64)
    dist2 = np.sum((sp[:3] - np.array([2.0, 3.0, 6.0])) ** 2)
    omega = 2 * math.pi * (1 - math.sqrt(1 - sp[3] ** 2 / dist2))
    tot_flux = sum(v[0] for k, v in st.items() if k != "segments")
    assert abs(tot_flux - 3 * 50.0 * omega) < 2e-5 * tot_flux
    assert abs(msum.sum() - st["deposited"][0]) < 1e-9 * msum.sum()
    assert cnt.sum() == st["deposited"][1]


def test_single_photon_map():
    """One photon through the ball lens lands in one cell with its whole
    flux I * Omega; every other cell is zero."""
    s = sg.ball_lens(2, -1.47)
    osc = oracle.OracleScene(s)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    m, msum, cnt, st = oracle.trace_photons(osc, 1, 8, wl, 5)
    d2 = 1.0e4 ** 2
    omega = 2 * math.pi * (1 - math.sqrt(1 - 0.1 ** 2 / d2))
    assert st["deposited"][1] == 1
    assert np.count_nonzero(msum) == 1 and cnt.sum() == 1
    assert abs(msum.sum() - omega) < 1e-6 * omega


@pytest.mark.slow
def test_ball_lens_focal_length():
    """A paraxial beam through the glass ball (radius 1) is brightest at the
    receiver height of the effective focal length f = n D / (4 (n - 1))
    below the centre, within 0.75% (the sweep step is 1 cm); the focus moves
    outwards with wavelength (n falls with lambda)."""
    heights = np.round(np.arange(-1.58, -1.38, 0.01), 3)
    peaks = {}
    for lam, fl in ((450.0, 1.460171), (550.0, 1.472982), (650.0, 1.480506)):
        wl = sg.Wavelengths(sg.WL_FIXED, 1, (lam,))
        best = (-1, None)
        for h in heights:
            s = sg.ball_lens(5, float(h), aperture=0.08, wc=256, ext=0.064)
            osc = oracle.OracleScene(s)
            m, msum, cnt, st = oracle.trace_photons(osc, 6000, 8, wl, 21)
            pk = msum.max()
            if pk > best[0]:
                best = (pk, h)
        peaks[lam] = -best[1]
        assert abs(-best[1] - fl) < 0.0075 * fl
    assert peaks[450.0] < peaks[550.0] < peaks[650.0]


def test_c1_caustic_peak_location():
    """The c1 ball-lens caustic peaks in the cell under the light-centre
    axis: i = 106 and j at the 95/96 row boundary (closed form: the axis
    meets z = 0 at (-2/3, -1)), holding about a tenth of the plane flux."""
    c = sg.config1()
    osc = oracle.OracleScene(c["scene"])
    m, msum, cnt, st = oracle.trace_photons(osc, 1 << 15, 8, c["wavelengths"], c["photon_seed"])
    share_expected = {0: 0.107, 1: 0.101, 2: 0.090}   # slots R, G, B (650, 550, 450 nm)
    for ch in range(3):
        j, i = np.unravel_index(np.argmax(msum[:, :, ch]), msum.shape[:2])
        assert 105 <= i <= 107 and 95 <= j <= 96, (ch, i, j)
        share = msum[j, i, ch] / msum[:, :, ch].sum()
        assert abs(share / share_expected[ch] - 1) < 0.3, (ch, share)


def test_tie_flag_tree_equals_brute_force():
    """The near-tie flag (a second distinct triangle within 1e-6 t of the
    first hit) found through the oracle's tree equals the brute-force scan
    over all triangles, on a scene built to have ties: two overlapping
    planes 2e-7 m apart above a third plane."""
    b = sg.SceneBuilder()
    dm = dict(type=sg.MAT_DIFFUSE, albedo_mode=sg.ALBEDO_CONST, rho_a=0.5)
    b.add(sg.quad((-3, -3, 0), (0.5, -3, 0), (0.5, 3, 0), (-3, 3, 0), (0, 0, 1)), dm)
    z = 2e-7
    b.add(sg.quad((-0.5, -3, z), (3, -3, z), (3, 3, z), (-0.5, 3, z), (0, 0, 1)), dm)
    b.add(sg.quad((-4, -4, -0.01), (4, -4, -0.01), (4, 4, -0.01), (-4, 4, -0.01), (0, 0, 1)), dm)
    b.add(sg.icosphere(2, 0.4, (1.0, 0.5, 0.6)), dm)
    scene = b.build(None)
    cam = sg.look_at((0.0, -3.0, 4.0), (0.0, 0.0, 0.0), (0, 0, 1), 60.0, 40, 32)
    osc = oracle.OracleScene(scene)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    a = oracle.render(osc, cam, 1, 1, wl, 3, want_tie=True)
    bf = oracle.render(osc, cam, 1, 1, wl, 3, want_tie=True, brute=True)
    assert np.array_equal(a["tie"], bf["tie"])
    assert np.array_equal(a["tri"], bf["tri"])
    assert 0 < a["tie"].sum() < a["tie"].size
