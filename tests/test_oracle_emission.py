"""Pins of three oracle parts that the scenes' paths depend on and that the
other pins leave open:

* the Lambert bounce at a diffuse camera vertex: Duff et al.'s orthonormal
  frame (JCGT 6(1), 2017) and the cosine-weighted direction built in it;
* the weight of a photon aimed at several overlapping target cones: the
  light's power into all cones over the number of cones that contain its
  direction (the exact density of the cone mixture);
* photons emitted by an area light: a uniform point y on the emitter, the
  cone construction from y, and the flux factor Le * A * cos(theta_y).

Each is checked against something the oracle does not compute: frame
identities, the known distribution of cosine-weighted directions, a
two-bounce radiance integral evaluated here by quadrature, solid angles of
spherical caps and of their unions, and the solid angle of a square seen
from a point (Van Oosterom and Strackee, IEEE Trans. Biomed. Eng. 30(2),
1983).  Planted mistakes (a dropped mixture weight, a containment test on
the wrong quantity, a missing cosine or area factor, a uniform instead of
a cosine bounce, a disc radius without the square root, a frame built
without Duff's sign) each fail one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import scenegen as sg


def _u24(rng, shape):
    """Uniform draws as the oracle forms them: multiples of 2^-24 in [0, 1)."""
    return (rng.integers(0, 1 << 24, size=shape) * 2.0 ** -24).astype(np.float32)


def _normals(rng, n):
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    special = np.array([[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, -1, 0],
                        [1e-4, 2e-4, -1], [-3e-4, 1e-4, 1], [0.6, 0.0, -0.8]], np.float64)
    special /= np.linalg.norm(special, axis=1, keepdims=True)
    return np.concatenate([special, v]).astype(np.float32)


# ---------------------------------------------------------------- frame

def test_duff_frame_is_orthonormal():
    """t1, t2, n are unit, pairwise orthogonal and right-handed (t1 x t2 =
    n) for every unit n, including n = -z and normals just off -z, where
    Duff's sign branch matters."""
    rng = np.random.default_rng(31)
    for n in _normals(rng, 4000):
        t1, t2 = (x.astype(np.float64) for x in oracle.onb(n))
        nn = n.astype(np.float64)
        for a in (t1, t2):
            assert abs(np.dot(a, a) - 1.0) < 2e-6
            assert abs(np.dot(a, nn)) < 2e-6
        assert abs(np.dot(t1, t2)) < 2e-6
        assert np.allclose(np.cross(t1, t2), nn, atol=3e-6)


# ---------------------------------------------------------------- bounce

def test_cosine_bounce_distribution():
    """Directions about n have density cos(theta)/pi: they lie on n's side,
    sin^2(theta) and the azimuth (measured in a frame built here) are
    uniform (Kolmogorov-Smirnov), and E[cos theta] = 2/3 (a uniform
    hemisphere gives 1/2)."""
    rng = np.random.default_rng(32)
    for n in _normals(rng, 5):
        u = _u24(rng, (20000, 2))
        d = oracle.cosine_dir(n, u).astype(np.float64)
        nn = n.astype(np.float64)
        assert np.all(np.abs(np.linalg.norm(d, axis=1) - 1) < 2e-6)
        c = d @ nn
        assert np.all(c >= 0)
        assert stats.kstest(1.0 - c * c, "uniform").pvalue > 1e-3
        a = np.array([1.0, 0.0, 0.0]) if abs(nn[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        b1 = a - np.dot(a, nn) * nn
        b1 /= np.linalg.norm(b1)
        b2 = np.cross(nn, b1)
        phi = np.arctan2(d @ b2, d @ b1) / (2 * math.pi) % 1.0
        assert stats.kstest(phi, "uniform").pvalue > 1e-3
        assert abs(c.mean() - 2.0 / 3.0) < 4 * c.std() / math.sqrt(len(c))


def _two_planes(rho_f, rho_c, h, light, L=30.0, w=16):
    b = sg.SceneBuilder()
    floor = sg.quad((-L, -L, 0), (L, -L, 0), (L, L, 0), (-L, L, 0), (0, 0, 1))
    b.add(floor, dict(type=sg.MAT_DIFFUSE, albedo_mode=sg.ALBEDO_CONST, rho_a=rho_f))
    ceil = sg.quad((-L, -L, h), (-L, L, h), (L, L, h), (L, -L, h), (0, 0, -1))
    b.add(ceil, dict(type=sg.MAT_DIFFUSE, albedo_mode=sg.ALBEDO_CONST, rho_a=rho_c))
    b.point_light(light, 1.0)
    scene = b.build(None, name="two-planes")
    cam = sg.look_at((0.0, 0.0, 0.9 * h), (0.0, 0.0, 0.0), (0, 1, 0), 0.01, w, w)
    return scene, cam


def test_second_bounce_radiance_between_two_planes():
    """Camera path through the Lambert bounce.  A floor (albedo rf) under a
    ceiling (albedo rc, height h), a point light between them, a camera
    looking straight down at the origin, max depth 2.  The pixel is the
    floor's direct term rf/pi * I cos/r^2 plus rf times the ceiling's
    direct term averaged over the bounce, whose density on the ceiling is
    h^2 / (pi r^4) for a cosine bounce (r the distance from the origin).
    That area integral is evaluated here by quadrature; the oracle's mean
    over 131k samples must agree within 4 sigma, and the value a uniform
    hemisphere bounce would give must be far outside."""
    rf, rc, h, L = 0.6, 0.9, 1.0, 30.0
    lx, ly, lz = 0.7, 0.2, 0.45
    scene, cam = _two_planes(rf, rc, h, (lx, ly, lz), L)
    osc = oracle.OracleScene(scene)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    spp = 512
    out = oracle.render(osc, cam, spp, 2, wl, 33)
    assert np.all(out["obj"] == 1)
    v = out["rgb"][..., 0].astype(np.float64).ravel()
    r1 = math.sqrt(lx * lx + ly * ly + lz * lz)
    direct = rf / math.pi * lz / r1 ** 3

    def ceiling_direct(y, x):
        dz = h - lz
        d2 = (x - lx) ** 2 + (y - ly) ** 2 + dz * dz
        return rc / math.pi * dz / d2 ** 1.5

    def cos_pdf(y, x):
        return h * h / (math.pi * (x * x + y * y + h * h) ** 2)

    def uni_pdf(y, x):
        return h / (2 * math.pi * (x * x + y * y + h * h) ** 1.5)

    opts = dict(epsabs=1e-12, epsrel=1e-10)
    e_cos = integrate.dblquad(lambda y, x: ceiling_direct(y, x) * cos_pdf(y, x), -L, L, -L, L, **opts)[0]
    e_uni = integrate.dblquad(lambda y, x: ceiling_direct(y, x) * uni_pdf(y, x), -L, L, -L, L, **opts)[0]
    expect = direct + rf * e_cos
    other = direct + rf * e_uni
    # pixel values are means over spp samples, the pixels independent
    sig = v.std() / math.sqrt(len(v))
    assert abs(v.mean() - expect) < 4 * sig + 1e-6 * expect, (v.mean(), expect, sig)
    assert abs(other - expect) > 20 * sig


# ---------------------------------------------------------------- photon cones

def _cap(dist, r):
    """Solid angle 2 pi (1 - cos theta) of a sphere of radius r at distance dist."""
    return 2 * math.pi * (1 - math.sqrt(1 - (r / dist) ** 2))


def _union_two_caps(a1, t1, a2, t2):
    """Solid angle of the union of two caps (unit axes a1, a2, half-angles
    t1, t2): cap 2 plus the part of cap 1 outside cap 2, integrated over
    cap 1 in polar coordinates about a1; at polar angle th the directions
    inside cap 2 form an arc of azimuths |phi| <= arccos((cos t2 - cos th
    cos b) / (sin th sin b)), b the angle between the axes."""
    b = math.acos(max(-1.0, min(1.0, float(np.dot(a1, a2)))))

    def outside(th):
        if th == 0.0:
            inside = 2 * math.pi if b <= t2 else 0.0
        else:
            x = (math.cos(t2) - math.cos(th) * math.cos(b)) / (math.sin(th) * math.sin(b))
            inside = 2 * math.acos(max(-1.0, min(1.0, x)))
        return (2 * math.pi - inside) * math.sin(th)

    return 2 * math.pi * (1 - math.cos(t2)) + integrate.quad(outside, 0.0, t1, epsabs=1e-13, limit=400)[0]


def _cone_scene(light, spheres, intensity=2.0):
    b = sg.SceneBuilder()
    plane = sg.quad((-20, -20, 0), (20, -20, 0), (20, 20, 0), (-20, 20, 0), (0, 0, 1))
    recv = b.add(plane, dict(type=sg.MAT_DIFFUSE, albedo_mode=sg.ALBEDO_CONST, rho_a=0.5))
    b.point_light(light, intensity)
    scene = b.build(sg.Receiver(recv, 16, 16, -20.0, -20.0, 40.0, 40.0), name="cones")
    scene.targets_obj = np.ones(len(spheres), np.uint32)
    scene.targets_sphere = np.ascontiguousarray(np.array(spheres, np.float32))
    return scene


def _total_flux(scene, n, seed, batches=1):
    osc = oracle.OracleScene(scene)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    tot = []
    for k in range(batches):
        p0, p1 = n * k // batches, n * (k + 1) // batches
        _, _, _, st = oracle.trace_photons(osc, n, 4, wl, seed, p0=p0, p1=p1)
        assert sum(v[1] for key, v in st.items() if key != "segments") == p1 - p0
        tot.append(sum(v[0] for key, v in st.items() if key != "segments"))
    return np.array(tot)


def test_coincident_cones_carry_one_cone_of_flux():
    """Two identical target spheres: every direction lies in both cones,
    so each photon is weighted by 1/2 and the pass carries I * Omega of a
    single cone, not twice that."""
    L = np.array([0.3, -0.2, 5.0])
    c, r = np.array([0.5, 0.4, 1.0]), 0.6
    s = _cone_scene(L, [[*c, r], [*c, r]])
    om = _cap(float(np.linalg.norm(c - L)), r)
    tot = _total_flux(s, 4096, 41)[0]
    assert abs(tot / (2.0 * om) - 1) < 2e-6


@pytest.mark.parametrize("s1,s2", [([1.5, 0.0, 1.0, 0.4], [-1.2, 0.8, 0.5, 0.3]),
                                   ([0.2, 0.1, 1.0, 0.4], [-0.1, 0.0, 9.0, 0.5])],
                         ids=["side-by-side", "opposite"])
def test_disjoint_cones_add(s1, s2):
    """Two target spheres whose cones do not meet, side by side or on
    opposite sides of the light (the axis of one then lies on the line of
    the other's directions, reversed): every photon is in one cone only
    and the pass carries I * (Omega1 + Omega2)."""
    L = np.array([0.0, 0.0, 5.0])
    s = _cone_scene(L, [s1, s2])
    om = sum(_cap(float(np.linalg.norm(np.array(q[:3]) - L)), q[3]) for q in (s1, s2))
    tot = _total_flux(s, 4096, 42)[0]
    assert abs(tot / (2.0 * om) - 1) < 2e-6


def test_overlapping_cones_give_the_union():
    """Two partly overlapping cones: the mixture-weighted flux estimates I
    times the solid angle of their union, integrated here; the standard
    error follows from the share of photons in the overlap (weight 1/2)
    and is checked to 5 sigma.  Dropping the weight, or testing
    containment on sin(theta) instead of sin^2(theta), misses by far more."""
    L = np.array([0.0, 0.0, 5.0])
    s1, s2 = np.array([0.0, 0.0, 1.0, 0.8]), np.array([0.9, 0.3, 1.2, 0.7])
    caps = []
    for q in (s1, s2):
        ax = q[:3] - L
        dist = float(np.linalg.norm(ax))
        caps.append((ax / dist, math.asin(q[3] / dist), _cap(dist, q[3])))
    union = _union_two_caps(caps[0][0], caps[0][1], caps[1][0], caps[1][1])
    om_sum = caps[0][2] + caps[1][2]
    inter = om_sum - union
    assert 0.2 * min(caps[0][2], caps[1][2]) < inter < 0.8 * min(caps[0][2], caps[1][2])
    n = 1 << 18
    tot = _total_flux(_cone_scene(L, [s1, s2]), n, 43)[0] / 2.0
    # per photon: weight om_sum / n in one cone, om_sum / (2 n) in both;
    # the sampled share of "both" is 2 inter / om_sum
    p2 = 2 * inter / om_sum
    sig = math.sqrt(n * p2 * (1 - p2)) * om_sum / (2 * n)
    assert abs(tot - union) < 5 * sig, (tot, union, sig)


def test_three_overlapping_cones_give_the_union():
    """Three cones with a region common to all (weights 1, 1/2, 1/3): the
    flux estimates the solid angle of their union, here integrated as an
    indicator over a fine grid of directions in double precision."""
    L = np.array([0.0, 0.0, 6.0])
    sph = np.array([[0.0, 0.0, 1.0, 0.9], [0.7, 0.0, 1.1, 0.8], [0.3, 0.6, 0.9, 0.7]])
    ax, ct = [], []
    for q in sph:
        v = q[:3] - L
        dist = np.linalg.norm(v)
        ax.append(v / dist)
        ct.append(math.sqrt(1 - (q[3] / dist) ** 2))
    # grid over a cap about -z that holds all three cones
    cmin = 0.9
    nz, nphi = 6000, 6000
    z = 1 - (np.arange(nz) + 0.5) / nz * (1 - cmin)
    phi = (np.arange(nphi) + 0.5) / nphi * 2 * math.pi
    cover = 0
    sz = np.sqrt(1 - z * z)
    for j in range(0, nz, 500):
        zz = z[j:j + 500, None]
        ss = sz[j:j + 500, None]
        d = np.stack([ss * np.cos(phi)[None, :], ss * np.sin(phi)[None, :], -zz * np.ones_like(phi)[None, :]], -1)
        inside = np.zeros(d.shape[:2], bool)
        for a, c in zip(ax, ct):
            inside |= d @ a >= c
        cover += int(inside.sum())
    cell = 2 * math.pi * (1 - cmin) / (nz * nphi)
    union = cover * cell
    n = 1 << 18
    tot = _total_flux(_cone_scene(L, sph), n, 44, batches=8) / 2.0
    sig = tot.std(ddof=1) / math.sqrt(len(tot)) * len(tot)
    assert abs(tot.sum() - union) < 5 * sig + 2e-4 * union, (tot.sum(), union, sig)


# ---------------------------------------------------------------- area light

def _solid_angle_triangle(p, a, b, c):
    """Van Oosterom and Strackee: solid angle of triangle abc seen from p."""
    r1, r2, r3 = a - p, b - p, c - p
    l1, l2, l3 = np.linalg.norm(r1), np.linalg.norm(r2), np.linalg.norm(r3)
    num = abs(np.dot(r1, np.cross(r2, r3)))
    den = l1 * l2 * l3 + np.dot(r1, r2) * l3 + np.dot(r1, r3) * l2 + np.dot(r2, r3) * l1
    return 2 * math.atan2(num, den)


def _emitter_scene(center, side, le, sphere, point_light=None):
    b = sg.SceneBuilder()
    plane = sg.quad((-20, -20, 0), (20, -20, 0), (20, 20, 0), (-20, 20, 0), (0, 0, 1))
    recv = b.add(plane, dict(type=sg.MAT_DIFFUSE, albedo_mode=sg.ALBEDO_CONST, rho_a=0.5))
    cx, cy, cz = center
    hs = 0.5 * side
    light = sg.quad((cx - hs, cy - hs, cz), (cx - hs, cy + hs, cz), (cx + hs, cy + hs, cz), (cx + hs, cy - hs, cz),
                    (0, 0, -1))
    b.add(light, dict(type=sg.MAT_EMISSIVE, le=le))
    if point_light is not None:
        b.point_light(point_light[:3], point_light[3])
    scene = b.build(sg.Receiver(recv, 16, 16, -20.0, -20.0, 40.0, 40.0), name="emitter")
    scene.targets_obj = np.ones(1, np.uint32)
    scene.targets_sphere = np.ascontiguousarray(np.array([sphere], np.float32))
    return scene


@pytest.mark.parametrize("sphere", [[0.0, 0.0, 1.0, 0.3], [1.1, -0.6, 0.8, 0.25]])
def test_area_light_photon_flux_closed_form(sphere):
    """A downward square emitter of side s and radiance Le, one target
    sphere (centre c, radius r) below it, on its axis or off it.  Photons
    start at a uniform point y of the square with flux Le A cos(theta_y)
    times the cone's solid angle; averaged over the cone that is Le A pi
    (r/|c-y|)^2 cos(tilt), and over y it is Le pi r^2 times the solid angle
    of the square seen from c (Van Oosterom-Strackee, two triangles).  No
    photon may start behind the emitter (it would be absorbed by it) or
    outside its hemisphere."""
    side, le, H = 0.8, 3.0, 3.0
    s = _emitter_scene((0.2, 0.1, H), side, le, sphere)
    c = np.array(sphere[:3])
    hs = side / 2
    corners = [np.array([0.2 - hs, 0.1 - hs, H]), np.array([0.2 - hs, 0.1 + hs, H]),
               np.array([0.2 + hs, 0.1 + hs, H]), np.array([0.2 + hs, 0.1 - hs, H])]
    om_sq = _solid_angle_triangle(c, corners[0], corners[1], corners[2]) + \
        _solid_angle_triangle(c, corners[0], corners[2], corners[3])
    expect = le * math.pi * sphere[3] ** 2 * om_sq
    n = 1 << 18
    osc = oracle.OracleScene(s)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    tots = []
    for k in range(16):
        _, _, _, st = oracle.trace_photons(osc, n, 4, wl, 51, p0=n * k // 16, p1=n * (k + 1) // 16)
        assert st["absorbed"][1] == 0 and st["emit_dead"][1] == 0 and st["lost"][1] == 0
        tots.append(sum(v[0] for key, v in st.items() if key != "segments"))
    tots = np.array(tots)
    sig = tots.std(ddof=1) * math.sqrt(len(tots))
    assert abs(tots.sum() - expect) < 5 * sig + 1e-6 * expect, (tots.sum(), expect, sig)
    # without the cosine the average would rise by the mean of 1/cos(theta_y)
    # over the cone: make sure the test can tell
    assert sig < 0.002 * expect


def test_area_and_point_light_share_photons_by_entry():
    """With a point light and an emitter in one scene a photon picks either
    with probability 1/2 and carries twice its light's flux: the pass
    carries the sum of the two single-light closed forms."""
    side, le, H = 0.6, 2.0, 3.0
    sphere = [0.0, 0.0, 1.0, 0.3]
    pl = (1.0, 0.5, 4.0, 1.5)
    s = _emitter_scene((0.0, 0.0, H), side, le, sphere, point_light=pl)
    c = np.array(sphere[:3])
    hs = side / 2
    cs = [np.array([-hs, -hs, H]), np.array([-hs, hs, H]), np.array([hs, hs, H]), np.array([hs, -hs, H])]
    om_sq = _solid_angle_triangle(c, cs[0], cs[1], cs[2]) + _solid_angle_triangle(c, cs[0], cs[2], cs[3])
    expect = le * math.pi * sphere[3] ** 2 * om_sq + pl[3] * _cap(float(np.linalg.norm(c - np.array(pl[:3]))),
                                                                   sphere[3])
    n = 1 << 18
    osc = oracle.OracleScene(s)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    tots = []
    for k in range(16):
        _, _, _, st = oracle.trace_photons(osc, n, 4, wl, 52, p0=n * k // 16, p1=n * (k + 1) // 16)
        tots.append(sum(v[0] for key, v in st.items() if key != "segments"))
    tots = np.array(tots)
    sig = tots.std(ddof=1) * math.sqrt(len(tots))
    assert abs(tots.sum() - expect) < 5 * sig, (tots.sum(), expect, sig)
