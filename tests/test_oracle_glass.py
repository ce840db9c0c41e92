"""Pins of the oracle's richer glass: Beer-Lambert absorption inside
dielectrics and nested / overlapping dielectrics resolved by priority.

Glass colour and thickness are among the scene variations the paper's
ablation lists (Sec. III-C); the method is not spelled out there, so the
oracle takes the textbook models: per-segment Beer-Lambert attenuation
exp(-sigma(lambda) t), and the nested-dielectric rules of Schmidt and Budge
(J. Graphics Tools 7(2), 2002).  What pins them here:

* exp(-x), the oracle's own arithmetic, against double-precision exp;
* the nesting rules on the cases whose answer the rules fix by hand;
* the transmittance of glass slabs at normal incidence, against the
  closed form of an incoherent multilayer (Fresnel reflectance
  ((n1 - n2) / (n1 + n2))^2 at each interface, exp(-sigma d) per pass,
  all inter-reflections summed): a plain slab, an absorbing slab at an
  interpolated wavelength, a denser slab nested inside it with higher
  priority (a real interface between the two glasses) and with lower
  priority (its faces are no interfaces at all);
* camera paths through an absorbing slab onto an emitter: every sample
  equals le * exp(-(2j + 1) sigma(lambda) d) for an integer j >= 0 (j
  internal round trips), with sigma(lambda) piecewise linear through the
  450 / 550 / 650 nm values and constant outside.
"""
import math

import numpy as np
import pytest

import oracle as orc
import scenegen as sg


# ---------------------------------------------------------------- exp(-x)

def test_exp_neg_accuracy():
    rng = np.random.default_rng(7)
    xs = np.concatenate([rng.uniform(0.0, 87.0, 4000),
                         np.exp(rng.uniform(math.log(1e-8), math.log(87.0), 4000)),
                         np.linspace(0.0, 87.0, 871)]).astype(np.float32)
    worst = 0.0
    for x in xs:
        ref = math.exp(-float(x))
        worst = max(worst, abs(orc.exp_neg(float(x)) - ref) / ref)
    assert worst < 2.5e-7, worst     # about four units of 2^-24


def test_exp_neg_special_values():
    assert orc.exp_neg(0.0) == 1.0
    assert orc.exp_neg(-3.0) == 1.0
    assert orc.exp_neg(88.0) == 0.0
    assert orc.exp_neg(1e-30) == 1.0
    assert orc.exp_neg(math.log(2.0)) == pytest.approx(0.5, rel=2.5e-7)
    # e^-(a+b) = e^-a e^-b within the rounding of both sides
    for a, b in ((0.3, 1.7), (5.0, 11.25), (40.0, 40.0)):
        assert orc.exp_neg(a + b) == pytest.approx(orc.exp_neg(a) * orc.exp_neg(b), rel=8e-7)


# ---------------------------------------------------------------- nesting rules

def _nest_scene():
    """Objects: 1 receiver (diffuse), 2 glass A (n 1.5, priority 1),
    3 glass B (n 1.9, priority 2), 4 glass C (n 1.3, priority 0),
    5 glass D (n 1.7, priority 1; ties with A, larger id wins)."""
    layers = [((1.0, 1.0, 0.4), 0.7, sg.glass(1.5, priority=1)),
              ((0.6, 0.6, 0.1), 0.7, sg.glass(1.9, priority=2)),
              ((0.5, 0.5, 0.05), 0.7, sg.glass(1.3, priority=0)),
              ((0.4, 0.4, 0.02), 0.7, sg.glass(1.7, priority=1))]
    return orc.OracleScene(sg.slab_stack(layers), use_bvh=False)


def test_media_single_object_is_plain_air_glass():
    s = _nest_scene()
    after, real, n1, n2 = orc.media_step(s, [], 2, True, 550.0)
    assert (sorted(after), real) == ([2], True)
    assert (n1, n2) == (1.0, np.float32(1.5))
    after, real, n1, n2 = orc.media_step(s, [2], 2, False, 550.0)
    assert (after, real) == ([], True)
    assert (n1, n2) == (np.float32(1.5), 1.0)
    # leaving an object the path was never recorded in: glass to air
    after, real, n1, n2 = orc.media_step(s, [], 3, False, 550.0)
    assert (after, real, n1, n2) == ([], True, np.float32(1.9), 1.0)


def test_media_nested_higher_priority_is_glass_glass_interface():
    s = _nest_scene()
    after, real, n1, n2 = orc.media_step(s, [2], 3, True, 550.0)
    assert (sorted(after), real, n1, n2) == ([2, 3], True, np.float32(1.5), np.float32(1.9))
    after, real, n1, n2 = orc.media_step(s, [3, 2], 3, False, 550.0)
    assert (after, real, n1, n2) == ([2], True, np.float32(1.9), np.float32(1.5))


def test_media_lower_priority_surfaces_are_false():
    s = _nest_scene()
    after, real, _, _ = orc.media_step(s, [2], 4, True, 550.0)     # C (prio 0) inside A (prio 1)
    assert (sorted(after), real) == ([2, 4], False)
    after, real, _, _ = orc.media_step(s, [2, 4], 4, False, 550.0)
    assert (after, real) == ([2], False)
    # overlap of A and B, leaving A inside B: B dominates, no interface
    after, real, _, _ = orc.media_step(s, [2, 3], 2, False, 550.0)
    assert (after, real) == ([3], False)
    # then leaving B: B to air
    after, real, n1, n2 = orc.media_step(s, [3], 3, False, 550.0)
    assert (after, real, n1, n2) == ([], True, np.float32(1.9), 1.0)


def test_media_priority_tie_goes_to_larger_id():
    s = _nest_scene()
    after, real, n1, n2 = orc.media_step(s, [2], 5, True, 550.0)   # D (id 5) ties with A (id 2)
    assert (sorted(after), real, n1, n2) == ([2, 5], True, np.float32(1.5), np.float32(1.7))
    after, real, _, _ = orc.media_step(s, [5], 2, True, 550.0)
    assert (sorted(after), real) == ([2, 5], False)


def test_media_capacity():
    s = _nest_scene()
    # full set {A, B, C, D}: adding is a no-op for members
    after, _, _, _ = orc.media_step(s, [2, 3, 4, 5], 4, True, 550.0)
    assert sorted(after) == [2, 3, 4, 5]
    # a fifth medium can only be the receiver id here, which is not glass:
    # the call itself rejects sets above capacity
    with pytest.raises(ValueError):
        orc.media_step(s, [2, 3, 4, 5, 2], 3, True, 550.0)
    # at capacity, the lowest-priority member (C) gives way to a higher one
    after, real, _, _ = orc.media_step(s, [2, 4, 5, 3], 3, False, 550.0)
    assert (sorted(after), real) == ([2, 4, 5], True)


def test_media_indices_follow_dispersion():
    layers = [((1.0, 1.0, 0.4), 0.7, sg.glass(1.5, 0.0042, priority=1)),
              ((0.6, 0.6, 0.1), 0.7, sg.glass(1.6, 0.01, priority=2))]
    s = orc.OracleScene(sg.slab_stack(layers), use_bvh=False)
    for lam in (450.0, 550.0, 650.0):
        l = np.float32(lam) * np.float32(0.001)
        na = np.float32(1.5) + np.float32(0.0042) / (l * l)
        nb = np.float32(1.6) + np.float32(0.01) / (l * l)
        _, real, n1, n2 = orc.media_step(s, [2], 3, True, lam)
        assert real and (n1, n2) == (na, nb)


# ---------------------------------------------------------------- slab transmittance

def _fresnel0(n1, n2):
    return ((n1 - n2) / (n1 + n2)) ** 2


def _interface(n1, n2):
    r = _fresnel0(n1, n2)
    return (r, r, 1.0 - r)


def _layer(tau):
    return (0.0, 0.0, tau)


def _add(a, b):
    """Adding method for incoherent layers: (R from above, R from below, T)."""
    ra, rab, ta = a
    rb, rbb, tb = b
    den = 1.0 - rab * rb
    return (ra + ta * ta * rb / den, rbb + tb * tb * rab / den, ta * tb / den)


def _stack(*elems):
    acc = elems[0]
    for e in elems[1:]:
        acc = _add(acc, e)
    return acc[2]


def _transmittance(layers, lam, n_photons=1 << 17, max_depth=32, seed=11):
    scene = sg.slab_stack(layers)
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (lam,))
    osc = orc.OracleScene(scene)
    _, _, _, st = orc.trace_photons(osc, n_photons, max_depth, wl, seed)
    # total emitted flux: the same photons with every sigma set to zero
    clear = [(sz, zc, dict(m, sigma=np.zeros(3, np.float32))) for sz, zc, m in layers]
    _, _, _, st0 = orc.trace_photons(orc.OracleScene(sg.slab_stack(clear)), n_photons, max_depth, wl, seed)
    total = sum(v[0] for k, v in st0.items() if k != "segments")
    assert st["truncated"][1] < n_photons * 1e-4
    return st["deposited"][0] / total, 2.5 / math.sqrt(n_photons)


def test_plain_slab_transmittance():
    got, tol = _transmittance([((1.0, 1.0, 0.4), 0.7, sg.glass(1.5))], 550.0)
    want = _stack(_interface(1.0, 1.5), _interface(1.5, 1.0))
    assert abs(got - want) < tol, (got, want)


def test_absorbing_slab_transmittance_interpolated_sigma():
    # sigma(500 nm) halfway between 1 and 3 per metre -> 2; d = 0.4 m
    mat = sg.glass(1.5, sigma=(1.0, 3.0, 8.0))
    got, tol = _transmittance([((1.0, 1.0, 0.4), 0.7, mat)], 500.0)
    want = _stack(_interface(1.0, 1.5), _layer(math.exp(-2.0 * 0.4)), _interface(1.5, 1.0))
    assert abs(got - want) < tol, (got, want)
    assert abs(want - _stack(_interface(1.0, 1.5), _interface(1.5, 1.0))) > 20 * tol


@pytest.mark.parametrize("lam, sigma", [(420.0, 1.0), (650.0, 8.0), (700.0, 8.0), (600.0, 5.5)])
def test_absorbing_slab_sigma_clamps_and_second_segment(lam, sigma):
    mat = sg.glass(1.5, sigma=(1.0, 3.0, 8.0))
    got, tol = _transmittance([((1.0, 1.0, 0.1), 0.7, mat)], lam, n_photons=1 << 15)
    want = _stack(_interface(1.0, 1.5), _layer(math.exp(-sigma * 0.1)), _interface(1.5, 1.0))
    assert abs(got - want) < tol, (got, want)


def test_nested_denser_slab_is_glass_glass():
    outer = ((1.0, 1.0, 0.4), 0.7, sg.glass(1.5, sigma=(0.5, 0.5, 0.5), priority=1))
    inner = ((0.6, 0.6, 0.1), 0.7, sg.glass(1.9, sigma=(2.0, 2.0, 2.0), priority=2))
    got, tol = _transmittance([outer, inner], 550.0)
    want = _stack(_interface(1.0, 1.5), _layer(math.exp(-0.5 * 0.15)), _interface(1.5, 1.9),
                  _layer(math.exp(-2.0 * 0.1)), _interface(1.9, 1.5), _layer(math.exp(-0.5 * 0.15)),
                  _interface(1.5, 1.0))
    assert abs(got - want) < tol, (got, want)
    # each interface taken as air-glass instead would be far off
    plain = _stack(_interface(1.0, 1.5), _layer(math.exp(-0.5 * 0.15)), _interface(1.5, 1.0),
                   _interface(1.0, 1.9), _layer(math.exp(-2.0 * 0.1)), _interface(1.9, 1.0),
                   _interface(1.0, 1.5), _layer(math.exp(-0.5 * 0.15)), _interface(1.5, 1.0))
    assert abs(plain - want) > 10 * tol


def test_nested_lower_priority_slab_is_invisible():
    outer = ((1.0, 1.0, 0.4), 0.7, sg.glass(1.5, sigma=(0.5, 0.5, 0.5), priority=2))
    inner = ((0.6, 0.6, 0.1), 0.7, sg.glass(1.9, sigma=(2.0, 2.0, 2.0), priority=1))
    got, tol = _transmittance([outer, inner], 550.0)
    want = _stack(_interface(1.0, 1.5), _layer(math.exp(-0.5 * 0.4)), _interface(1.5, 1.0))
    assert abs(got - want) < tol, (got, want)


# ---------------------------------------------------------------- camera paths

def _sigma_of(lam, s):
    if lam <= 450.0:
        return s[0]
    if lam >= 650.0:
        return s[2]
    if lam < 550.0:
        return s[0] + (s[1] - s[0]) * (lam - 450.0) / 100.0
    return s[1] + (s[2] - s[1]) * (lam - 550.0) / 100.0


def test_camera_paths_through_absorbing_slab():
    d, le = 0.3, 2.0
    sig = (1.5, 0.5, 4.0)
    wl = sg.Wavelengths(sg.WL_UNIFORM, 1, (550.0,), 400.0, 700.0, 8)
    pix = np.arange(64, dtype=np.uint32)
    scene, cam = sg.slab_over_light(d, sg.glass(1.5, 0.0042, sigma=sig), le=le)
    L, lam = orc.path_samples(orc.OracleScene(scene), cam, 16, 16, wl, 99, pix)
    scene0, _ = sg.slab_over_light(d, sg.glass(1.5, 0.0042), le=le)
    L0, lam0 = orc.path_samples(orc.OracleScene(scene0), cam, 16, 16, wl, 99, pix)
    assert np.array_equal(lam, lam0)
    assert set(np.unique(L0).tolist()) <= {0.0, le}          # lossless glass: weight 1 per event
    lit = L0 == le
    assert lit.mean() > 0.8
    assert np.all(L[~lit] == 0.0)
    passes = []
    for Lv, lv in zip(L[lit], lam[lit]):
        k = -math.log(float(Lv) / le) / (_sigma_of(float(lv), sig) * d)
        j = round((k - 1.0) / 2.0)
        assert j >= 0 and abs(k - (2 * j + 1)) < 2e-4 * (2 * j + 1), (k, float(lv))
        passes.append(j)
    assert np.mean(np.array(passes) == 0) > 0.9


def test_oracle_material_layout_matches_scene_records():
    import ctypes
    assert ctypes.sizeof(orc.Material) == 48 == sg.MATERIAL_DTYPE.itemsize
    for name, _ in orc.Material._fields_:
        assert getattr(orc.Material, name).offset == sg.MATERIAL_DTYPE.fields[name][1], name


def test_nearly_smooth_rough_slab_keeps_the_closed_form():
    """A microfacet slab with tiny alpha behaves as the smooth one, absorption
    included (the rough branch carries the media set and the weights)."""
    mat = sg.glass(1.5, sigma=(1.0, 3.0, 8.0), roughness=1e-4)
    got, tol = _transmittance([((1.0, 1.0, 0.4), 0.7, mat)], 500.0, n_photons=1 << 15)
    want = _stack(_interface(1.0, 1.5), _layer(math.exp(-2.0 * 0.4)), _interface(1.5, 1.0))
    assert abs(got - want) < tol, (got, want)


def test_rough_slab_conserves_flux():
    """Single-scattering microfacet glass loses a little energy, never gains:
    the flux over all photon outcomes stays within [0.9, 1] of the emitted."""
    layers = [((1.0, 1.0, 0.4), 0.7, sg.glass(1.5, roughness=0.3))]
    wl = sg.Wavelengths(sg.WL_FIXED, 1, (550.0,))
    n = 1 << 15
    _, _, _, st = orc.trace_photons(orc.OracleScene(sg.slab_stack(layers)), n, 32, wl, 5)
    _, _, _, st0 = orc.trace_photons(orc.OracleScene(sg.slab_stack([(s, z, sg.glass(1.5)) for s, z, _ in layers])),
                                     n, 32, wl, 5)
    tot = sum(v[0] for k, v in st.items() if k != "segments")
    tot0 = sum(v[0] for k, v in st0.items() if k != "segments")
    assert 0.9 * tot0 < tot < tot0 * (1.0 + 2.5 / math.sqrt(n))
