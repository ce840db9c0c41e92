"""Pins of the oracle's rough (GGX) dielectric interface.

Glass roughness is one of the scene variations of the paper's ablation
(Sec. III-C); the oracle models it with the microfacet refraction model of
Walter, Marschner, Li and Torrance (EGSR 2007), sampled through the
distribution of visible normals (Heitz, JCGT 2018) with the Fresnel term
at m choosing reflection or refraction, so that every weight is
G1(o) <= 1.  The pin is Walter et al.'s closed-form BSDF, which does not
depend on how it is sampled: the expected sampling weight that lands in a
bin of outgoing directions must equal the integral over that bin of

    f_r |o.n| = F(i.h) D(h) G(i, o) / (4 |i.n|)                       (eq. 20)
    f_t |o.n| = |i.h| |o.h| n_o^2 (1 - F(i.h)) D(h) G(i, o)
                / (|i.n| (n_i (i.h) + n_o (o.h))^2)                    (eq. 21)

with the GGX distribution D (eq. 33), Smith G = G1(i) G1(o) (eq. 34) and
the exact unpolarised Fresnel reflectance, all evaluated here in double
and integrated on a fine grid.  A mistake in the sampled distribution,
the weight, the refraction geometry or the Fresnel choice moves weight
between bins or between the two hemispheres.  As alpha goes to 0 the
interface must become the smooth one.
"""
import math

import numpy as np
import pytest

import oracle as orc


def _fresnel(n1, n2, c):
    s2 = (n1 / n2) ** 2 * np.maximum(0.0, 1.0 - c * c)
    tir = s2 >= 1.0
    ct = np.sqrt(np.maximum(0.0, 1.0 - s2))
    rs = (n1 * c - n2 * ct) / (n1 * c + n2 * ct)
    rp = (n1 * ct - n2 * c) / (n1 * ct + n2 * c)
    return np.where(tir, 1.0, 0.5 * (rs * rs + rp * rp))


def _D(cm, a):
    cm = np.clip(cm, 1e-300, 1.0)
    t2 = (1.0 - cm * cm) / (cm * cm)
    return np.where(cm > 0, a * a / (math.pi * cm ** 4 * (a * a + t2) ** 2), 0.0)


def _G1(cv, a):
    cv = np.clip(np.abs(cv), 1e-300, 1.0)
    t2 = (1.0 - cv * cv) / (cv * cv)
    return 2.0 / (1.0 + np.sqrt(1.0 + a * a * t2))


TH_BINS = np.radians(np.arange(0, 91, 10.0))
PHI_BINS = np.radians([0.0, 45.0, 135.0, 180.0])


def _bin_integrals(i, n1, n2, a, reflect, nth=1800, nph=1440):
    """Integral of f |o.n| over (theta_o, |phi_o|) bins of the given
    hemisphere; frame: n = +z on the incoming side, i in the x-z plane."""
    th = (np.arange(nth) + 0.5) * (math.pi / 2 / nth)
    ph = (np.arange(nph) + 0.5) * (2 * math.pi / nph) - math.pi
    T, P = np.meshgrid(th, ph, indexing="ij")
    sz = 1.0 if reflect else -1.0
    o = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), sz * np.cos(T)], -1)
    on = o[..., 2]
    inn = i[2]
    if reflect:
        h = i + o
        h = h / np.linalg.norm(h, axis=-1, keepdims=True)
        ih = h @ i
        val = _fresnel(n1, n2, ih) * _D(h[..., 2], a) * _G1(inn, a) * _G1(on, a) / (4.0 * inn)
        ok = (ih > 0) & ((o * h).sum(-1) > 0)
    else:
        h = -(n1 * i + n2 * o)
        h = h / np.linalg.norm(h, axis=-1, keepdims=True)
        h = np.where(h[..., 2:3] < 0, -h, h)
        ih = h @ i
        oh = (o * h).sum(-1)
        den = (n1 * ih + n2 * oh) ** 2
        val = (np.abs(ih) * np.abs(oh) * n2 * n2 * (1.0 - _fresnel(n1, n2, ih)) * _D(h[..., 2], a)
               * _G1(inn, a) * _G1(on, a) / (inn * den))
        ok = (ih > 0) & (oh < 0)
    val = np.where(ok, val, 0.0) * np.sin(T) * (math.pi / 2 / nth) * (2 * math.pi / nph)
    ti = np.digitize(T, TH_BINS) - 1
    pi_ = np.digitize(np.abs(P), PHI_BINS) - 1
    out = np.zeros((len(TH_BINS) - 1, len(PHI_BINS) - 1))
    np.add.at(out, (ti.ravel(), np.clip(pi_.ravel(), 0, len(PHI_BINS) - 2)), val.ravel())
    return out


def _sample_bins(o, w, mask, reflect):
    z = o[:, 2] if reflect else -o[:, 2]
    th = np.arccos(np.clip(z, -1.0, 1.0))
    ph = np.abs(np.arctan2(o[:, 1], o[:, 0]))
    ti = np.clip(np.digitize(th, TH_BINS) - 1, 0, len(TH_BINS) - 2)
    pi_ = np.clip(np.digitize(ph, PHI_BINS) - 1, 0, len(PHI_BINS) - 2)
    s1 = np.zeros((len(TH_BINS) - 1, len(PHI_BINS) - 1))
    s2 = np.zeros_like(s1)
    np.add.at(s1, (ti[mask], pi_[mask]), w[mask])
    np.add.at(s2, (ti[mask], pi_[mask]), w[mask] ** 2)
    return s1, s2


CASES = [  # (theta_i deg, n1, n2, alpha)
    (30.0, 1.0, 1.5, 0.2),
    (70.0, 1.0, 1.5, 0.5),
    (25.0, 1.5, 1.0, 0.3),      # leaving glass: microfacets past the critical angle reflect totally
    (50.0, 1.5, 1.9, 0.1),      # glass to denser glass
]


@pytest.mark.parametrize("theta_i,n1,n2,alpha", CASES)
def test_sampling_matches_walter_bsdf(theta_i, n1, n2, alpha):
    N = 400_000
    t = math.radians(theta_i)
    i = np.array([math.sin(t), 0.0, math.cos(t)])          # towards where the ray came from
    d = (-i).astype(np.float32)
    rng = np.random.default_rng(int(theta_i * 10 + alpha * 100))
    u = rng.random((N, 3), dtype=np.float32)
    o, refl, w = orc.rough_dielectric(d, np.array([0.0, 0.0, 1.0], np.float32), n1, n2, alpha, u)
    o, w = o.astype(np.float64), w.astype(np.float64)
    assert np.all(np.isfinite(w)) and np.all(w >= 0.0) and np.all(w <= 1.0)
    for reflect in (True, False):
        want = _bin_integrals(i, n1, n2, alpha, reflect)
        s1, s2 = _sample_bins(o, w, refl == (1 if reflect else 0), reflect)
        got = s1 / N
        sd = np.sqrt(np.maximum(s2 / N - got * got, 0.0) / N)
        tol = 5.0 * sd + 3e-3 * want + 2e-5
        assert np.all(np.abs(got - want) <= tol), (reflect, np.max(np.abs(got - want) - tol))
        # the totals too
        assert abs(got.sum() - want.sum()) <= 5.0 * math.sqrt((s2.sum() / N - got.sum() ** 2) / N) + 3e-3 * want.sum()


def test_small_alpha_becomes_smooth():
    rng = np.random.default_rng(3)
    n = np.array([0.0, 0.0, 1.0], np.float32)
    agree = 0
    for k in range(400):
        t = rng.uniform(0.0, 1.3)
        p = rng.uniform(0.0, 2 * math.pi)
        inside = k % 2 == 1
        d = np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), -math.cos(t)], np.float32)
        if inside:
            d[2] = -d[2]
        n1, n2 = (1.5, 1.0) if inside else (1.0, 1.5)
        u = rng.random((1, 3), dtype=np.float32)
        o, refl, w = orc.rough_dielectric(d, n, n1, n2, 1e-6, u)
        ok, _, d2, r2, _ = orc.dielectric(d, n, n, np.zeros(3, np.float32), 550.0, 1.5, 0.0, float(u[0, 2]))
        assert ok
        if refl[0] == int(r2):
            agree += 1
            assert np.abs(o[0] - d2).max() < 2e-5
            assert abs(w[0] - 1.0) < 1e-4
    assert agree >= 396


def test_rough_rejects_bad_alpha():
    with pytest.raises(ValueError):
        orc.rough_dielectric(np.array([0, 0, -1], np.float32), np.array([0, 0, 1], np.float32), 1.0, 1.5, 0.0,
                             np.zeros((1, 3), np.float32))
