"""Planted mistakes: each case below edits a copy of the oracle's C source
(on the CPU, in a temporary directory), builds it, and runs the pins that
should catch that mistake against the broken build.  A case passes when at
least one of its pins fails, so the pins are shown to see the mistakes a
plausible slip would make, not only to agree with the oracle as written.
"""
import gc
import os
import subprocess

import pytest

import oracle
from tests import test_oracle_emission as E

SRC = os.path.join(os.path.dirname(oracle.__file__), "sco.c")
HDR = os.path.join(os.path.dirname(oracle.__file__), "sco.h")

# (name, [(text, replacement), ...], pins that must catch it)
CASES = [
    ("mixture weight dropped",
     [("/ (nslot * (float)m);", "/ (nslot);")],
     [E.test_coincident_cones_carry_one_cone_of_flux, E.test_overlapping_cones_give_the_union]),
    ("cone containment on sin instead of sin^2",
     [("vdot(cr, cr) <= q", "sqrtf(vdot(cr, cr)) <= q")],
     [E.test_overlapping_cones_give_the_union, E.test_three_overlapping_cones_give_the_union]),
    ("containment ignores the cone's side",
     [("(vdot(om, ax) > 0.0f && vdot(cr, cr) <= q)", "(vdot(cr, cr) <= q)")],
     [lambda: E.test_disjoint_cones_add([0.2, 0.1, 1.0, 0.4], [-0.1, 0.0, 9.0, 0.5])]),
    ("area-light photons without cos(theta_y)",
     [("phi = (((power * cy) * osum)", "phi = (((power) * osum)")],
     [lambda: E.test_area_light_photon_flux_closed_form([1.1, -0.6, 0.8, 0.25])]),
    ("area-light power without the emitter area",
     [("power = s->mat[s->tri_obj[lprim]].le * D.a_tot;", "power = s->mat[s->tri_obj[lprim]].le;")],
     [lambda: E.test_area_light_photon_flux_closed_form([0.0, 0.0, 1.0, 0.3])]),
    ("area-light photons start behind the emitter",
     [("o = offset_ray(y, Nl);", "o = offset_ray(y, vneg(Nl));")],
     [lambda: E.test_area_light_photon_flux_closed_form([0.0, 0.0, 1.0, 0.3])]),
    ("point and area lights not weighted by the entry count",
     [("phi = (((power * cy) * osum) * (float)D.n_entries)", "phi = (((power * cy) * osum))")],
     [E.test_area_and_point_light_share_photons_by_entry]),
    ("bounce disc radius without the square root",
     [("    float rr = sqrtf(u0);\n    float sp, cp;\n    sco_sincos2pi(u1, &sp, &cp);\n    float x = rr * cp",
       "    float rr = u0;\n    float sp, cp;\n    sco_sincos2pi(u1, &sp, &cp);\n    float x = rr * cp")],
     [E.test_cosine_bounce_distribution, E.test_second_bounce_radiance_between_two_planes]),
    ("uniform hemisphere instead of a cosine bounce",
     [("    float rr = sqrtf(u0);\n    float sp, cp;\n    sco_sincos2pi(u1, &sp, &cp);\n    float x = rr * cp",
       "    float rr = sqrtf(u0 * (2.0f - u0));\n    float sp, cp;\n    sco_sincos2pi(u1, &sp, &cp);\n"
       "    float x = rr * cp"),
      ("float z = sqrtf(fmaxf(0.0f, 1.0f - u0));\n    v3 t1, t2;\n    onb(n, &t1, &t2);",
       "float z = 1.0f - u0;\n    v3 t1, t2;\n    onb(n, &t1, &t2);")],
     [E.test_cosine_bounce_distribution, E.test_second_bounce_radiance_between_two_planes]),
    ("bounce half the azimuth range",
     [("sco_sincos2pi(u1, &sp, &cp);\n    float x = rr * cp", "sco_sincos2pi(0.5f * u1, &sp, &cp);\n    float x = rr * cp")],
     [E.test_cosine_bounce_distribution]),
    ("frame without Duff's sign",
     [("float sign = copysignf(1.0f, n.z);", "float sign = 1.0f;")],
     [E.test_duff_frame_is_orthonormal]),
]


def _build_mutant(tmp, edits):
    src = open(SRC).read()
    for a, b in edits:
        assert src.count(a) >= 1, f"mutation anchor not found: {a!r}"
        src = src.replace(a, b)
    c = os.path.join(tmp, "sco.c")
    with open(c, "w") as f:
        f.write(src)
    with open(os.path.join(tmp, "sco.h"), "w") as f:
        f.write(open(HDR).read())
    so = os.path.join(tmp, "libsco_mutant.so")
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fno-finite-math-only",
                    "-fPIC", "-shared", "-w", "-o", so, c, "-lm"], check=True)
    return so


@pytest.mark.parametrize("name,edits,pins", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_is_caught(tmp_path, name, edits, pins):
    so = _build_mutant(str(tmp_path), edits)
    good = oracle.lib()
    oracle._LIB = oracle.load(so)
    caught = []
    try:
        for pin in pins:
            try:
                pin()
            except (AssertionError, ValueError, ZeroDivisionError, FloatingPointError):
                caught.append(getattr(pin, "__name__", "pin"))
    finally:
        gc.collect()
        oracle._LIB = good
    assert caught, f"no pin caught the planted mistake: {name}"
