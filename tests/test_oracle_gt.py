"""Pins of the ground-truth pass oracle on synthetic buffers whose answer is
known in closed form."""
import numpy as np
import pytest

from oracle import gt


@pytest.mark.parametrize("t", [1, 2, 5])
def test_outline_band_width(t):
    """A square object of side s away from the border: the outline is the
    band of width t inside its edge, (s^2 - (s - 2t)^2) pixels."""
    s = 20
    obj = np.zeros((40, 40), np.uint32)
    obj[10:10 + s, 8:8 + s] = 3
    o = gt.outline(obj, t)
    assert o.sum() == s * s - (s - 2 * t) ** 2
    assert o[10 + t:10 + s - t, 8 + t:8 + s - t].sum() == 0
    assert np.all(o[obj == 0] == 0)
    # two touching objects: both sides of the shared edge are outlined
    obj2 = np.ones((10, 10), np.uint32)
    obj2[:, 5:] = 2
    o2 = gt.outline(obj2, 1)
    assert np.all(o2[:, 4] == 1) and np.all(o2[:, 5] == 1) and o2.sum() == 20


def test_occlusion_near_side_only():
    d = np.full((12, 12), 2.0, np.float32)
    d[:, 6:] = 5.0            # far wall on the right
    o = gt.occlusion_boundary(d, 0.1)
    assert np.all(o[:, 5] == 1) and o.sum() == 12
    d[0, 0] = np.inf          # a miss next to near pixels marks them
    o = gt.occlusion_boundary(d, 0.1)
    assert o[0, 1] == 1 and o[1, 0] == 1 and o[1, 1] == 1 and o[0, 0] == 0
    # a jump just at the threshold does not count
    e = np.full((3, 3), 1.0, np.float32)
    e[1, 2] = np.float32(1.0) + np.float32(0.25) * np.float32(1.0)
    assert gt.occlusion_boundary(e, 0.25)[1, 1] == 0


def test_caustic_mask_classes():
    w = np.zeros((4, 4, 3), np.float32)
    wo = np.zeros((4, 4, 3), np.float32)
    w[0, 0] = [1.0, 1.0, 1.0]    # bright caustic on glass
    w[1, 1] = [0.0, 1.0, 0.0]    # caustic on another surface
    w[2, 2] = [0.0, 0.0, 0.01]   # below threshold
    trans = np.zeros((4, 4), np.uint8)
    trans[0, 0] = 1
    m = gt.caustic_mask(w, wo, trans, 0.05)
    assert m[0, 0] == 1 and m[1, 1] == 2 and m[2, 2] == 0 and m.sum() == 3
    assert gt.luminance_f32(np.array([1.0, 1.0, 1.0], np.float32)) == np.float32(
        (np.float32(0.2126) + np.float32(0.7152)) + np.float32(0.0722))
