"""Oracle of the ground-truth passes -- TEST INFRASTRUCTURE.

Plain per-pixel definitions (Sec. III-D of the paper):
  caustic mask  -- luminance difference of a render with and without the
                   caustic light, local where the pixel sees glass;
  outlines      -- object pixels within Chebyshev distance `thickness` of a
                   pixel with another object id;
  occlusion     -- pixels on the near side of a depth jump larger than
                   rel * depth to one of their 8 neighbours.
Luminance is evaluated in float32, one rounding per operation, in the
order (0.2126 R + 0.7152 G) + 0.0722 B.
"""
import numpy as np


def luminance_f32(rgb):
    rgb = np.asarray(rgb, dtype=np.float32)
    a = np.float32(0.2126) * rgb[..., 0]
    b = np.float32(0.7152) * rgb[..., 1]
    c = np.float32(0.0722) * rgb[..., 2]
    return (a + b) + c


def caustic_mask(rgb_with, rgb_without, trans, threshold):
    d = luminance_f32(rgb_with) - luminance_f32(rgb_without)
    t = np.zeros(d.shape, bool) if trans is None else np.asarray(trans).astype(bool)
    return np.where(d > np.float32(threshold), np.where(t, 1, 2), 0).astype(np.uint8)


def outline(obj, thickness):
    obj = np.asarray(obj)
    h, w = obj.shape
    out = np.zeros((h, w), np.uint8)
    t = int(thickness)
    for y in range(h):
        for x in range(w):
            o = obj[y, x]
            if o == 0:
                continue
            win = obj[max(0, y - t):min(h, y + t + 1), max(0, x - t):min(w, x + t + 1)]
            out[y, x] = 1 if np.any(win != o) else 0
    return out


def occlusion_boundary(depth, rel):
    depth = np.asarray(depth, dtype=np.float32)
    h, w = depth.shape
    out = np.zeros((h, w), np.uint8)
    rel = np.float32(rel)
    for y in range(h):
        for x in range(w):
            d = depth[y, x]
            if not np.isfinite(d):
                continue
            lim = rel * d
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    yy, xx = y + dy, x + dx
                    if (dx or dy) and 0 <= yy < h and 0 <= xx < w:
                        if np.float32(depth[yy, xx] - d) > lim:
                            out[y, x] = 1
    return out
