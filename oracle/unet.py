"""Oracle of the learned denoiser -- TEST INFRASTRUCTURE.

The paper trains a U-Net (Ronneberger et al. 2015) for segmentation
(Sec. IV-A-3); the same architecture family denoises low-sample renders
here.  Plain float64 NumPy: 3x3 convolutions with zero padding written as
nine shifted matrix products, ReLU, 2x2 max pooling, nearest 2x
upsampling, channel concatenation of the skip connection, a 1x1 output
convolution; L1 loss on log(1 + rgb); Adam.  With ``bf16=True`` the tensors
the GPU stores in bfloat16 (weights, the network input, every convolution
output and every gradient fed back into a convolution) are rounded to
bfloat16 (round to nearest even) at the same points, arithmetic staying in
float64.

Layout: activations [B, H, W, C]; weights [Cout, 3, 3, Cin] (1x1 for the
output layer); the flat parameter vector concatenates, layer by layer, the
weights in that order followed by the biases.
"""
from __future__ import annotations

import numpy as np

IN_CH = 9           # log1p(rgb) x3, albedo, normal x3, depth/10, transparent
OUT_CH = 3
WIDTHS = (32, 48, 64, 96, 128)


def layer_shapes(widths=WIDTHS, in_ch=IN_CH, out_ch=OUT_CH):
    """(name, cout, ksize, cin) of every convolution, in parameter order."""
    L = []
    cin = in_ch
    for i, w in enumerate(widths):
        L.append((f"enc{i}a", w, 3, cin))
        L.append((f"enc{i}b", w, 3, w))
        cin = w
    for i in range(len(widths) - 2, -1, -1):
        L.append((f"dec{i}a", widths[i], 3, cin + widths[i]))
        L.append((f"dec{i}b", widths[i], 3, widths[i]))
        cin = widths[i]
    L.append(("out", out_ch, 1, cin))
    return L


def n_params(widths=WIDTHS):
    return sum(co * k * k * ci + co for _, co, k, ci in layer_shapes(widths))


def unpack(theta, widths=WIDTHS):
    p = {}
    off = 0
    for name, co, k, ci in layer_shapes(widths):
        nw = co * k * k * ci
        p[name] = (theta[off:off + nw].reshape(co, k, k, ci), theta[off + nw:off + nw + co])
        off += nw + co
    assert off == len(theta)
    return p


def pack(grads, widths=WIDTHS):
    return np.concatenate([np.concatenate([grads[n][0].ravel(), grads[n][1].ravel()])
                           for n, _, _, _ in layer_shapes(widths)])


def init_params(seed: int, widths=WIDTHS):
    """He-normal weights, zero biases (float32 values)."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, co, k, ci in layer_shapes(widths):
        std = np.sqrt(2.0 / (k * k * ci))
        parts.append(rng.normal(0.0, std, size=co * k * k * ci))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def bf16_round(x):
    """Round float64/float32 values to the nearest bfloat16 (ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    out = np.where(np.isnan(f), f, out)
    return out.astype(np.float64)


def features(rgb, albedo, normal, depthn, trans):
    """Network input from the renderer's outputs ([H,W,...] arrays)."""
    return np.concatenate([np.log1p(np.maximum(rgb, 0.0)), albedo[..., None], normal, depthn[..., None],
                           trans[..., None].astype(np.float64)], axis=-1)


# ------------------------------------------------------------------ layers

def conv(x, w, b):
    """'same' convolution: y[b,y,x,o] = sum_{ky,kx,c} w[o,ky,kx,c] x[b,y+ky-r,x+kx-r,c] + b[o]."""
    k = w.shape[1]
    r = k // 2
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    y = np.zeros((B, H, W, w.shape[0]))
    for ky in range(k):
        for kx in range(k):
            y += xp[:, ky:ky + H, kx:kx + W, :] @ w[:, ky, kx, :].T
    return y + b


def conv_backward(x, w, dz):
    """Gradients of conv w.r.t. input, weights and bias given dL/dy = dz."""
    k = w.shape[1]
    r = k // 2
    B, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (r, r), (r, r), (0, 0)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(k):
        for kx in range(k):
            win = xp[:, ky:ky + H, kx:kx + W, :]
            dw[:, ky, kx, :] = np.einsum("bhwo,bhwc->oc", dz, win)
            dxp[:, ky:ky + H, kx:kx + W, :] += dz @ w[:, ky, kx, :]
    dx = dxp[:, r:r + H, r:r + W, :]
    db = dz.sum(axis=(0, 1, 2))
    return dx, dw, db


def maxpool(x):
    B, H, W, C = x.shape
    v = x.reshape(B, H // 2, 2, W // 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(B, H // 2, W // 2, 4, C)
    idx = np.argmax(v, axis=3)          # first maximum in the order (0,0),(0,1),(1,0),(1,1)
    return np.take_along_axis(v, idx[:, :, :, None, :], axis=3)[:, :, :, 0, :], idx


def maxpool_backward(dy, idx, shape):
    B, H, W, C = shape
    g = np.zeros((B, H // 2, W // 2, 4, C))
    np.put_along_axis(g, idx[:, :, :, None, :], dy[:, :, :, None, :], axis=3)
    return g.reshape(B, H // 2, W // 2, 2, 2, C).transpose(0, 1, 3, 2, 4, 5).reshape(B, H, W, C)


def upsample(x):
    return x.repeat(2, axis=1).repeat(2, axis=2)


def upsample_backward(dy):
    B, H, W, C = dy.shape
    return dy.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# ------------------------------------------------------------------ network

class UNet:
    def __init__(self, theta, widths=WIDTHS, bf16=False):
        self.widths = tuple(widths)
        self.bf16 = bf16
        th = np.asarray(theta, dtype=np.float64)
        self.p = unpack(th, self.widths)
        if bf16:
            self.p = {k: (bf16_round(w), b) for k, (w, b) in self.p.items()}

    def _q(self, x):
        return bf16_round(x) if self.bf16 else x

    def forward(self, x):
        """x [B,H,W,IN_CH] -> predicted log(1+rgb) [B,H,W,3]; keeps the
        intermediates for backward()."""
        c = {}
        h = self._q(x)
        skips = []
        L = len(self.widths)
        for i in range(L):
            if i > 0:
                h, c[f"pool{i}"] = maxpool(h)
            c[f"enc{i}a_in"] = h
            h = self._q(np.maximum(conv(h, *self.p[f"enc{i}a"]), 0.0))
            c[f"enc{i}b_in"] = h
            h = self._q(np.maximum(conv(h, *self.p[f"enc{i}b"]), 0.0))
            c[f"enc{i}b_out"] = h
            skips.append(h)
        for i in range(L - 2, -1, -1):
            u = upsample(h)
            h = np.concatenate([u, skips[i]], axis=-1)
            c[f"dec{i}a_in"] = h
            h = self._q(np.maximum(conv(h, *self.p[f"dec{i}a"]), 0.0))
            c[f"dec{i}b_in"] = h
            h = self._q(np.maximum(conv(h, *self.p[f"dec{i}b"]), 0.0))
            c[f"dec{i}b_out"] = h
        c["out_in"] = h
        y = conv(h, *self.p["out"])
        self.cache = c
        return y

    def backward(self, dy):
        """Gradient of the loss w.r.t. the parameters given dL/d(output)."""
        c = self.cache
        g = {}
        L = len(self.widths)
        dy = self._q(dy)
        dh, dw, db = conv_backward(c["out_in"], self.p["out"][0], dy)
        g["out"] = (dw, db)
        dh = self._q(dh)
        dskips = [None] * L
        for i in range(0, L - 1):
            for part in ("b", "a"):
                name = f"dec{i}{part}"
                yout = c[f"dec{i}b_out"] if part == "b" else c[f"dec{i}b_in"]
                dz = self._q(dh * (yout > 0))
                dh, dw, db = conv_backward(c[f"{name}_in"], self.p[name][0], dz)
                g[name] = (dw, db)
                dh = self._q(dh)
            w_up = dh.shape[-1] - self.widths[i]
            dskips[i] = dh[..., w_up:]
            dh = upsample_backward(dh[..., :w_up])
        for i in range(L - 1, -1, -1):
            if dskips[i] is not None and i < L - 1:
                dh = dh + dskips[i]
            for part in ("b", "a"):
                name = f"enc{i}{part}"
                yout = c[f"enc{i}b_out"] if part == "b" else c[f"enc{i}b_in"]
                dz = self._q(dh * (yout > 0))
                dh, dw, db = conv_backward(c[f"{name}_in"], self.p[name][0], dz)
                g[name] = (dw, db)
                dh = self._q(dh)
            if i > 0:
                shape = c[f"enc{i}a_in"].shape
                dh = maxpool_backward(dh, c[f"pool{i}"], (shape[0], shape[1] * 2, shape[2] * 2, shape[3]))
        return pack(g, self.widths)


def l1_log_loss(pred, target_rgb):
    """Mean over pixels and channels of |pred - log(1 + target)|, and its
    gradient w.r.t. pred (sign / N, sign(0) = 0)."""
    t = np.log1p(np.maximum(target_rgb, 0.0))
    d = pred - t
    n = d.size
    return float(np.abs(d).sum() / n), np.sign(d) / n


def adam(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015) with bias correction; step >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def rel_mse(x, ref, eps=0.01):
    """mean over pixels and channels of (x - ref)^2 / (ref^2 + eps)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.mean((x - ref) ** 2 / (ref * ref + eps)))
