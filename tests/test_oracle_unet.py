"""Pins of the denoiser oracle: gradients against finite differences, and
each layer against PyTorch's CPU routines (an independent library)."""
import numpy as np
import pytest
import torch

from oracle import unet as U


def test_param_count_and_packing():
    th = U.init_params(0)
    assert len(th) == U.n_params()
    assert 0.9e6 < len(th) < 1.2e6
    p = U.unpack(th.astype(np.float64))
    assert np.array_equal(U.pack(p), th.astype(np.float64))


def test_conv_matches_torch():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 8, 12, 5))
    w = rng.normal(size=(7, 3, 3, 5))
    b = rng.normal(size=7)
    y = U.conv(x, w, b)
    ref = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(w).permute(0, 3, 1, 2),
                                     torch.from_numpy(b), padding=1).permute(0, 2, 3, 1).numpy()
    assert np.allclose(y, ref, atol=1e-12)
    w1 = rng.normal(size=(3, 1, 1, 5))
    y1 = U.conv(x, w1, b[:3])
    ref1 = torch.nn.functional.conv2d(torch.from_numpy(x).permute(0, 3, 1, 2), torch.from_numpy(w1).permute(0, 3, 1, 2),
                                      torch.from_numpy(b[:3])).permute(0, 2, 3, 1).numpy()
    assert np.allclose(y1, ref1, atol=1e-12)


def test_conv_backward_matches_torch():
    rng = np.random.default_rng(1)
    x = torch.from_numpy(rng.normal(size=(2, 6, 8, 4))).requires_grad_()
    w = torch.from_numpy(rng.normal(size=(5, 3, 3, 4))).requires_grad_()
    b = torch.from_numpy(rng.normal(size=5)).requires_grad_()
    dz = rng.normal(size=(2, 6, 8, 5))
    y = torch.nn.functional.conv2d(x.permute(0, 3, 1, 2), w.permute(0, 3, 1, 2), b, padding=1).permute(0, 2, 3, 1)
    y.backward(torch.from_numpy(dz))
    dx, dw, db = U.conv_backward(x.detach().numpy(), w.detach().numpy(), dz)
    assert np.allclose(dx, x.grad.numpy(), atol=1e-10)
    assert np.allclose(dw, w.grad.numpy(), atol=1e-10)
    assert np.allclose(db, b.grad.numpy(), atol=1e-10)


def test_pool_and_upsample_match_torch():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 8, 6, 3))
    y, idx = U.maxpool(x)
    ref = torch.nn.functional.max_pool2d(torch.from_numpy(x).permute(0, 3, 1, 2), 2).permute(0, 2, 3, 1).numpy()
    assert np.array_equal(y, ref)
    up = U.upsample(y)
    ref_up = torch.nn.functional.interpolate(torch.from_numpy(y).permute(0, 3, 1, 2), scale_factor=2,
                                             mode="nearest").permute(0, 2, 3, 1).numpy()
    assert np.array_equal(up, ref_up)
    g = rng.normal(size=y.shape)
    xt = torch.from_numpy(x).permute(0, 3, 1, 2).requires_grad_()
    torch.nn.functional.max_pool2d(xt, 2).backward(torch.from_numpy(g).permute(0, 3, 1, 2))
    assert np.allclose(U.maxpool_backward(g, idx, x.shape), xt.grad.permute(0, 2, 3, 1).numpy())
    assert np.allclose(U.upsample_backward(up), 4 * y)


@pytest.mark.parametrize("widths", [(4, 8), (4, 8, 8)])
def test_gradient_finite_differences(widths):
    """Directional derivatives of a linear functional of the output agree
    with central differences (float64, relative error <= 1e-6)."""
    rng = np.random.default_rng(3)
    th = U.init_params(5, widths).astype(np.float64)
    th += rng.normal(scale=0.05, size=th.shape)      # non-zero biases
    H = 4 * 2 ** (len(widths) - 1)
    x = rng.normal(size=(2, H, H, U.IN_CH))
    r = rng.normal(size=(2, H, H, 3))
    net = U.UNet(th, widths)
    net.forward(x)
    g = net.backward(r)
    for trial in range(3):
        v = rng.normal(size=th.shape)
        eps = 1e-6
        lp = (U.UNet(th + eps * v, widths).forward(x) * r).sum()
        lm = (U.UNet(th - eps * v, widths).forward(x) * r).sum()
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g @ v) <= 1e-6 * max(1.0, abs(fd)), (fd, g @ v)


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    th = rng.normal(size=50)
    t = torch.from_numpy(th.copy()).requires_grad_()
    opt = torch.optim.Adam([t], lr=1e-3)
    m = np.zeros(50)
    v = np.zeros(50)
    for step in range(1, 4):
        g = rng.normal(size=50)
        t.grad = torch.from_numpy(g.copy())
        opt.step()
        th, m, v = U.adam(th, m, v, g, step, 1e-3)
    assert np.allclose(th, t.detach().numpy(), atol=1e-12)


def test_bf16_round_special_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 1e-40, 3.0e38])
    r = U.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -7 and r[3] == -2.5 and r[4] == 0.0
    assert np.all(np.abs(r - x) <= np.abs(x) * 2 ** -8 + 1e-38)
