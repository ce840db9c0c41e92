"""Each convolution kernel of the denoiser alone, through the C ABI
(sc_unet_layer_forward / sc_unet_layer_backward), against the oracle's
plain float64 convolution and its gradients on bfloat16-representable
inputs, weights and output gradients (so both sides start from the same
values and differ only by the GPU's float accumulation and its rounding of
stored results to bfloat16).

Bars (the survey's): forward relative L2 <= 1e-3 against the oracle's
output rounded to bfloat16 where the network stores bfloat16 (3x3 layers)
and against the float output of the 1x1 layer; gradients relative L2
<= 1e-2 and cosine >= 0.999 (input gradient against the oracle's rounded
to bfloat16; weight and bias gradients in float).  Layers: the first (9
input channels padded to 16), encoder layers of every width, a decoder
layer reading a concatenation (224 channels), and the 1x1 output layer;
a 24 x 40 image leaves ragged tiles in x; both tile shapes of the 3x3
kernel."""
import numpy as np
import pytest
import torch

from oracle import unet as U

pytestmark = pytest.mark.gpu

WIDTHS = (32, 48, 64, 96, 128)
LAYERS = [0, 1, 3, 7, 9, 10, 16, 18]


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _cos(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.fixture(scope="module")
def net():
    import paper_2107_11008_amd as sc
    ctx = sc.Context(0)
    rng = np.random.default_rng(31)
    th = U.init_params(17, WIDTHS).astype(np.float64)
    th = th + rng.normal(scale=0.05, size=th.shape)          # non-zero biases
    th = U.bf16_round(th).astype(np.float32)                  # weights exactly representable in bfloat16
    n = sc.UNet(ctx, WIDTHS, th)
    yield ctx, n, U.unpack(th.astype(np.float64), WIDTHS)
    n.close()


@pytest.fixture(params=[2048, 0], ids=["default-tiles", "12-row-tiles"])
def tiles(request, net):
    import paper_2107_11008_amd as sc
    ctx = net[0]
    ctx.set_option(sc._sc.SC_OPT_CONV_BIG_TILE, request.param)
    yield request.param
    ctx.set_option(sc._sc.SC_OPT_CONV_BIG_TILE, 2048)


def _layer(net, li):
    name, co, k, ci = U.layer_shapes(WIDTHS)[li]
    return name, co, k, ci


@pytest.mark.parametrize("li", LAYERS)
@pytest.mark.parametrize("relu", [1, 0])
def test_layer_forward(net, tiles, li, relu):
    ctx, n, P = net
    name, co, k, ci = _layer(net, li)
    rng = np.random.default_rng(100 + li)
    x = U.bf16_round(rng.normal(size=(2, 24, 40, ci))).astype(np.float32)
    g = n.layer_forward(li, torch.from_numpy(x).cuda(), relu=bool(relu)).cpu().numpy()
    w, b = P[name]
    o = U.conv(x.astype(np.float64), w, b)
    if relu:
        o = np.maximum(o, 0.0)
    if k == 3:
        o = U.bf16_round(o)
    e = _rel(g, o)
    print(f"layer {li} ({name}, {ci}->{co}, {k}x{k}, relu {relu}, tiles {tiles}): forward rel L2 {e:.2e}")
    assert e <= 1e-3, e


@pytest.mark.parametrize("li", LAYERS)
def test_layer_backward(net, tiles, li):
    ctx, n, P = net
    name, co, k, ci = _layer(net, li)
    rng = np.random.default_rng(200 + li)
    x = U.bf16_round(rng.normal(size=(2, 24, 40, ci))).astype(np.float32)
    dz = U.bf16_round(rng.normal(size=(2, 24, 40, co)) * 1e-2).astype(np.float32)
    dx, dw = (t.cpu().numpy() for t in n.layer_backward(li, torch.from_numpy(x).cuda(), torch.from_numpy(dz).cuda()))
    w, _ = P[name]
    odx, odw, odb = U.conv_backward(x.astype(np.float64), w, dz.astype(np.float64))
    nw = co * k * k * ci
    e_dx = _rel(dx, U.bf16_round(odx))
    e_dw = _rel(dw[:nw], odw)
    e_db = _rel(dw[nw:], odb)
    print(f"layer {li} ({name}, {ci}->{co}, {k}x{k}, tiles {tiles}): dX rel L2 {e_dx:.2e}, dW {e_dw:.2e}, "
          f"db {e_db:.2e}")
    assert e_dx <= 1e-2 and _cos(dx, odx) >= 0.999, e_dx
    assert e_dw <= 1e-2 and _cos(dw[:nw], odw) >= 0.999, e_dw
    assert e_db <= 1e-2 and _cos(dw[nw:], odb) >= 0.999, e_db


def test_layer_arguments_checked(net):
    import paper_2107_11008_amd as sc
    ctx, n, _ = net
    x = torch.zeros((1, 8, 8, 9), device="cuda")
    y = torch.zeros((1, 8, 8, 32), device="cuda")
    lib = sc._sc.load()
    assert lib.sc_unet_layer_forward(ctx.h, n.h, 19, x.data_ptr(), 1, 8, 8, 1, y.data_ptr()) == -1
    assert lib.sc_unet_layer_forward(ctx.h, n.h, 0, x.data_ptr(), 0, 8, 8, 1, y.data_ptr()) == -1
    assert lib.sc_unet_layer_backward(ctx.h, n.h, 0, x.data_ptr(), y.data_ptr(), 1, 8, 8, None, None) == -1
