"""Each layer kind of the networks through the library's BF16 MFMA kernels
against the oracle's direct convolutions (inputs rounded to BF16 on both
sides, so the comparison isolates the kernels from the storage precision)."""
import numpy as np
import pytest
import torch

from helpers import relerr
from oracle import unet as U
from paper_2405_17696_amd import api

pytestmark = pytest.mark.gpu


def bf(x):
    return torch.tensor(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def rnd(shape, seed, scale=1.0):
    return bf(scale * np.random.default_rng(seed).standard_normal(shape))


CONV_CASES = [
    # name, stride, B, H, W, c1, c2, bcast2, cout, relu, resid
    ("s1", 1, 2, 8, 16, 32, 0, False, 32, True, False),
    ("s2", 2, 2, 16, 8, 32, 0, False, 64, True, False),
    ("concat", 1, 2, 8, 8, 32, 32, False, 32, True, False),
    ("bcast", 1, 3, 8, 8, 64, 64, True, 64, True, False),
    ("first", 1, 2, 16, 16, 2, 0, False, 32, True, False),
    ("first_n48", 1, 2, 12, 20, 2, 0, False, 48, True, False),   # matrix-core first layer, three channel tiles
    ("first_c3", 1, 2, 16, 16, 3, 0, False, 32, True, False),    # FP32 first-layer kernel
    ("last", 1, 2, 8, 8, 32, 0, False, 2, False, False),
    ("resid", 1, 2, 8, 8, 32, 0, False, 32, False, True),
    ("wide", 2, 1, 8, 8, 128, 0, False, 256, True, False),
    ("odd", 2, 1, 6, 10, 32, 0, False, 32, True, False),
    # several 16 x 16 pixel tiles with ragged edges (halo-tiled kernel)
    ("tiles", 1, 2, 37, 50, 64, 0, False, 64, True, False),
    ("tiles_ctx", 1, 2, 33, 20, 32, 32, True, 96, True, False),
    ("tiles_head", 1, 2, 40, 24, 32, 0, False, 2, False, False),
    ("tiles_resid", 1, 1, 18, 31, 128, 0, False, 128, False, True),
]


def ref_conv(x1, x2, W, b, stride, bcast2, relu, resid):
    x = x1 if x2 is None else np.concatenate([x1, np.broadcast_to(x2, x1.shape[:3] + x2.shape[3:])], axis=-1)
    y = U.conv3x3(x, W, b, stride)
    if resid is not None:
        y = y + resid
    return np.maximum(y, 0) if relu else y


@pytest.mark.parametrize("case", CONV_CASES, ids=[c[0] for c in CONV_CASES])
def test_conv_layer_forward_backward(gpu, case):
    name, s, B, H, W_, c1, c2, bc, cout, relu, use_resid = case
    print("layer", name, flush=True)
    x1 = rnd((B, H, W_, c1), 1)
    x2 = rnd(((1 if bc else B), H, W_, c2), 2) if c2 else None
    Wt = rnd((cout, 3, 3, c1 + c2), 3, scale=np.sqrt(2.0 / (9 * (c1 + c2))))
    b = rnd((cout,), 4, 0.1)
    Ho, Wo = (H + s - 1) // s, (W_ + s - 1) // s
    resid = rnd((B, Ho, Wo, cout), 5) if use_resid else None
    y = api.cnn_layer_forward(0, s, x1, Wt, b, x2=x2, bcast2=bc, resid=resid, relu=relu)
    yr = ref_conv(x1, x2, Wt, b, s, bc, relu, resid)
    assert relerr(y, yr) <= 1e-5
    # backward
    g = rnd(y.shape, 6)
    gx1, gx2, gw, gb = api.cnn_layer_backward(0, s, x1, Wt, y, g, x2=x2, bcast2=bc, relu=relu)
    gm = bf(g * (y > 0)) if relu else g
    x = x1 if x2 is None else np.concatenate([x1, np.broadcast_to(x2, x1.shape[:3] + x2.shape[3:])], axis=-1)
    rx, rw, rb = U.conv3x3_backward(x, Wt, gm, s)
    assert relerr(gw, rw) <= 1e-5
    assert relerr(gb, rb) <= 1e-5
    assert relerr(gx1, rx[..., :c1]) <= 1e-5
    if c2:
        assert relerr(gx2, rx[..., c1:]) <= 1e-5     # per-sample context gradient


@pytest.mark.parametrize("B,H,W_,cin,cout", [(2, 4, 8, 64, 32), (1, 8, 8, 256, 128), (2, 16, 16, 128, 64)])
def test_upconv_layer_forward_backward(gpu, B, H, W_, cin, cout):
    x = rnd((B, H, W_, cin), 7)
    Wt = rnd((2, 2, cout, cin), 8, scale=np.sqrt(2.0 / cin))
    b = rnd((cout,), 9, 0.1)
    y = api.cnn_layer_forward(1, 2, x, Wt, b, relu=True)
    yr = np.maximum(U.upconv(x, Wt, b), 0)
    assert relerr(y, yr) <= 5e-3                # output stored in BF16
    g = rnd(y.shape, 10)
    gx, _, gw, gb = api.cnn_layer_backward(1, 2, x, Wt, y, g, relu=True)
    gm = bf(g * (y > 0))
    rx, rw, rb = U.upconv_backward(x, Wt, gm)
    assert relerr(gx, rx) <= 1e-5
    assert relerr(gw, rw) <= 1e-5
    assert relerr(gb, rb) <= 1e-5


def test_autotuner_choice_keeps_results(gpu, tmp_path):
    """Tuned and rule-based kernel choices give the same layer within BF16 rounding."""
    x1 = rnd((2, 40, 48, 32), 11)
    Wt = rnd((32, 3, 3, 32), 12, scale=np.sqrt(2.0 / 288))
    b = rnd((32,), 13, 0.1)
    ref = np.maximum(U.conv3x3(x1, Wt, b, 1), 0)
    api.helm_autotune(2)
    api.helm_autotune(0)
    y0 = api.cnn_layer_forward(0, 1, x1, Wt, b, relu=True)
    n0 = api.helm_autotune(-1)
    api.helm_autotune(1)
    y1 = api.cnn_layer_forward(0, 1, x1, Wt, b, relu=True)
    n1 = api.helm_autotune(-1)
    assert n0 == 0 and n1 >= 1
    assert relerr(y0, ref) <= 1e-5 and relerr(y1, ref) <= 1e-5
    # the tuned table survives a save / clear / load round trip
    f = tmp_path / "tune.txt"
    api.helm_autotune_file(f, save=True)
    api.helm_autotune(2)
    assert api.helm_autotune(-1) == 0
    api.helm_autotune_file(f, save=False)
    assert api.helm_autotune(-1) == n1
    y2 = api.cnn_layer_forward(0, 1, x1, Wt, b, relu=True)
    assert np.array_equal(y1, y2)


@pytest.mark.parametrize("B,H,W_", [(2, 14, 14), (2, 37, 50), (1, 16, 30), (3, 5, 9)])
def test_fused_resblock32(gpu, B, H, W_):
    """y = x + conv2(ReLU(conv1(x) + b1)) + b2 in one kernel (14 x 14 output
    tiles): against the oracle's layers, ragged tiles and grids smaller than a tile."""
    x = rnd((B, H, W_, 32), 21)
    W1 = rnd((32, 3, 3, 32), 22, scale=np.sqrt(2.0 / 288))
    W2 = rnd((32, 3, 3, 32), 23, scale=np.sqrt(2.0 / 288))
    b1 = rnd((32,), 24, 0.1)
    b2 = rnd((32,), 25, 0.1)
    y = api.cnn_layer_resblock(x, W1, b1, W2, b2)
    h = bf(np.maximum(U.conv3x3(x, W1, b1, 1), 0))       # the kernel keeps h in BF16
    ref = x + U.conv3x3(h, W2, b2, 1)
    assert relerr(y, ref) <= 5e-3                         # output stored in BF16


FORCE_CASES = [
    # name, kind, stride, B, H, W, c1, c2, bcast2, cout, relu, resid
    ("s1_tiles", 0, 1, 2, 37, 50, 64, 0, False, 64, True, False),
    ("s1_odd", 0, 1, 3, 33, 33, 64, 0, False, 64, True, False),    # 27 tiles: a tile pair spans two samples
    ("s1_n128", 0, 1, 1, 20, 18, 32, 0, False, 128, True, False),
    ("concat", 0, 1, 2, 18, 20, 32, 32, False, 32, True, False),
    ("ctx", 0, 1, 2, 17, 16, 32, 32, True, 64, True, False),
    ("resid", 0, 1, 1, 18, 31, 128, 0, False, 128, False, True),
    ("head", 0, 1, 2, 20, 24, 32, 0, False, 2, False, False),
    ("first", 0, 1, 2, 16, 20, 2, 0, False, 32, True, False),
    ("s2", 0, 2, 2, 20, 18, 64, 0, False, 128, True, False),
    ("s2_wide", 0, 2, 1, 16, 16, 128, 0, False, 256, True, False),
    ("up", 1, 2, 2, 9, 10, 128, 0, False, 64, True, False),
    ("up_wide", 1, 2, 1, 8, 8, 256, 0, False, 128, True, False),
    ("up64", 1, 2, 3, 19, 13, 64, 0, False, 32, True, False),      # 741 pixels: 12 tiles of 64, ragged
]


def test_every_convolution_kernel_against_oracle(gpu):
    """Each convolution kernel kind, pinned in turn, on every layer shape it
    applies to (stride 1 and 2, concatenated and broadcast context, residual,
    2-channel head, first layer, up-convolution, ragged 16 x 16 tiles) against
    the oracle's direct convolution, and on the stride-1 layers also the data
    gradient, which runs the same kernels with flipped taps."""
    count = api.helm_conv_force(-1)
    assert count >= 9
    try:
        for k in range(count):
            api.helm_conv_force(k)
            for name, kind, s, B, H, W_, c1, c2, bc, cout, relu, use_resid in FORCE_CASES:
                print("kernel", k, "case", name, flush=True)
                if kind == 1:
                    x = rnd((B, H, W_, c1), 21)
                    Wt = rnd((2, 2, cout, c1), 22, scale=np.sqrt(2.0 / c1))
                    b = rnd((cout,), 23, 0.1)
                    y = api.cnn_layer_forward(1, 2, x, Wt, b, relu=True)
                    assert relerr(y, np.maximum(U.upconv(x, Wt, b), 0)) <= 5e-3
                    continue
                x1 = rnd((B, H, W_, c1), 24)
                x2 = rnd(((1 if bc else B), H, W_, c2), 25) if c2 else None
                Wt = rnd((cout, 3, 3, c1 + c2), 26, scale=np.sqrt(2.0 / (9 * (c1 + c2))))
                b = rnd((cout,), 27, 0.1)
                Ho, Wo = (H + s - 1) // s, (W_ + s - 1) // s
                resid = rnd((B, Ho, Wo, cout), 28) if use_resid else None
                y = api.cnn_layer_forward(0, s, x1, Wt, b, x2=x2, bcast2=bc, resid=resid, relu=relu)
                assert relerr(y, ref_conv(x1, x2, Wt, b, s, bc, relu, resid)) <= 1e-5
                if s == 1 and c1 >= 32:
                    # the data gradient: a flipped-kernel convolution accumulated into FP32
                    g = rnd(y.shape, 29)
                    gx1, gx2, _, _ = api.cnn_layer_backward(0, s, x1, Wt, y, g, x2=x2, bcast2=bc, relu=relu)
                    gm = bf(g * (y > 0)) if relu else g
                    x = x1 if x2 is None else np.concatenate([x1, np.broadcast_to(x2, x1.shape[:3] + x2.shape[3:])],
                                                             axis=-1)
                    rx, _, _ = U.conv3x3_backward(x, Wt, gm, s)
                    assert relerr(gx1, rx[..., :c1]) <= 1e-5
    finally:
        api.helm_conv_force(-1)
    with pytest.raises(Exception):
        api.helm_conv_force(count)
