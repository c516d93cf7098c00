"""How far BF16 storage alone (weights, activations, masked output gradients;
FP64 arithmetic) moves the network oracle's output and loss gradient: the
floor under the GPU-vs-FP64 tolerances of the network tests (CPU only).

Measured on the shapes of the GPU parity tests: forward 1.2-1.3% relative L2,
loss gradient 6.2% relative L2 with cosine 0.9981.  The GPU tests hold the
forward to 2e-2 and the gradient to 8e-2 / cosine 0.998, i.e. within about
1.5x and 1.3x of what BF16 storage costs before any kernel is involved."""
import numpy as np
import pytest

import bf16_storage as B
from helpers import medium, rand_c, relerr
from oracle import train as T
from oracle import unet as U


def small_theta(seed, widths, down_res):
    layers = U.all_layers(widths, down_res)
    theta = U.init_params(layers, np.random.default_rng(seed)).astype(np.float32)
    o = 0
    rng = np.random.default_rng(seed + 1)
    for l in layers:
        o += int(np.prod(l.wshape()))
        theta[o:o + l.cout] = 0.05 * rng.standard_normal(l.cout)
        o += l.cout
    return theta.astype(np.float64)


def test_bf16_rounding_is_round_to_nearest_even():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5e-3, 3.0e38])
    r = B.bf16(x)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0 + 2 ** -6 and r[3] == 1.0
    assert abs(r[4] - x[4]) <= 2 ** -8 * abs(x[4])
    assert np.all(np.abs(r - x) <= 2 ** -8 * np.abs(x))    # unit roundoff of an 8-bit significand


@pytest.mark.parametrize("nz,nx,B_,widths,dr,seeds", [
    (32, 32, 2, (32, 32, 32, 32), 1, (7, 3, 5)),
    (48, 80, 3, (32, 64, 128, 256), 2, (9, 11, 6)),
])
def test_forward_floor(nz, nx, B_, widths, dr, seeds):
    med = medium(nz, nx, seed=seeds[0])
    th = small_theta(seeds[1], widths, dr)
    rin = np.random.default_rng(seeds[2]).standard_normal((B_, nz, nx, 2)).astype(np.float32).astype(np.float64)
    enc = U.encoder_input(med.kappa2, med.gamma, med.omega, med.h, med.h)
    ref, _ = U.network_forward(th, enc, rin, widths, dr)
    emu = B.network_forward(th, enc, rin, widths, dr)
    e = relerr(emu, ref)
    print("forward floor", e)
    assert 5e-3 <= e <= 1.6e-2


def test_loss_gradient_floor():
    W, DR = (32, 32, 32, 32), 1
    nz = nx = 32
    med = medium(nz, nx, seed=8)
    th = small_theta(4, W, DR)
    r = rand_c((3, nz, nx), 1).astype(np.complex64).astype(np.complex128)
    e = (1e-4 * rand_c((3, nz, nx), 2)).astype(np.complex64).astype(np.complex128)
    enc = U.encoder_input(med.kappa2, med.gamma, med.omega, med.h, med.h)
    L0, g0 = T.loss_and_grad(th, enc, r, e, med.h, med.h, W, DR)
    L1, g1 = B.loss_and_grad(th, enc, r, e, med.h, med.h, W, DR)
    cos = g1 @ g0 / np.linalg.norm(g1) / np.linalg.norm(g0)
    print("gradient floor", relerr(g1, g0), cos, abs(L1 - L0) / L0)
    assert abs(L1 - L0) <= 2e-2 * L0
    assert 3e-2 <= relerr(g1, g0) <= 8e-2
    assert 0.997 <= cos <= 0.9995
