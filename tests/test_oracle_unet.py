"""Pins of the oracle's network, optimiser and training-data parts (eq. 4.1-4.3,
Alg. 2) against direct loops, an independent library correlation, central
differences, closed forms of Adam and of one GMRES iteration, and invariants
(CPU only)."""
import numpy as np
import pytest
from scipy import signal

from helpers import medium, rand_c, relerr
from oracle import krylov as kr
from oracle import multigrid as mg
from oracle import operator as op
from oracle import train as T
from oracle import unet as U

TINY = (4, 8, 8, 8)


# ---------------------------------------------------------------- primitive layers
def conv_loops(x, W, b, s):
    B, H, Wd, C = x.shape
    O = W.shape[0]
    Ho, Wo = (H + s - 1) // s, (Wd + s - 1) // s
    out = np.zeros((B, Ho, Wo, O))
    for bb in range(B):
        for y in range(Ho):
            for xx in range(Wo):
                for o in range(O):
                    v = b[o]
                    for ky in range(3):
                        for kx in range(3):
                            yi, xi = s * y + ky - 1, s * xx + kx - 1
                            if 0 <= yi < H and 0 <= xi < Wd:
                                for c in range(C):
                                    v += x[bb, yi, xi, c] * W[o, ky, kx, c]
                    out[bb, y, xx, o] = v
    return out


@pytest.mark.parametrize("s,H,Wd", [(1, 5, 6), (2, 5, 6), (2, 6, 4), (1, 1, 3)])
def test_conv3x3_equals_direct_loops(s, H, Wd):
    rng = np.random.default_rng(s * 10 + H)
    x = rng.standard_normal((2, H, Wd, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    assert np.abs(U.conv3x3(x, W, b, s) - conv_loops(x, W, b, s)).max() < 1e-12


def test_conv3x3_equals_scipy_correlate():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((1, 9, 7, 2))
    W = rng.standard_normal((3, 3, 3, 2))
    b = np.zeros(3)
    out = U.conv3x3(x, W, b, 1)
    for o in range(3):
        ref = sum(signal.correlate2d(x[0, :, :, c], W[o, :, :, c], mode="same", boundary="fill")
                  for c in range(2))
        assert np.abs(out[0, :, :, o] - ref).max() < 1e-12


def test_upconv_equals_direct_loops():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2, 3, 4, 3))
    W = rng.standard_normal((2, 2, 5, 3))
    b = rng.standard_normal(5)
    ref = np.zeros((2, 6, 8, 5))
    for bb in range(2):
        for Y in range(6):
            for X in range(8):
                for o in range(5):
                    ref[bb, Y, X, o] = b[o] + sum(x[bb, Y // 2, X // 2, c] * W[Y % 2, X % 2, o, c] for c in range(3))
    assert np.abs(U.upconv(x, W, b) - ref).max() < 1e-12


def _fd_check(f, args, grads, rng, picks=6, eps=1e-6):
    """Central differences of scalar f along single entries of each argument."""
    for ai, (a, g) in enumerate(zip(args, grads)):
        for _ in range(picks):
            idx = tuple(rng.integers(0, n) for n in a.shape)
            old = a[idx]
            a[idx] = old + eps
            fp = f()
            a[idx] = old - eps
            fm = f()
            a[idx] = old
            fd = (fp - fm) / (2 * eps)
            assert abs(g[idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (ai, idx, g[idx], fd)


@pytest.mark.parametrize("s", [1, 2])
def test_conv3x3_backward_central_differences(s):
    rng = np.random.default_rng(5 + s)
    x = rng.standard_normal((2, 6, 5, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    G = rng.standard_normal(U.conv3x3(x, W, b, s).shape)
    gx, gW, gb = U.conv3x3_backward(x, W, G, s)
    _fd_check(lambda: float(np.sum(G * U.conv3x3(x, W, b, s))), [x, W, b], [gx, gW, gb], rng)


def test_upconv_backward_central_differences():
    rng = np.random.default_rng(8)
    x = rng.standard_normal((2, 3, 4, 3))
    W = rng.standard_normal((2, 2, 5, 3))
    b = rng.standard_normal(5)
    G = rng.standard_normal((2, 6, 8, 5))
    gx, gW, gb = U.upconv_backward(x, W, G)
    _fd_check(lambda: float(np.sum(G * U.upconv(x, W, b))), [x, W, b], [gx, gW, gb], rng)


# ---------------------------------------------------------------- whole network
def tiny_net(seed=0, B=2, H=16, Wd=16):
    rng = np.random.default_rng(seed)
    layers = U.all_layers(TINY, 2)
    theta = U.init_params(layers, rng) + 0.01 * rng.standard_normal(U.n_params(layers))
    enc_in = rng.standard_normal((1, H, Wd, 2))
    rin = rng.standard_normal((B, H, Wd, 2))
    return theta, enc_in, rin, layers


def test_network_shapes_and_parameter_count():
    theta, enc_in, rin, layers = tiny_net()
    out, _ = U.network_forward(theta, enc_in, rin, TINY)
    assert out.shape == rin.shape
    assert U.n_params(layers) == theta.size
    full = U.all_layers(U.WIDTHS, 2)
    # every layer of the full network: 3x3 convs (9 Cin Cout + Cout) and 2x2 up-convs (4 Cin Cout + Cout)
    assert U.n_params(full) == sum((9 if l.kind == "conv" else 4) * l.cin * l.cout + l.cout for l in full)


def test_network_backward_central_differences():
    theta, enc_in, rin, layers = tiny_net(seed=1)
    out, st = U.network_forward(theta, enc_in, rin, TINY)
    G = np.random.default_rng(2).standard_normal(out.shape)
    grad = U.network_backward(st, G, TINY)
    n_enc = U.n_params(U.encoder_layers(TINY, down_res=2))
    rng = np.random.default_rng(3)
    for part in ("encoder", "solver", "all"):
        d = rng.standard_normal(theta.size)
        if part == "encoder":
            d[n_enc:] = 0
        elif part == "solver":
            d[:n_enc] = 0
        eps = 1e-6
        fp = np.sum(G * U.network_forward(theta + eps * d, enc_in, rin, TINY)[0])
        fm = np.sum(G * U.network_forward(theta - eps * d, enc_in, rin, TINY)[0])
        fd = (fp - fm) / (2 * eps)
        assert abs(np.dot(grad, d) - fd) <= 1e-6 * abs(fd), (part, np.dot(grad, d), fd)


def test_preconditioner_is_positively_homogeneous_and_zero_at_zero():
    med = medium(16, 16, seed=3)
    layers = U.all_layers(TINY, 2)
    theta = U.init_params(layers, np.random.default_rng(1))
    r = rand_c((2, 16, 16), 4)
    e1 = U.cnn_precond(theta, med.kappa2, med.gamma, med.omega, med.h, med.h, r, TINY)
    e2 = U.cnn_precond(theta, med.kappa2, med.gamma, med.omega, med.h, med.h, 2.5 * r, TINY)
    assert relerr(e2, 2.5 * e1) < 1e-12
    z = U.cnn_precond(theta, med.kappa2, med.gamma, med.omega, med.h, med.h, np.zeros((1, 16, 16)), TINY)
    assert np.abs(z).max() == 0.0


# ---------------------------------------------------------------- loss and Adam
def test_scaled_input_has_norm_sqrt_n_and_mse_gradient():
    r = rand_c((3, 8, 8), 5)
    e = rand_c((3, 8, 8), 6)
    rin, tgt = T.scaled_pair(r, e, 0.5, 0.25)
    assert np.allclose(np.sum(rin ** 2, axis=(1, 2, 3)), 64.0)
    # target = (e / r-norm) * sqrt(N) / (hx hz)
    assert np.allclose(tgt[..., 0] + 1j * tgt[..., 1],
                       e * (8.0 / np.linalg.norm(r.reshape(3, -1), axis=1))[:, None, None] / 0.125)
    out = np.random.default_rng(7).standard_normal(rin.shape)
    L, g = T.mse_loss_and_grad(out, tgt)
    assert L == pytest.approx(np.sum((out - tgt) ** 2) / 3)
    rng = np.random.default_rng(8)
    _fd_check(lambda: T.mse_loss_and_grad(out, tgt)[0], [out], [g], rng, picks=8, eps=1e-2)


def test_adam_first_step_and_constant_gradient():
    # With bias correction, m_hat = g and v_hat = g^2 whenever the gradient has
    # been constant so far: every step moves by lr g / (|g| + eps).
    lr, eps = 1e-3, 1e-8
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    th = np.array([1.0, 1.0, 1.0, 1.0])
    opt = T.Adam(4, lr=lr, eps=eps)
    for t in range(5):
        new = opt.step(th, g)
        assert np.allclose(th - new, lr * g / (np.abs(g) + eps), rtol=1e-9, atol=1e-15)
        th = new


def test_adam_zero_after_sign_flip_of_equal_halves():
    # gradients g then -g: m_2 = -0.01 g, so the second step moves against g
    opt = T.Adam(1, lr=1.0)
    th = opt.step(np.zeros(1), np.ones(1))
    th2 = opt.step(th, -np.ones(1))
    assert th2[0] > th[0]


# ---------------------------------------------------------------- training data (eq. 4.3, Alg. 2)
def _setup(n=16, seed=9):
    med = medium(n, n, seed=seed)
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    V = mg.VCycle(med.kappa2, med.gamma, med.omega, med.h)
    return med, coef, V


def test_sample_k_is_uniform_on_1_to_10():
    ks = np.array([T.sample_k(i, 5) for i in range(3000)])
    counts = np.bincount(ks, minlength=11)[1:]
    assert ks.min() == 1 and ks.max() == 10
    assert (np.abs(counts - 300) < 60).all()


def test_pairs_satisfy_h_e_equals_r():
    med, coef, V = _setup()
    R, E, ks = T.make_pairs(coef, med.h, med.h, V, (16, 16), 6, seed=3)
    for t in range(6):
        HE = op.apply(coef, E[t], med.h, med.h)
        # r = b - H x~ cancels: rounding relative to ||r|| grows like ||b|| / ||r||
        assert relerr(HE, R[t]) < 1e-9
        assert 1 <= ks[t] <= 10


def test_one_iteration_pair_closed_form():
    med, coef, V = _setup()
    i = next(i for i in range(200) if T.sample_k(i, 3) == 1)
    R, E, ks = T.make_pairs(coef, med.h, med.h, V, (16, 16), 1, seed=3, first=i)
    assert ks == [1]
    x = T.sample_x(i, 256, 3).reshape(16, 16)
    b = op.apply(coef, x, med.h, med.h)
    z = V(b)                                       # M b (V is linear)
    w = op.apply(coef, z, med.h, med.h)
    alpha = np.vdot(w, b) / np.vdot(w, w)          # argmin ||b - alpha H M b||
    xt = alpha * z
    assert relerr(E[0], x - xt) < 1e-10
    assert relerr(R[0], b - op.apply(coef, xt, med.h, med.h)) < 1e-10


def test_alg2_step_closed_form_and_invariant():
    med, coef, V = _setup()
    R, E, _ = T.make_pairs(coef, med.h, med.h, V, (16, 16), 3, seed=4)
    layers = U.all_layers(TINY, 2)
    theta = U.init_params(layers, np.random.default_rng(2), small_residual=True)
    Rn, En = T.alg2_new_pairs(theta, coef, med.h, med.h, V, med.kappa2, med.gamma, med.omega, R, E, TINY)
    e_new = U.cnn_precond(theta, med.kappa2, med.gamma, med.omega, med.h, med.h, R, TINY)
    for t in range(3):
        r0 = R[t] - op.apply(coef, e_new[t], med.h, med.h)
        z = V(r0)
        w = op.apply(coef, z, med.h, med.h)
        alpha = np.vdot(w, r0) / np.vdot(w, w)
        assert relerr(En[t], e_new[t] + alpha * z) < 1e-10
        assert relerr(op.apply(coef, En[t], med.h, med.h), Rn[t]) < 1e-9


def test_pairs_match_k_step_gmres_residual_reduction():
    # the pair's residual is what k right-preconditioned GMRES steps leave, and
    # it shrinks monotonically in k (GMRES minimises over nested spaces)
    med, coef, V = _setup()
    A = lambda v: op.apply(coef, v.reshape(16, 16), med.h, med.h).ravel()
    M = lambda v: V(v.reshape(16, 16)).ravel()
    x = T.sample_x(0, 256, 7)
    b = A(x)
    prev = np.linalg.norm(b)
    for k in range(1, 6):
        res = kr.fgmres(A, b, M=M, max_iters_exact=k)
        cur = np.linalg.norm(b - A(res.x))
        assert cur <= prev * (1 + 1e-12)
        prev = cur
