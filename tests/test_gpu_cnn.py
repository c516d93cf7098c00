"""GPU parity of the encoder-solver network (BF16 MFMA kernels) against the FP64
oracle: forward, loss gradient, Adam, training-pair generation, Alg. 2, the
preconditioner inside FGMRES, and training itself."""
import numpy as np
import pytest
import torch

import bf16_storage as BS
from helpers import medium, rand_c, relerr
from oracle import krylov as kr
from oracle import multigrid as mg
from oracle import operator as op
from oracle import train as T
from oracle import unet as U
from paper_2405_17696_amd import api

pytestmark = pytest.mark.gpu

W = (32, 32, 32, 32)
DR = 1


def setup(med):
    k2 = torch.tensor(med.kappa2, dtype=torch.float32, device="cuda")
    g = torch.tensor(med.gamma, dtype=torch.float32, device="cuda")
    return api.helm_setup(k2, g, med.omega, med.h)


def small_net(seed=3, widths=W, down_res=DR):
    net = api.cnn_create(widths, seed=0, down_res=down_res)
    theta = U.init_params(U.all_layers(widths, down_res), np.random.default_rng(seed)).astype(np.float32)
    # small non-zero biases so that the bias path is exercised
    layers = U.all_layers(widths, down_res)
    o = 0
    rng = np.random.default_rng(seed + 1)
    for l in layers:
        o += int(np.prod(l.wshape()))
        theta[o:o + l.cout] = 0.05 * rng.standard_normal(l.cout)
        o += l.cout
    assert net.nparams == theta.size
    api.cnn_set_params(net, theta)
    return net, theta.astype(np.float64)


def test_param_layout_matches_oracle(gpu):
    for widths, dr in ((W, DR), ((32, 64, 128, 256), 2)):
        net = api.cnn_create(widths, seed=1, down_res=dr)
        assert net.nparams == U.n_params(U.all_layers(widths, dr))


@pytest.mark.parametrize("nz,nx", [(32, 32), (48, 64), (40, 56)])
def test_forward_parity(gpu, nz, nx):
    print(f"cnn forward {nz}x{nx}", flush=True)
    med = medium(nz, nx, seed=7)
    H = setup(med)
    net, theta = small_net()
    rin = np.random.default_rng(5).standard_normal((2, nz, nx, 2)).astype(np.float32)
    out = api.cnn_forward(net, H, torch.tensor(rin, device="cuda")).cpu().numpy()
    enc = U.encoder_input(med.kappa2, med.gamma, med.omega, med.h, med.h)
    ref, _ = U.network_forward(theta, enc, rin.astype(np.float64), W, DR)
    print("rel err", relerr(out, ref))
    assert relerr(out, ref) <= 2e-2      # BF16 storage alone: 1.3% on this shape


@pytest.mark.parametrize("nz,nx,B", [(32, 32, 1), (48, 80, 3), (40, 56, 2)])
def test_forward_parity_full_width(gpu, nz, nx, B):
    """Default architecture (32-256, two residual blocks per encoder level), on
    the inference path (fused first layer and residual blocks).  48 x 80 spans
    several 16 x 16 tiles and leaves ragged 14 x 14 residual-block tiles; 40 x 56
    leaves ragged 16 x 16 tiles on every level (40 x 56 down to 5 x 7)."""
    widths = (32, 64, 128, 256)
    med = medium(nz, nx, seed=9)
    H = setup(med)
    net, theta = small_net(seed=11, widths=widths, down_res=2)
    rin = np.random.default_rng(6).standard_normal((B, nz, nx, 2)).astype(np.float32)
    out = api.cnn_forward(net, H, torch.tensor(rin, device="cuda")).cpu().numpy()
    enc = U.encoder_input(med.kappa2, med.gamma, med.omega, med.h, med.h)
    ref, _ = U.network_forward(theta, enc, rin.astype(np.float64), widths, 2)
    print("rel err", relerr(out, ref))
    assert relerr(out, ref) <= 2e-2      # BF16 storage alone: 1.2% on the 48 x 80 shape


def test_loss_gradient_parity(gpu):
    print("cnn gradient", flush=True)
    nz = nx = 32
    med = medium(nz, nx, seed=8)
    H = setup(med)
    net, theta = small_net(seed=4)
    r = rand_c((3, nz, nx), 1).astype(np.complex64)
    e = (1e-4 * rand_c((3, nz, nx), 2)).astype(np.complex64)
    api.cnn_zero_grad(net)
    loss = api.cnn_loss_grad(net, H, torch.tensor(r, device="cuda"), torch.tensor(e, device="cuda"))
    g = api.cnn_get_grad(net).astype(np.float64)
    enc = U.encoder_input(med.kappa2, med.gamma, med.omega, med.h, med.h)
    L, gref = T.loss_and_grad(theta, enc, r.astype(np.complex128), e.astype(np.complex128), med.h, med.h, W, DR)
    cos = g @ gref / np.linalg.norm(g) / np.linalg.norm(gref)
    _, gemu = BS.loss_and_grad(theta, enc, r.astype(np.complex128), e.astype(np.complex128), med.h, med.h, W, DR)
    print("loss", loss, L, "grad rel", relerr(g, gref), "cos", cos, "vs BF16-storage oracle", relerr(g, gemu),
          "floor", relerr(gemu, gref))
    # BF16 weights, activations and masked gradients through ~40 layers and
    # their mirror: the oracle with only its storage rounded to BF16 is 6.2%
    # (cosine 0.9981) from the FP64 gradient on this very case
    # (test_bf16_floor); the GPU lands at that floor (5.5-6.2%, cosine
    # 0.9981-0.9985 with the kernel choices of different runs)
    assert abs(loss - L) <= 2e-2 * L
    assert relerr(g, gref) <= 8e-2
    assert cos >= 0.997


def test_adam_step_parity(gpu):
    nz = nx = 32
    med = medium(nz, nx, seed=8)
    H = setup(med)
    net, theta = small_net(seed=4)
    r = torch.tensor(rand_c((2, nz, nx), 1).astype(np.complex64), device="cuda")
    e = torch.tensor((1e-4 * rand_c((2, nz, nx), 2)).astype(np.complex64), device="cuda")
    th0 = api.cnn_get_params(net).astype(np.float64)
    opt = T.Adam(th0.size, lr=1e-3)
    th = th0.copy()
    for step in range(3):
        api.cnn_zero_grad(net)
        api.cnn_loss_grad(net, H, r, e)
        g = api.cnn_get_grad(net).astype(np.float64)
        api.cnn_adam_step(net, 1e-3)
        th = opt.step(th, g)
        got = api.cnn_get_params(net).astype(np.float64)
        assert np.max(np.abs(got - th)) <= 1e-6 + 1e-6 * np.max(np.abs(th))
        api.cnn_set_params(net, th.astype(np.float32))   # keep both sides on the same iterate
        th = api.cnn_get_params(net).astype(np.float64)
    assert np.abs(api.cnn_get_grad(net)).max() == 0.0    # the step zeroes the gradient


def test_make_pairs_parity_and_invariant(gpu):
    nz = nx = 32
    med = medium(nz, nx, seed=12)
    H = setup(med)
    r, e = api.cnn_make_pairs(H, first=5, npairs=4, seed=77)
    r = r.cpu().numpy().astype(np.complex128)
    e = e.cpu().numpy().astype(np.complex128)
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    for t in range(4):
        he = op.apply(coef, e[t], med.h, med.h)
        assert relerr(he, r[t]) <= 1e-5            # H e = r by construction (eq. 4.3)
    V = mg.VCycle(med.kappa2, med.gamma, med.omega, med.h)
    R0, E0, ks = T.make_pairs(coef, med.h, med.h, V, (nz, nx), 4, seed=77, first=5)
    print("k", ks, "e rel", [relerr(e[t], E0[t]) for t in range(4)])
    for t in range(4):
        assert relerr(e[t], E0[t]) <= 2e-3
        assert relerr(r[t], R0[t]) <= 2e-3


def test_alg2_epoch(gpu):
    nz = nx = 32
    med = medium(nz, nx, seed=13)
    H = setup(med)
    net, theta = small_net(seed=6)
    n = 3
    r0, e0 = api.cnn_make_pairs(H, first=0, npairs=n, seed=5)
    R = torch.zeros((2 * n, nz, nx), dtype=torch.complex64, device="cuda")
    E = torch.zeros_like(R)
    R[:n] = r0
    E[:n] = e0
    api.cnn_alg2_epoch(net, H, R, E, n)
    Rn = R[n:].cpu().numpy().astype(np.complex128)
    En = E[n:].cpu().numpy().astype(np.complex128)
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    for t in range(n):
        assert relerr(op.apply(coef, En[t], med.h, med.h), Rn[t]) <= 1e-5   # r~ = H e~
    V = mg.VCycle(med.kappa2, med.gamma, med.omega, med.h)
    Rr, Er = T.alg2_new_pairs(theta, coef, med.h, med.h, V, med.kappa2, med.gamma, med.omega,
                              r0.cpu().numpy().astype(np.complex128), e0.cpu().numpy().astype(np.complex128), W, DR)
    print("alg2 rel", [relerr(En[t], Er[t]) for t in range(n)])
    for t in range(n):
        assert relerr(En[t], Er[t]) <= 5e-2


def test_precond_apply_parity(gpu):
    nz, nx = 32, 48
    med = medium(nz, nx, seed=14)
    H = setup(med)
    net, theta = small_net(seed=7)
    r = rand_c((2, nz, nx), 3).astype(np.complex64)
    e = api.cnn_precond_apply(net, H, torch.tensor(r, device="cuda")).cpu().numpy()
    ref = U.cnn_precond(theta, med.kappa2, med.gamma, med.omega, med.h, med.h, r.astype(np.complex128), W, DR)
    print("apply rel", relerr(e, ref))
    assert relerr(e, ref) <= 3e-2
    # 1-homogeneity: M(a r) = a M(r) for a > 0
    e2 = api.cnn_precond_apply(net, H, torch.tensor((3.5 * r).astype(np.complex64), device="cuda")).cpu().numpy()
    assert relerr(e2, 3.5 * e) <= 1e-5


def test_cnn_vu_fgmres_converges(gpu):
    """M_VU(r) = e0 + V(r - H e0) inside flexible GMRES with a network that
    starts near the zero map: converges to the FP64 tolerance and agrees with
    the direct solve; the iteration count is close to MG-GMRES's."""
    n = 64
    med = medium(n, n, seed=15)
    H = setup(med)
    net = api.cnn_create((32, 32, 32, 32), seed=5, down_res=1)
    b = rand_c((3, n, n), 4).astype(np.complex64)
    bt = torch.tensor(b, device="cuda")
    x, it, rr, st, code = api.helm_solve(H, bt, tol=1e-6, precond="cnn_vu", maxit=600, net=net, restart=20)
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    rel = op.relres(coef, x.cpu().numpy(), b.astype(np.complex128), med.h, med.h)
    _, itm, _, _, cm = api.helm_solve(H, bt, tol=1e-6, precond="mg", maxit=600)
    print("cnn_vu iterations", it, "mg", itm, rel)
    assert code == 0 and np.all(rel <= 1e-6)
    assert np.all(it <= 1.5 * itm + 10)
    xs = op.DirectSolver(op.assemble(coef, med.h, med.h)).solve(b.reshape(3, -1).astype(np.complex128))
    assert relerr(x.cpu().numpy().reshape(3, -1), xs) <= 1e-4
    # graph replay of the same solve (network kernels captured too)
    xg, itg, _, _, cg = api.helm_solve(H, bt, tol=1e-6, precond="cnn_vu", maxit=600, net=net, restart=20,
                                       use_graph=True)
    assert cg == 0 and np.array_equal(it, itg) and torch.equal(x, xg)
    # a fresh operator whose first solve is graph-captured: the encoder context
    # and buffers are prepared eagerly before the capture
    H2 = setup(med)
    x2, it2, _, _, c2 = api.helm_solve(H2, bt, tol=1e-6, precond="cnn_vu", maxit=600, net=net, restart=20,
                                       use_graph=True)
    assert c2 == 0 and np.array_equal(it, it2) and torch.equal(x, x2)


def test_cnn_only_preconditioner_reports_status(gpu):
    """M = SolverNet alone with an untrained network: the solve runs, the
    residual does not grow, and the iteration cap is reported per RHS."""
    n = 32
    med = medium(n, n, seed=18)
    H = setup(med)
    net = api.cnn_create((32, 32, 32, 32), seed=6, down_res=1)
    b = rand_c((2, n, n), 5).astype(np.complex64)
    x, it, rr, st, code = api.helm_solve(H, torch.tensor(b, device="cuda"), tol=1e-10, precond="cnn", maxit=20,
                                         net=net)
    assert code == 1 and np.all(st == 1) and np.all(it == 20) and np.all(rr <= 1.0 + 1e-6)


def test_training_reduces_loss_and_roundtrip(gpu, tmp_path):
    n = 32
    med = medium(n, n, seed=16)
    H = setup(med)
    net, _ = small_net(seed=9)
    hist, dsz = api.cnn_precond_train(net, H, npairs=64, batch=8, steps=48, lr=1e-3, seed=3)
    print("loss", hist[:4], hist[-4:])
    assert len(hist) == 48 and dsz == 64
    assert np.mean(hist[-8:]) < 0.8 * np.mean(hist[:8])
    p = tmp_path / "net.bin"
    api.cnn_save(net, p)
    net2 = api.cnn_load(p)
    assert np.array_equal(api.cnn_get_params(net), api.cnn_get_params(net2))
    # the Adam state travels too: one more identical step on both
    r, e = api.cnn_make_pairs(H, 0, 8, 3)
    for nn in (net, net2):
        api.cnn_zero_grad(nn)
        api.cnn_loss_grad(nn, H, r, e)
        api.cnn_adam_step(nn, 1e-3)
    assert np.array_equal(api.cnn_get_params(net), api.cnn_get_params(net2))


def test_alg2_training_doubles_dataset(gpu):
    n = 32
    med = medium(n, n, seed=17)
    H = setup(med)
    net, _ = small_net(seed=10)
    hist, dsz = api.cnn_precond_train(net, H, batch=8, steps=1000, lr=1e-3, seed=4, alg2_initial=16,
                                      alg2_data_epochs=3, alg2_epochs=5)
    assert dsz == 16 * 2 ** 3
    # epochs: 16/8 + 32/8 + 64/8 + 128/8 + 128/8 steps
    assert len(hist) == 2 + 4 + 8 + 16 + 16


@pytest.mark.parametrize("bscale", [1e3, 1e-4])
def test_one_iteration_closed_form_cnn_vu(gpu, bscale):
    """One FGMRES step from x0 with M_VU equals the closed form
    z = M_VU(r0/||r0||), w = H z, y = w^H r0 / w^H w, x1 = x0 + y z, where
    M_VU(v) = e0 + V(v - H e0), e0 = M_net(v); ||r0|| far from 1 exercises the
    scaling of the network inside the Krylov loop."""
    n = 32
    med = medium(n, n, seed=19)
    H = setup(med)
    net, _ = small_net(seed=12)
    b = (bscale * rand_c((1, n, n), 6)).astype(np.complex64)
    x0 = (bscale * 1e-3 * rand_c((1, n, n), 7)).astype(np.complex128)
    bt = torch.tensor(b, device="cuda")
    x = torch.tensor(x0, device="cuda")
    x1, it, rr, st, code = api.helm_solve(H, bt, x=x, tol=1e-12, precond="cnn_vu", maxit=1, net=net, x0_given=True)
    assert it[0] == 1
    # closed form from the library's building blocks, combined in FP64 on the host
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    r0 = b.astype(np.complex128) - op.apply(coef, x0, med.h, med.h)
    v = (r0 / np.linalg.norm(r0)).astype(np.complex64)
    e0 = api.cnn_precond_apply(net, H, torch.tensor(v, device="cuda")).cpu().numpy().astype(np.complex128)
    res = (v - op.apply(coef, e0, med.h, med.h)).astype(np.complex64)
    z = e0 + api.helm_vcycle(H, torch.tensor(res, device="cuda")).cpu().numpy()
    w = op.apply(coef, z, med.h, med.h)
    y = np.vdot(w, r0) / np.vdot(w, w)
    ref = x0 + y * z
    print("closed form rel", relerr(x1.cpu().numpy(), ref))
    assert relerr(x1.cpu().numpy() - x0, ref - x0) <= 1e-4


def test_non_finite_network_output_falls_back_to_vcycle(gpu):
    """A network whose output is NaN (a poisoned head bias): inside M_VU every
    affected right-hand side falls back to e0 = 0, i.e. M_VU = V_SL, so
    CNN-FGMRES(10) converges like MG-GMRES(10) instead of breaking down."""
    n = 64
    med = medium(n, n, seed=20)
    H = setup(med)
    net, theta = small_net(seed=13)
    theta = theta.astype(np.float32)
    theta[-1] = np.nan                     # bias of the head's second output channel
    api.cnn_set_params(net, theta)
    b = rand_c((3, n, n), 8).astype(np.complex64)
    bt = torch.tensor(b, device="cuda")
    e = api.cnn_precond_apply(net, H, bt).cpu().numpy()
    assert np.isnan(e).any()               # the raw preconditioner keeps the NaN
    x, it, rr, st, code = api.helm_solve(H, bt, tol=1e-6, precond="cnn_vu", maxit=800, net=net, restart=10)
    _, itm, _, _, cm = api.helm_solve(H, bt, tol=1e-6, precond="mg", maxit=800, restart=10)
    print("poisoned network: cnn_vu iterations", it, "mg(10)", itm)
    assert code == 0 and np.all(st == 0) and cm == 0
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    assert np.all(op.relres(coef, x.cpu().numpy(), b.astype(np.complex128), med.h, med.h) <= 1e-6)
    assert np.all(np.abs(it - itm) <= 2)


def test_trained_network_beats_multigrid(gpu):
    """What the learned part gains: a network trained by the library's own
    kernels on eq. (4.3) pairs of a 64 x 64 layered medium makes CNN-FGMRES(10)
    need fewer iterations than MG-GMRES(20) on surface sources of that medium
    (the sources are not training data), and fewer than the untrained network."""
    from paper_2405_17696_amd import synth
    n = 64
    rng = np.random.default_rng(61)
    c = synth.velocity_layered(n, n, rng)
    med = synth.medium_from_velocity(c)
    med.kappa2 = np.asarray(med.kappa2, np.float32).astype(np.float64)
    med.gamma = np.asarray(med.gamma, np.float32).astype(np.float64)
    H = setup(med)
    src = synth.point_sources(n, n, synth.surface_positions(n, 8), h=med.h)
    b = torch.tensor(src, dtype=torch.complex64, device="cuda")
    net = api.cnn_create(seed=1)
    _, it0, _, _, c0 = api.helm_solve(H, b, tol=1e-6, precond="cnn_vu", maxit=1000, net=net, restart=10)
    _, itm, _, _, cm = api.helm_solve(H, b, tol=1e-6, precond="mg", maxit=1000, restart=20)
    print("training 64x64 network", flush=True)
    for rnd, lr in enumerate((1e-3, 1e-3, 5e-4, 2.5e-4)):
        api.cnn_precond_train(net, H, npairs=1024, batch=16, steps=500, lr=lr, seed=100 + rnd)
    x, it1, rr, st, c1 = api.helm_solve(H, b, tol=1e-6, precond="cnn_vu", maxit=1000, net=net, restart=10)
    print("iterations: untrained", it0.mean(), "trained", it1.mean(), "MG-GMRES(20)", itm.mean())
    assert c0 == 0 and cm == 0 and c1 == 0
    assert it1.mean() < itm.mean() and it1.mean() < it0.mean()


def test_pretrain_then_retrain_lowers_iterations(gpu):
    """The paper's regime at 64 x 64 (Sec. 4.1-4.2): a network pre-trained on
    random linear slowness-squared media, then retrained on a layered medium
    it has not seen, needs fewer CNN-FGMRES(10) iterations on that medium's
    surface sources after the retraining than before it."""
    from paper_2405_17696_amd import synth, training
    n = 64
    net = api.cnn_create(seed=1)
    print("pre-training on linear media at 64x64", flush=True)
    info = training.pretrain(net, 2000, grids=((n, n),), ppw_range=(10.0, 10.0), pairs_per_medium=1024,
                             steps_per_medium=250, halvings=(125, 375, 1000, 1500), seed=21)
    c = synth.velocity_layered(n, n, np.random.default_rng(62))
    med = synth.medium_from_velocity(c)
    k2 = torch.tensor(np.asarray(med.kappa2, np.float32), device="cuda")
    g = torch.tensor(np.asarray(med.gamma, np.float32), device="cuda")
    b = torch.tensor(synth.point_sources(n, n, synth.surface_positions(n, 8), h=med.h), dtype=torch.complex64,
                     device="cuda")
    before = training.solve_iterations(net, k2, g, med.omega, med.h, b)
    hist, dsz, sec = training.retrain(net, k2, g, med.omega, med.h, alg2=False, npairs=1024, steps=200, lr=1e-4,
                                      seed=22)
    after = training.solve_iterations(net, k2, g, med.omega, med.h, b)
    mg = training.solve_iterations(None, k2, g, med.omega, med.h, b, precond="mg", restart=20)
    print("pre-training", info["seconds"], "s; iterations before", before, "after", after, "MG-GMRES(20)", mg)
    assert before["converged"] == after["converged"] == 8
    assert after["iters_mean"] < before["iters_mean"]
