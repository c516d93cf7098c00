"""Pins of the oracle's misfit gradient (eq. 3.5, 3.10, 4.8) against central
finite differences of the misfit, a dot-product test between independently
computed Born and adjoint-Born operators, and special cases (CPU only).  The
simultaneous-source misfit (eq. 3.6-3.8) is pinned by its identity-encoding
case, by the exact average over all sign vectors, and by finite differences."""
import numpy as np
import pytest

from oracle import fwi
from paper_2405_17696_amd import synth


def small_problem(nz=20, nx=24, seed=3, nsrc=3, nrec=5):
    rng = np.random.default_rng(seed)
    c = synth.velocity_grf(nz, nx, rng)
    # a thin absorbing layer so that gamma != 0 on part of the grid
    gamma = synth.abl_gamma(nz, nx, width=5)
    k2 = synth.kappa2_from_velocity(c)
    h = synth.H_DEFAULT
    omegas = [synth.omega_for_ppw(float(c.min()), p, h) for p in (12.0, 8.0)]
    src = 2 * nx + np.array([6, 11, 17])[:nsrc]
    rec = 3 * nx + np.linspace(5, nx - 6, nrec).astype(int)
    # observed data from a perturbed model
    kt = k2 * (1.0 + 0.05 * synth.grf(nz, nx, np.random.default_rng(seed + 1), corr_len=4.0))
    dobs = fwi.forward_data(kt, gamma, omegas, h, src, rec)
    return k2, gamma, omegas, h, src, rec, dobs


def test_gradient_matches_central_differences():
    k2, gamma, omegas, h, src, rec, dobs = small_problem()
    phi, g = fwi.misfit_and_grad(k2, gamma, omegas, h, src, rec, dobs)
    assert phi > 0
    rng = np.random.default_rng(11)
    for t in range(4):
        d = rng.standard_normal(k2.shape)
        eps = 1e-3 * np.abs(k2).max() / np.abs(d).max()
        fp = fwi.misfit(k2 + eps * d, gamma, omegas, h, src, rec, dobs)
        fm = fwi.misfit(k2 - eps * d, gamma, omegas, h, src, rec, dobs)
        fd = (fp - fm) / (2 * eps)
        assert abs(np.sum(g * d) - fd) <= 1e-5 * abs(fd), (t, np.sum(g * d), fd)


def test_gradient_in_absorbing_layer_nodes():
    # directions supported only where gamma > 0: a dropped (1 - i gamma) fails here
    k2, gamma, omegas, h, src, rec, dobs = small_problem()
    _, g = fwi.misfit_and_grad(k2, gamma, omegas, h, src, rec, dobs)
    d = np.where(gamma > 0.2, 1.0, 0.0) * np.random.default_rng(5).standard_normal(k2.shape)
    eps = 1e-3 * np.abs(k2).max()
    fd = (fwi.misfit(k2 + eps * d, gamma, omegas, h, src, rec, dobs)
          - fwi.misfit(k2 - eps * d, gamma, omegas, h, src, rec, dobs)) / (2 * eps)
    assert abs(np.sum(g * d) - fd) <= 1e-5 * abs(fd)


def test_single_node_derivative_brute_force():
    k2, gamma, omegas, h, src, rec, dobs = small_problem(nz=12, nx=14, nsrc=2, nrec=3)
    _, g = fwi.misfit_and_grad(k2, gamma, omegas, h, src, rec, dobs)
    for (i, k) in ((5, 7), (2, 3), (9, 1)):
        e = np.zeros_like(k2)
        e[i, k] = 1.0
        eps = 1e-4 * k2[i, k]
        fd = (fwi.misfit(k2 + eps * e, gamma, omegas, h, src, rec, dobs)
              - fwi.misfit(k2 - eps * e, gamma, omegas, h, src, rec, dobs)) / (2 * eps)
        assert abs(g[i, k] - fd) <= 1e-5 * abs(fd) + 1e-12 * np.abs(g).max()


def test_born_dot_product():
    k2, gamma, omegas, h, src, rec, dobs = small_problem()
    rng = np.random.default_rng(21)
    dm = rng.standard_normal(k2.shape)
    dd = rng.standard_normal(dobs.shape) + 1j * rng.standard_normal(dobs.shape)
    lhs = np.real(np.vdot(dd, fwi.born(k2, gamma, omegas, h, src, rec, dm)))
    rhs = np.sum(fwi.born_adjoint(k2, gamma, omegas, h, src, rec, dd) * dm)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_gradient_is_adjoint_born_of_residual():
    # the gradient's conjugation solve (eq. 4.8) against SuperLU's H^H solve
    k2, gamma, omegas, h, src, rec, dobs = small_problem()
    _, g = fwi.misfit_and_grad(k2, gamma, omegas, h, src, rec, dobs)
    res = fwi.forward_data(k2, gamma, omegas, h, src, rec) - dobs
    ga = fwi.born_adjoint(k2, gamma, omegas, h, src, rec, res)
    assert np.linalg.norm(g - ga) <= 1e-10 * np.linalg.norm(ga)


def test_zero_residual_gives_zero_misfit_and_gradient():
    k2, gamma, omegas, h, src, rec, _ = small_problem()
    d = fwi.forward_data(k2, gamma, omegas, h, src, rec)
    phi, g = fwi.misfit_and_grad(k2, gamma, omegas, h, src, rec, d)
    assert phi == pytest.approx(0.0, abs=1e-20)
    assert np.abs(g).max() == 0.0


def test_point_source_scaling():
    g = fwi.point_source_rhs((4, 5), [7], 0.5, 0.25)
    assert g.shape == (1, 4, 5)
    assert g[0, 1, 2] == 8.0 and np.count_nonzero(g) == 1


def test_encoded_with_identity_is_unencoded_over_p():
    # X = I (p = ns): the encoded sources are the point sources themselves
    k2, gamma, omegas, h, src, rec, dobs = small_problem()
    phi, g = fwi.misfit_and_grad(k2, gamma, omegas, h, src, rec, dobs)
    p = len(src)
    phx, gx = fwi.misfit_and_grad_encoded(k2, gamma, omegas, h, src, rec, dobs, np.eye(p))
    assert abs(phx * p - phi) <= 1e-12 * phi
    assert np.abs(gx * p - g).max() <= 1e-10 * np.abs(g).max()


def test_encoded_average_over_all_sign_vectors_is_exact():
    # with every one of the 2^ns sign vectors as a column, (1/p) X X^T = I
    # exactly, so the trace estimator returns the misfit and gradient exactly
    k2, gamma, omegas, h, src, rec, dobs = small_problem()
    ns = len(src)
    X = np.array([[1.0 if (j >> s) & 1 else -1.0 for j in range(2 ** ns)] for s in range(ns)])
    assert np.allclose(X @ X.T / X.shape[1], np.eye(ns))
    phi, g = fwi.misfit_and_grad(k2, gamma, omegas, h, src, rec, dobs)
    phx, gx = fwi.misfit_and_grad_encoded(k2, gamma, omegas, h, src, rec, dobs, X)
    assert abs(phx - phi) <= 1e-12 * phi
    assert np.abs(gx - g).max() <= 1e-10 * np.abs(g).max()
    # one sign vector alone is not the misfit: the estimator is random
    ph1, _ = fwi.misfit_and_grad_encoded(k2, gamma, omegas, h, src, rec, dobs, X[:, :1])
    assert abs(ph1 - phi) > 1e-6 * phi


def test_encoded_gradient_central_differences():
    k2, gamma, omegas, h, src, rec, dobs = small_problem()
    X = np.where(np.random.default_rng(8).random((len(src), 2)) < 0.5, -1.0, 1.0)
    _, g = fwi.misfit_and_grad_encoded(k2, gamma, omegas, h, src, rec, dobs, X)
    rng = np.random.default_rng(12)
    for t in range(3):
        d = rng.standard_normal(k2.shape)
        eps = 1e-3 * np.abs(k2).max() / np.abs(d).max()
        fp = fwi.misfit_and_grad_encoded(k2 + eps * d, gamma, omegas, h, src, rec, dobs, X)[0]
        fm = fwi.misfit_and_grad_encoded(k2 - eps * d, gamma, omegas, h, src, rec, dobs, X)[0]
        fd = (fp - fm) / (2 * eps)
        assert abs(np.sum(g * d) - fd) <= 1e-5 * abs(fd), (t, np.sum(g * d), fd)


def test_born_is_the_derivative_of_the_data():
    # J dm against central differences of the forward data (the sign of eq. 3.10 decided here too)
    k2, gamma, omegas, h, src, rec, _ = small_problem()
    dm = np.random.default_rng(31).standard_normal(k2.shape)
    jdm = fwi.born(k2, gamma, omegas, h, src, rec, dm)
    eps = 1e-4 * np.abs(k2).max() / np.abs(dm).max()
    fd = (fwi.forward_data(k2 + eps * dm, gamma, omegas, h, src, rec)
          - fwi.forward_data(k2 - eps * dm, gamma, omegas, h, src, rec)) / (2 * eps)
    assert np.linalg.norm(jdm - fd) <= 1e-6 * np.linalg.norm(fd)


def test_gn_hessvec_symmetric_positive_and_norm_of_jv():
    k2, gamma, omegas, h, src, rec, _ = small_problem()
    rng = np.random.default_rng(32)
    v, w = rng.standard_normal(k2.shape), rng.standard_normal(k2.shape)
    hv = fwi.gn_hessvec(k2, gamma, omegas, h, src, rec, v)
    hw = fwi.gn_hessvec(k2, gamma, omegas, h, src, rec, w)
    assert abs(np.sum(w * hv) - np.sum(v * hw)) <= 1e-10 * abs(np.sum(v * hw))
    jv = fwi.born(k2, gamma, omegas, h, src, rec, v)
    assert abs(np.sum(v * hv) - np.linalg.norm(jv) ** 2) <= 1e-10 * np.linalg.norm(jv) ** 2


def test_gn_cg_reaches_the_dense_solution():
    # tiny grid: the damped Gauss-Newton matrix assembled column by column from
    # gn_hessvec and solved densely; CG with as many steps as unknowns reaches it
    k2, gamma, omegas, h, src, rec, _ = small_problem(nz=8, nx=8, nsrc=2, nrec=3)
    n = k2.size
    damping = 1e-3
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(fwi.gn_hessvec(k2, gamma, omegas, h, src, rec, e.reshape(k2.shape)).ravel())
    A = np.array(cols).T + damping * np.eye(n)
    assert np.abs(A - A.T).max() <= 1e-10 * np.abs(A).max()
    b = np.random.default_rng(33).standard_normal(k2.shape)
    x_dense = np.linalg.solve(A, b.ravel())
    x, norms = fwi.gn_cg(k2, gamma, omegas, h, src, rec, b, damping, 3 * n)
    assert np.linalg.norm(x.ravel() - x_dense) <= 1e-6 * np.linalg.norm(x_dense)
    assert abs(norms[0] - np.linalg.norm(b)) <= 1e-12 * norms[0]
    # after k steps the reported residual is b - A x_k
    x3, n3 = fwi.gn_cg(k2, gamma, omegas, h, src, rec, b, damping, 3)
    assert abs(n3[-1] - np.linalg.norm(b.ravel() - A @ x3.ravel())) <= 1e-8 * n3[0]


def test_gauss_newton_frequency_continuation_reduces_misfit_and_model_error():
    # the driver recovers part of the perturbation the data came from: the
    # misfit of every window falls from one step to the next, and the model
    # moves towards the true one
    nz, nx = 20, 24
    rng = np.random.default_rng(3)
    c = synth.velocity_grf(nz, nx, rng)
    gamma = synth.abl_gamma(nz, nx, width=5)
    k2 = synth.kappa2_from_velocity(c)
    h = synth.H_DEFAULT
    omegas = [synth.omega_for_ppw(float(c.min()), p, h) for p in (16.0, 12.0, 10.0)]
    src = 2 * nx + np.array([4, 9, 14, 19])
    rec = 3 * nx + np.arange(3, nx - 3)
    kt = k2 * (1.0 + 0.03 * synth.grf(nz, nx, np.random.default_rng(4), corr_len=5.0))
    dobs = fwi.forward_data(kt, gamma, omegas, h, src, rec)
    m, hist = fwi.frequency_continuation(k2, gamma, omegas, h, src, rec, dobs, cycles=[(0, 2)], window=1,
                                         gn_iters=2, damping=1e-3, cg_iters=8, mu=1.0)
    assert len(hist) == 6
    for w in range(3):                      # two steps per window: the second starts lower
        assert hist[2 * w + 1] < hist[2 * w]
    assert np.linalg.norm(m - kt) < np.linalg.norm(k2 - kt)
