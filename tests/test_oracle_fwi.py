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


# ---------------------------------------------------------------- regularisers (eq. 5.1, 5.2)
def _grad_matrix(nz, nx, hx, hz):
    """The nodal-grid gradient as an explicit matrix, one row per edge, built
    entry by entry: x-edges (i, k)-(i, k+1) first, then z-edges (i, k)-(i+1, k)."""
    rows = []
    for i in range(nz):
        for k in range(nx - 1):
            r = np.zeros(nz * nx)
            r[i * nx + k + 1] = 1.0 / hx
            r[i * nx + k] = -1.0 / hx
            rows.append(r)
    for i in range(nz - 1):
        for k in range(nx):
            r = np.zeros(nz * nx)
            r[(i + 1) * nx + k] = 1.0 / hz
            r[i * nx + k] = -1.0 / hz
            rows.append(r)
    return np.array(rows)


def test_regularisers_brute_force_matrices():
    nz, nx, hx, hz = 4, 5, 0.7, 1.3
    rng = np.random.default_rng(40)
    m, mref = rng.standard_normal((nz, nx)), rng.standard_normal((nz, nx))
    G = _grad_matrix(nz, nx, hx, hz)
    Lap = -G.T @ G
    d = (m - mref).ravel()
    r_diff, g_diff = fwi.regulariser(fwi.REG_DIFF, m, mref, hx, hz)
    r_high, g_high = fwi.regulariser(fwi.REG_HIGH, m, mref, hx, hz)
    assert abs(r_diff - np.sum((G @ d) ** 2)) <= 1e-12 * r_diff
    assert abs(r_high - np.sum((Lap @ d) ** 2)) <= 1e-12 * r_high
    assert np.allclose(g_diff.ravel(), 2 * G.T @ G @ d, rtol=1e-12, atol=1e-12 * np.abs(g_diff).max())
    assert np.allclose(g_high.ravel(), 2 * Lap.T @ Lap @ d, rtol=1e-12, atol=1e-12 * np.abs(g_high).max())
    v = rng.standard_normal((nz, nx))
    assert np.allclose(fwi.reg_hessvec(fwi.REG_DIFF, v, hx, hz).ravel(), 2 * G.T @ G @ v.ravel(), atol=1e-10)
    assert np.allclose(fwi.reg_hessvec(fwi.REG_HIGH, v, hx, hz).ravel(), 2 * Lap @ Lap @ v.ravel(), atol=1e-8)
    # interior rows of Lap are the 5-point stencil (sum of neighbours - 4 u over h^2 for hx = hz)
    i, k = 2, 2
    row = Lap[i * nx + k].reshape(nz, nx)
    assert abs(row[i, k] + 2 / hx ** 2 + 2 / hz ** 2) < 1e-12
    assert abs(row[i, k - 1] - 1 / hx ** 2) < 1e-12 and abs(row[i - 1, k] - 1 / hz ** 2) < 1e-12


def test_regularisers_closed_forms():
    """A linear ramp has constant differences (R_diff closed form, R_high = 0
    in the interior rows ... and everywhere, since the ends see one-sided
    constant differences that cancel); a product of cosine modes
    cos(pi q (k + 1/2) / nx) cos(pi p (i + 1/2) / nz) is an eigenvector of the
    nodal Laplacian with eigenvalue -lam, lam = 4/hx^2 sin^2(pi q / 2nx) +
    4/hz^2 sin^2(pi p / 2nz), so R_diff = lam ||d||^2 and R_high = lam^2 ||d||^2;
    constants cost nothing."""
    nz, nx, hx, hz = 9, 12, 0.5, 0.8
    i = np.arange(nz)[:, None] * np.ones((1, nx))
    k = np.arange(nx)[None, :] * np.ones((nz, 1))
    a, b = 0.3, -0.7
    ramp = a * k * hx + b * i * hz
    r, _ = fwi.regulariser(fwi.REG_DIFF, ramp, 0 * ramp, hx, hz)
    assert abs(r - (a * a * nz * (nx - 1) + b * b * (nz - 1) * nx)) <= 1e-12 * r
    for p, q in ((1, 1), (3, 5), (nz - 1, nx - 1), (0, 4)):
        d = np.cos(np.pi * q * (k + 0.5) / nx) * np.cos(np.pi * p * (i + 0.5) / nz)
        lam = 4 / hx ** 2 * np.sin(np.pi * q / (2 * nx)) ** 2 + 4 / hz ** 2 * np.sin(np.pi * p / (2 * nz)) ** 2
        assert np.allclose(fwi.reg_laplacian(d, hx, hz), -lam * d, atol=1e-12 * lam)
        rd, _ = fwi.regulariser(fwi.REG_DIFF, d + 2.0, 2.0 * np.ones_like(d), hx, hz)
        rh, _ = fwi.regulariser(fwi.REG_HIGH, d + 2.0, 2.0 * np.ones_like(d), hx, hz)
        nd = np.sum(d * d)
        assert abs(rd - lam * nd) <= 1e-10 * lam * nd and abs(rh - lam ** 2 * nd) <= 1e-10 * lam ** 2 * nd
    for kind in (fwi.REG_HIGH, fwi.REG_DIFF):
        r, g = fwi.regulariser(kind, np.full((nz, nx), 3.0), np.full((nz, nx), 1.0), hx, hz)
        assert r == 0.0 and np.all(g == 0)


@pytest.mark.parametrize("kind", [fwi.REG_HIGH, fwi.REG_DIFF])
def test_regulariser_gradient_and_hessian_by_differences(kind):
    nz, nx, hx, hz = 10, 13, 0.4, 0.6
    rng = np.random.default_rng(41 + kind)
    m, mref = rng.standard_normal((nz, nx)), rng.standard_normal((nz, nx))
    r0, g = fwi.regulariser(kind, m, mref, hx, hz)
    for t in range(4):
        v = rng.standard_normal((nz, nx))
        eps = 1e-4
        rp, gp = fwi.regulariser(kind, m + eps * v, mref, hx, hz)
        rm, gm = fwi.regulariser(kind, m - eps * v, mref, hx, hz)
        fd = (rp - rm) / (2 * eps)
        assert abs(fd - np.sum(g * v)) <= 1e-7 * abs(fd)
        hv = fwi.reg_hessvec(kind, v, hx, hz)
        assert np.allclose((gp - gm) / (2 * eps), hv, rtol=1e-6, atol=1e-6 * np.abs(hv).max())
        assert np.sum(v * hv) >= 0
    u, w = rng.standard_normal((nz, nx)), rng.standard_normal((nz, nx))
    lhs, rhs = np.sum(u * fwi.reg_hessvec(kind, w, hx, hz)), np.sum(w * fwi.reg_hessvec(kind, u, hx, hz))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


def test_regularised_gn_cg_and_step():
    """The regularised Gauss-Newton matrix (Re(J^H J) + alpha nabla^2 R + damping I)
    assembled densely: CG reaches its solution; the step's gradient is
    dPhi/dm + alpha dR/dm (central differences of Phi + alpha R)."""
    k2, gamma, omegas, h, src, rec, dobs = small_problem(nz=8, nx=8, nsrc=2, nrec=3)
    n = k2.size
    damping = 1e-2
    mref = k2 * (1 + 0.02 * np.random.default_rng(42).standard_normal(k2.shape))
    # weights that put alpha nabla^2 R on the scale of Re(J^H J) (largest eigenvalue ~70 here)
    for kind, alpha in ((fwi.REG_HIGH, 1e-8), (fwi.REG_DIFF, 1e-4)):
        cols = []
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1.0
            ej = e.reshape(k2.shape)
            cols.append((fwi.gn_hessvec(k2, gamma, omegas, h, src, rec, ej)
                         + alpha * fwi.reg_hessvec(kind, ej, h)).ravel())
        A = np.array(cols).T + damping * np.eye(n)
        b = np.random.default_rng(43).standard_normal(k2.shape)
        x, _ = fwi.gn_cg(k2, gamma, omegas, h, src, rec, b, damping, 3 * n, reg=kind, alpha=alpha)
        xd = np.linalg.solve(A, b.ravel())
        assert np.linalg.norm(x.ravel() - xd) <= 1e-6 * np.linalg.norm(xd)
        m_new, phi, norms, rv, g = fwi.gn_step(k2, gamma, omegas, h, src, rec, dobs, damping, 4, 1.0, reg=kind,
                                               alpha=alpha, m_ref=mref)
        obj = lambda m: (fwi.misfit(m, gamma, omegas, h, src, rec, dobs)
                         + alpha * fwi.regulariser(kind, m, mref, h)[0])
        v = np.random.default_rng(44).standard_normal(k2.shape) * k2
        eps = 1e-5
        fd = (obj(k2 + eps * v) - obj(k2 - eps * v)) / (2 * eps)
        assert abs(fd - np.sum(g * v)) <= 1e-5 * abs(fd)
        assert rv == fwi.regulariser(kind, k2, mref, h)[0]
        # the step is a descent direction of the regularised objective
        assert np.sum((m_new - k2) * g) < 0


def test_resample_bilinear():
    """Identity on the same grid, exact on fields linear in the coordinates
    (bilinear interpolation reproduces them), a hand-computed midpoint."""
    rng = np.random.default_rng(45)
    f = rng.standard_normal((9, 13))
    assert np.allclose(fwi.resample_bilinear(f, 9, 13), f, atol=1e-15)
    Z, X = np.meshgrid(np.arange(9.0), np.arange(13.0), indexing="ij")
    lin = 0.3 + 0.5 * Z - 0.25 * X + 0.1 * Z * X          # bilinear, so reproduced exactly
    r = fwi.resample_bilinear(lin, 17, 7)
    z = np.arange(17) * 8 / 16
    x = np.arange(7) * 12 / 6
    Zr, Xr = np.meshgrid(z, x, indexing="ij")
    assert np.allclose(r, 0.3 + 0.5 * Zr - 0.25 * Xr + 0.1 * Zr * Xr, atol=1e-12)
    # 3 x 3 -> 5 x 5: node (1, 1) of the output sits at (0.5, 0.5): mean of the four corners
    g = rng.standard_normal((3, 3))
    assert abs(fwi.resample_bilinear(g, 5, 5)[1, 1] - g[:2, :2].mean()) < 1e-14
