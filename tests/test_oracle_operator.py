"""Pins of the oracle's operator, multigrid, Krylov and RNG parts against
definitions, closed forms and independent library routines (CPU only)."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import scipy.special as sps

from helpers import medium, rand_c, relerr
from oracle import krylov as kr
from oracle import multigrid as mg
from oracle import operator as op
from oracle import philox
from paper_2405_17696_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- operator (eq. 3.1-3.2)
@pytest.mark.parametrize("nz,nx,hz", [(5, 7, None), (16, 16, None), (9, 12, 0.02)])
def test_dense_bruteforce_equals_sparse_and_stencil(nz, nx, hz):
    med = medium(nz, nx, seed=nz + nx)
    hz = med.h if hz is None else hz
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    D = op.dense_bruteforce(coef, med.h, hz)
    S = op.assemble(coef, med.h, hz).toarray()
    assert np.array_equal(D, S)
    u = rand_c((nz, nx), 1)
    assert relerr(op.apply(coef, u, med.h, hz).ravel(), D @ u.ravel()) < 1e-14


def test_sine_eigenvectors_closed_form():
    nz, nx, h, hz = 12, 15, 0.01, 0.013
    m, omega = 0.3, 40.0
    coef = op.helmholtz_coef(np.full((nz, nx), m), np.zeros((nz, nx)), omega)
    i = np.arange(nz)[:, None]
    k = np.arange(nx)[None, :]
    for p, q in ((1, 1), (3, 7), (nz, nx), (5, 2)):
        v = np.sin(np.pi * p * (i + 1) / (nz + 1)) * np.sin(np.pi * q * (k + 1) / (nx + 1))
        lam = (4 / hz ** 2) * np.sin(np.pi * p / (2 * (nz + 1))) ** 2 + \
              (4 / h ** 2) * np.sin(np.pi * q / (2 * (nx + 1))) ** 2 - omega ** 2 * m
        assert relerr(op.apply(coef, v, h, hz), lam * v) < 1e-12


def test_complex_symmetry_and_adjoint_identity():
    med = medium(20, 24, seed=3)
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    A = op.assemble(coef, med.h, med.h)
    assert abs(A - A.T).max() == 0
    u, v = rand_c((20 * 24,), 1), rand_c((20 * 24,), 2)
    lhs = np.vdot(A @ u, v)
    rhs = np.vdot(u, A.conj().T @ v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # adjoint by conjugation (eq. 4.8): H^* x = b  <=>  H conj(x) = conj(b)
    b = rand_c((20 * 24,), 3)
    x_adj = spla.spsolve(A.conj().T.tocsc(), b)
    x_conj = np.conj(op.DirectSolver(A).solve(np.conj(b)))
    assert relerr(x_conj, x_adj) < 1e-10


def test_manufactured_solution_direct():
    med = medium(40, 36, seed=4)
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    u = rand_c((40, 36), 5)
    q = op.apply(coef, u, med.h, med.h)
    x = op.DirectSolver(op.assemble(coef, med.h, med.h)).solve(q.ravel()).reshape(40, 36)
    assert relerr(x, u) < 1e-10


@pytest.mark.slow
def test_greens_function_second_order():
    """Constant medium, 4-sided layer 3 wavelengths thick, centre source e_s/h^2:
    compare with the outgoing free-space Green's function -(i/4) H0^(2)(k r)
    2-2.5 wavelengths from the source; the error falls ~4x from 20 to 40 ppw."""
    c, f = 2.0, 4.0
    lam = c / f
    means = []
    for ppw in (20, 40):
        h = lam / ppw
        L = 3 * ppw
        n = 5 * ppw + 2 * L
        k2 = np.full((n, n), 1 / c ** 2)
        g = synth.abl_gamma(n, n, width=L, gmax=1.0, sides="lrbt")
        omega = 2 * np.pi * f
        s = n // 2
        b = np.zeros(n * n, complex)
        b[s * n + s] = 1 / h ** 2
        u = op.DirectSolver(op.assemble_helmholtz(k2, g, omega, h)).solve(b).reshape(n, n)
        errs = []
        for d in np.linspace(2, 2.5, 6):
            for ang in (0, np.pi / 4, 0.3):
                di, dk = int(round(d * ppw * np.sin(ang))), int(round(d * ppw * np.cos(ang)))
                G = -0.25j * sps.hankel2(0, (omega / c) * h * np.hypot(di, dk))
                errs.append(abs(u[s + di, s + dk] - G) / abs(G))
        means.append(np.mean(errs))
    assert means[1] < 0.025
    assert means[0] / means[1] > 3.0


# ---------------------------------------------------------------- Krylov
def test_gmres_matches_direct():
    med = medium(32, 32, seed=8)
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    A = op.assemble(coef, med.h, med.h)
    b = rand_c((32 * 32,), 9)
    xs = op.DirectSolver(A).solve(b)
    V = mg.VCycle(med.kappa2, med.gamma, med.omega, med.h)
    res = kr.gmres(lambda v: A @ v, b, M=lambda v: V(v.reshape(32, 32)).ravel(), restart=20, tol=1e-12,
                   maxit=2000)
    assert res.converged
    assert relerr(res.x, xs) < 1e-9


def test_gmres_one_iteration_closed_form():
    """One GMRES step from x0: z = M(r0/||r0||), w = H z, y = w^H r0 / w^H w."""
    med = medium(24, 24, seed=10)
    coef = op.helmholtz_coef(med.kappa2, med.gamma, med.omega)
    A = op.assemble(coef, med.h, med.h)
    V = mg.VCycle(med.kappa2, med.gamma, med.omega, med.h)
    M = lambda v: V(v.reshape(24, 24)).ravel()
    b, x0 = rand_c((576,), 1), rand_c((576,), 2)
    r0 = b - A @ x0
    z = M(r0 / np.linalg.norm(r0))
    w = A @ z
    y = np.vdot(w, r0) / np.vdot(w, w)
    res = kr.fgmres(lambda v: A @ v, b, M=M, x0=x0, max_iters_exact=1)
    assert relerr(res.x, x0 + y * z) < 1e-12


def test_gmres_equals_scipy_unpreconditioned():
    """Fixed-iteration GMRES minimises the residual over the Krylov space:
    compare with a least-squares solve on an explicitly built Krylov basis."""
    med = medium(12, 12, seed=12)
    A = op.assemble(op.helmholtz_coef(med.kappa2, med.gamma, med.omega), med.h, med.h).toarray()
    b = rand_c((144,), 3)
    k = 6
    K = np.stack([np.linalg.matrix_power(A, i) @ b for i in range(k)], axis=1)
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
    res = kr.fgmres(lambda v: A @ v, b, max_iters_exact=k)
    assert relerr(res.x, Q @ y) < 1e-8


# ---------------------------------------------------------------- multigrid (eq. 3.12, Sec. 3.4)
def _dense(fn, shape_in):
    n = int(np.prod(shape_in))
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1
        cols.append(np.asarray(fn(e.reshape(shape_in))).ravel())
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("nz,nx", [(8, 8), (9, 6), (7, 11)])
def test_prolongation_is_4_restriction_transpose(nz, nx):
    R = _dense(mg.restrict_fw, (nz, nx))
    cz, cxn = mg.coarse_shape(nz, nx)
    P = _dense(lambda e: mg.prolong_bilinear(e, (nz, nx)), (cz, cxn))
    assert np.allclose(P, 4 * R.T, atol=1e-15)


def test_transfer_exactness_on_linear_functions():
    nz, nx = 17, 21
    i = np.arange(nz)[:, None] * np.ones((1, nx))
    k = np.arange(nx)[None, :] * np.ones((nz, 1))
    f = 0.3 + 0.7 * i - 0.2 * k
    fc = mg.restrict_fw(f)
    cz, cxn = fc.shape
    I = np.arange(cz)[:, None]
    J = np.arange(cxn)[None, :]
    exact = 0.3 + 0.7 * (2 * I + 1) - 0.2 * (2 * J + 1)      # coarse node I on fine node 2I+1
    assert np.allclose(fc[:-1, :-1], exact[:-1, :-1], atol=1e-12)   # away from the far boundary: exact
    up = mg.prolong_bilinear(exact + 0 * I, (nz, nx))
    assert np.allclose(up[1:-1, 1:-1], f[1:-1, 1:-1], atol=1e-12)


def test_coarse_polynomial_is_gmres_polynomial():
    """p(P) v0 from the Leja-ordered harmonic Ritz roots equals what fixed-
    iteration GMRES returns for the start vector v0 (same Krylov space)."""
    med = medium(64, 64, seed=14)
    V = mg.VCycle(med.kappa2, med.gamma, med.omega, med.h, coarse_degree=12)
    L = V.levels[-1]
    n = L.coef.size
    v0 = philox.complex_uniform(n, mg.COARSE_KEY)
    v0 = v0 / np.linalg.norm(v0)
    xp = mg.apply_root_polynomial(L, V.roots, v0.reshape(L.coef.shape)).ravel()
    res = kr.fgmres(lambda v: L.apply(v.reshape(L.coef.shape)).ravel(), v0, max_iters_exact=12)
    assert relerr(xp, res.x) < 1e-6


def test_vcycle_linear_and_smoother_fixed_point():
    med = medium(48, 40, seed=15)
    V = mg.VCycle(med.kappa2, med.gamma, med.omega, med.h)
    f1, f2 = rand_c((48, 40), 1), rand_c((48, 40), 2)
    a, b = 0.3 - 1.2j, 2.0 + 0.1j
    assert relerr(V(a * f1 + b * f2), a * V(f1) + b * V(f2)) < 1e-12
    L0 = V.levels[0]
    e = rand_c((48, 40), 3)
    f = L0.apply(e)
    assert relerr(V.jacobi(L0, e, f, 3), e) < 1e-13


@pytest.mark.parametrize("ppw", [40.0, 10.0])
def test_vcycle_contracts_as_stationary_iteration(ppw):
    """Iterating e <- e + V(f - P e) drives the shifted-Laplacian residual down
    (contraction < 0.6 per cycle at 10 and 40 points per wavelength)."""
    med = medium(64, 64, seed=16, ppw=ppw)
    V = mg.VCycle(med.kappa2, med.gamma, med.omega, med.h)
    L0 = V.levels[0]
    f = rand_c((64, 64), 4)
    e = np.zeros_like(f)
    for _ in range(8):
        e = e + V(f - L0.apply(e))
    assert np.linalg.norm(f - L0.apply(e)) / np.linalg.norm(f) < 0.6 ** 8


def test_coarse_boundary_stencil_consistent():
    """The non-uniform far-boundary stencil is exact on quadratics vanishing at
    the boundary node, and reduces to the regular stencil when delta = H."""
    H, d = 0.2, 0.05
    nx = 6
    xs = H * np.arange(1, nx + 1)              # nodes; boundary at xs[-1] + d
    xb = xs[-1] + d
    u = (xb - xs) * (xs + 0.3)                 # u(xb) = 0, u'' = -2
    L = Level1D = mg.Level(np.zeros((1, nx)), H, 1.0, d, 1.0)
    lap_x = L.dgx * u - L.cwx * np.r_[0.0, u[:-1]] - L.cex * np.r_[u[1:], 0.0]
    assert abs(lap_x[-1] - 2.0) < 1e-9
    L2 = mg.Level(np.zeros((3, 4)), 0.1, 0.1)
    assert np.allclose(L2.dgx, 2 / 0.01) and np.allclose(L2.cwx, 1 / 0.01)


# ---------------------------------------------------------------- Philox
def test_philox_known_answers():
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        rows = [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(t, 16) for t in r]
        out = philox.philox4x32(np.array(w[:4], dtype=np.uint64), (w[4], w[5]))
        assert [int(v) for v in out] == w[6:]


def test_philox_normal_moments():
    z = philox.complex_normal(200000, (1, 2))
    assert abs(np.mean(np.abs(z) ** 2) - 1.0) < 0.01
    assert abs(np.mean(z)) < 0.01


# ---------------------------------------------------------------- shifted Laplacian (eq. 3.12)
def _sine_spectrum(nz, nx, hx, hz):
    """Eigenvalues of -Lap_h with Dirichlet-0 ghosts (sine modes), independent of
    the sparse assembly."""
    p = np.arange(1, nz + 1)[:, None]
    q = np.arange(1, nx + 1)[None, :]
    return ((4 / hz ** 2) * np.sin(np.pi * p / (2 * (nz + 1))) ** 2
            + (4 / hx ** 2) * np.sin(np.pi * q / (2 * (nx + 1))) ** 2).ravel()


@pytest.mark.parametrize("nz,nx,beta", [(12, 14, 0.5), (16, 16, 0.5), (9, 13, 0.3)])
def test_shifted_laplacian_spectrum_on_circle_in_lower_half_plane(nz, nx, beta):
    """gamma = 0, constant m: H and P share the sine eigenvectors, so the
    eigenvalues of P^-1 H are (mu - k^2) / (mu - k^2 + i beta k^2).  They lie on
    the circle |lambda - 1/2| = 1/2, in the lower half plane for every Laplacian
    eigenvalue mu > k^2 and in the upper one for mu < k^2.  A sign slip in the
    shift (1 + beta i) mirrors them into the other half plane."""
    h = 0.01
    mus = _sine_spectrum(nz, nx, h, h)
    # k^2 between two eigenvalues, off the centre of the (symmetric) sine
    # spectrum, so that the two half planes hold different numbers of modes
    srt = np.sort(mus)
    j = int(0.3 * srt.size)
    k2 = 0.5 * (srt[j] + srt[j + 1])
    m = 0.4
    omega = np.sqrt(k2 / m)
    kap = np.full((nz, nx), m)
    gam = np.zeros((nz, nx))
    H = op.assemble(op.helmholtz_coef(kap, gam, omega), h, h).toarray()
    P = op.assemble(op.shifted_coef(kap, gam, omega, beta=beta), h, h).toarray()
    lam = np.linalg.eigvals(np.linalg.solve(P, H))
    assert np.allclose(np.abs(lam - 0.5), 0.5, atol=1e-9)
    a = mus - omega ** 2 * m
    b = beta * omega ** 2 * m
    expect = a / (a + 1j * b)
    d = np.abs(lam[:, None] - expect[None, :])
    assert d.min(axis=1).max() < 1e-9 and d.min(axis=0).max() < 1e-9
    above = a > 1e-9 * np.abs(a).max()
    below = a < -1e-9 * np.abs(a).max()
    assert above.sum() > 0 and below.sum() > 0
    assert np.all(expect[above].imag < 0) and np.all(expect[below].imag > 0)
    assert (lam.imag < -1e-12).sum() == above.sum()
    assert (lam.imag > 1e-12).sum() == below.sum()


def test_shifted_laplacian_with_constant_gamma_spectrum():
    """Constant gamma0: the reading P = -Lap - w^2 m (1 - (gamma + beta) i)
    gives eigenvalues (a + i g0 w^2 m) / (a + i (g0 + beta) w^2 m) of P^-1 H,
    a = mu - w^2 m; with_gamma=False (the literal no-gamma form) gives
    (a + i g0 w^2 m) / (a + i beta w^2 m).  A wrong sign or placement of gamma
    in either operator changes these sets."""
    nz, nx, h, m, g0, beta = 10, 12, 0.02, 0.25, 0.3, 0.5
    mus = _sine_spectrum(nz, nx, h, h)
    srt = np.sort(mus)
    omega = np.sqrt(0.5 * (srt[40] + srt[41]) / m)
    kap = np.full((nz, nx), m)
    gam = np.full((nz, nx), g0)
    H = op.assemble(op.helmholtz_coef(kap, gam, omega), h, h).toarray()
    a = mus - omega ** 2 * m
    k2 = omega ** 2 * m
    for with_gamma, shift in ((True, g0 + beta), (False, beta)):
        P = op.assemble(op.shifted_coef(kap, gam, omega, beta=beta, with_gamma=with_gamma), h, h).toarray()
        lam = np.linalg.eigvals(np.linalg.solve(P, H))
        expect = (a + 1j * g0 * k2) / (a + 1j * shift * k2)
        d = np.abs(lam[:, None] - expect[None, :])
        assert d.min(axis=1).max() < 1e-9 and d.min(axis=0).max() < 1e-9


def test_finest_level_is_the_shifted_operator():
    """Level 0 of the V-cycle applies -Lap_h - diag(shifted_coef) exactly (the
    far-boundary stencil reduces to the regular one when delta = h)."""
    med = medium(24, 30, seed=21)
    hz = 1.3 * med.h
    V = mg.VCycle(med.kappa2, med.gamma, med.omega, med.h, hz)
    u = rand_c((3, 24, 30), 5)
    ref = op.apply(op.shifted_coef(med.kappa2, med.gamma, med.omega), u, med.h, hz)
    assert relerr(V.levels[0].apply(u), ref) < 1e-14
    D = op.assemble(op.shifted_coef(med.kappa2, med.gamma, med.omega), med.h, hz).diagonal()
    assert np.allclose(V.levels[0].diag.ravel(), D, rtol=0, atol=1e-12 * np.abs(D).max())


def test_restrict_coef_field_weights():
    """Normalised full weighting: constants are kept everywhere (including the
    truncated stencils at the far boundary); interior coarse nodes take the
    (1/16)[1 2 1; 2 4 2; 1 2 1] average of the 3 x 3 fine nodes around 2I+1;
    the last coarse row of an even grid renormalises the rows that exist."""
    rng = np.random.default_rng(3)
    nz, nx = 10, 9                       # even nz: fine row 2I+2 = 10 is outside for the last I
    f = rng.uniform(0.2, 1.0, (nz, nx))
    c = mg.restrict_coef_field(f)
    assert c.shape == (5, 4)
    assert np.allclose(mg.restrict_coef_field(np.full((nz, nx), 0.37)), 0.37, atol=1e-15)
    w = np.array([1.0, 2.0, 1.0])
    for I, J in ((1, 1), (2, 3), (3, 2)):
        blk = f[2 * I:2 * I + 3, 2 * J:2 * J + 3]
        assert abs(c[I, J] - (np.outer(w, w) * blk).sum() / 16) < 1e-14
    I, J = 4, 1                          # rows 8, 9 exist, row 10 does not
    blk = f[8:10, 2 * J:2 * J + 3]
    ww = np.outer(w[:2], w)
    assert abs(c[I, J] - (ww * blk).sum() / ww.sum()) < 1e-14
