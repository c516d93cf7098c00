"""Data misfit and its gradient w.r.t. the squared slowness (eq. 3.5, 3.10,
4.8) -- oracle, test infrastructure only.

Forward model, per frequency w_f and source s: H_f u_fs = g_s with
g_s = e_src(s) / (hx hz) (a grid delta), H_f = -Lap_h - w_f^2 m (1 - i gamma)
(eq. 3.1), m = kappa^2.  Data: the wavefield sampled at the receiver nodes,
R u_fs.

Misfit (eq. 3.5 with an identity covariance):
    Phi(m) = 1/2 sum_{f,s} || R u_fs - d_fs ||_2^2 .

Gradient by the adjoint state.  Differentiating H_f u = g gives
du = -H_f^{-1} (dH_f) u with dH_f/dm_k = -w_f^2 (1 - i gamma_k) e_k e_k^T, so
the Jacobian of the data is J_fs = +w_f^2 R H_f^{-1} diag((1 - i gamma) u_fs)
(the sign printed with eq. 3.10 is the opposite one; finite differences in the
tests decide).  With the adjoint field
    lambda_fs = H_f^{-*} R^T (R u_fs - d_fs)
            = conj( H_f^{-1} conj(R^T (R u_fs - d_fs)) )    (H_f^T = H_f, eq. 4.8)
the gradient is
    dPhi/dm_k = sum_{f,s} Re( conj(lambda_fs[k]) w_f^2 (1 - i gamma_k) u_fs[k] ).

Simultaneous sources (Sec. 3.2, eq. 3.6-3.8): the sum over sources of a
frequency's data term is a squared Frobenius norm, ||R H_f^{-1} G - D_f||_F^2
with G = [g_1 .. g_ns] and D_f = [d_f1 .. d_fns], and the trace estimator with
an ns x p matrix X of Rademacher columns replaces it by
(1/p) ||R H_f^{-1} G X - D_f X||_F^2.  Every receiver here records every
source, so the auxiliary data of eq. 3.7 are the observed data themselves.
The encoded misfit and its gradient are those above with the p encoded
sources G x_i and encoded data D_f x_i in place of the ns point sources, and a
factor 1/p.

Gauss-Newton (eq. 3.9-3.11): the Hessian of the misfit without its
second-order term, applied to a model perturbation, is Re(J^H J dm), with
J dm from born and Re(J^H dd) from born_adjoint.  gn_cg is textbook conjugate
gradients on the damped system (Re(J^H J) + damping I) x = b built on it;
gn_step is one Gauss-Newton step m + mu dm with dm from CG on -grad, and
frequency_continuation runs Alg. 1 (cycles of sliding frequency windows) with
those steps.

Regularisation (Sec. 5, eq. 5.1 and 5.2): the objective gains alpha R(m) with
    R_high(m) = || Lap_h (m - m_ref) ||_2^2,   R_diff(m) = || grad_h (m - m_ref) ||_2^2,
grad_h the forward differences between neighbouring nodes of the nodal grid
and Lap_h = -grad_h^T grad_h its divergence (so both terms vanish on constant
m - m_ref; sums over nodes and edges, no cell-area factor).  Their gradients are
2 Lap_h^2 (m - m_ref) and 2 grad_h^T grad_h (m - m_ref), their Hessians 2 Lap_h^2
and 2 grad_h^T grad_h, the alpha nabla^2 R term of the Gauss-Newton matrix of
eq. 3.11.

All solves are SuperLU factorisations in complex128.
"""
from __future__ import annotations

import numpy as np

from . import operator as op


def point_source_rhs(shape, src_idx, hx, hz=None):
    """g_s = e_src / (hx hz) for every source index (flat node index), [ns][nz][nx]."""
    hz = hx if hz is None else hz
    nz, nx = shape
    g = np.zeros((len(src_idx), nz * nx), np.complex128)
    for s, k in enumerate(src_idx):
        g[s, int(k)] = 1.0 / (hx * hz)
    return g.reshape(len(src_idx), nz, nx)


def _solvers(kappa2, gamma, omegas, hx, hz):
    return [op.DirectSolver(op.assemble_helmholtz(kappa2, gamma, w, hx, hz)) for w in omegas]


def wavefields(kappa2, gamma, omegas, hx, src_idx, hz=None):
    """u[f][s] = H_f^{-1} g_s, complex128 [nf][ns][nz][nx]."""
    hz = hx if hz is None else hz
    g = point_source_rhs(kappa2.shape, src_idx, hx, hz)
    return np.stack([S.solve(g) for S in _solvers(kappa2, gamma, omegas, hx, hz)])


def forward_data(kappa2, gamma, omegas, hx, src_idx, rec_idx, hz=None):
    """d[f][s][r] = u_fs at receiver r."""
    u = wavefields(kappa2, gamma, omegas, hx, src_idx, hz)
    nf, ns = u.shape[:2]
    return np.ascontiguousarray(u.reshape(nf, ns, -1)[:, :, np.asarray(rec_idx)])


def misfit(kappa2, gamma, omegas, hx, src_idx, rec_idx, dobs, hz=None):
    d = forward_data(kappa2, gamma, omegas, hx, src_idx, rec_idx, hz)
    res = d - dobs
    return 0.5 * float(np.sum(np.abs(res) ** 2))


def misfit_and_grad(kappa2, gamma, omegas, hx, src_idx, rec_idx, dobs, hz=None):
    """Phi and dPhi/dm (float64 [nz][nx]) by one forward and one adjoint solve per (f, s)."""
    hz = hx if hz is None else hz
    nz, nx = kappa2.shape
    n = nz * nx
    rec = np.asarray(rec_idx)
    g = point_source_rhs((nz, nx), src_idx, hx, hz).reshape(len(src_idx), n)
    phi = 0.0
    grad = np.zeros(n)
    gam = np.asarray(gamma, np.float64).ravel()
    for f, (w, S) in enumerate(zip(omegas, _solvers(kappa2, gamma, omegas, hx, hz))):
        u = S.solve(g)                                   # [ns][n]
        res = u[:, rec] - dobs[f]                        # [ns][nrec]
        phi += 0.5 * float(np.sum(np.abs(res) ** 2))
        src_adj = np.zeros_like(u)
        src_adj[:, rec] = res                            # R^T res
        lam = np.conj(S.solve(np.conj(src_adj)))         # H^{-*} R^T res by conjugation
        grad += np.sum(np.real(np.conj(lam) * (w ** 2) * (1.0 - 1j * gam) * u), axis=0)
    return phi, grad.reshape(nz, nx)


def born(kappa2, gamma, omegas, hx, src_idx, rec_idx, dm, hz=None):
    """Linearised data J dm = w^2 R H^{-1} ((1 - i gamma) u dm), complex [nf][ns][nrec]."""
    hz = hx if hz is None else hz
    nz, nx = kappa2.shape
    g = point_source_rhs((nz, nx), src_idx, hx, hz).reshape(len(src_idx), -1)
    gam = np.asarray(gamma, np.float64).ravel()
    out = []
    for w, S in zip(omegas, _solvers(kappa2, gamma, omegas, hx, hz)):
        u = S.solve(g)
        du = S.solve((w ** 2) * (1.0 - 1j * gam) * u * np.asarray(dm).ravel())
        out.append(du[:, np.asarray(rec_idx)])
    return np.stack(out)


def born_adjoint(kappa2, gamma, omegas, hx, src_idx, rec_idx, dd, hz=None):
    """Re(J^H dd) for real model perturbations, float64 [nz][nx]; the adjoint
    solve here uses SuperLU's conjugate-transpose solve, not the conjugation trick."""
    hz = hx if hz is None else hz
    nz, nx = kappa2.shape
    g = point_source_rhs((nz, nx), src_idx, hx, hz).reshape(len(src_idx), -1)
    gam = np.asarray(gamma, np.float64).ravel()
    rec = np.asarray(rec_idx)
    acc = np.zeros(nz * nx)
    for f, (w, S) in enumerate(zip(omegas, _solvers(kappa2, gamma, omegas, hx, hz))):
        u = S.solve(g)
        q = np.zeros_like(u)
        q[:, rec] = dd[f]
        lam = S.solve(q, trans="H")
        acc += np.sum(np.real(np.conj((w ** 2) * (1.0 - 1j * gam) * u) * lam), axis=0)
    return acc.reshape(nz, nx)


def misfit_and_grad_encoded(kappa2, gamma, omegas, hx, src_idx, rec_idx, dobs, X, hz=None):
    """Phi_X = 1/2 (1/p) sum_f sum_i || R H_f^{-1} G x_i - D_f x_i ||^2 and its
    gradient w.r.t. m (float64 [nz][nx]); X real [ns][p] (Rademacher in use,
    any real matrix here), dobs [nf][ns][nrec]."""
    hz = hx if hz is None else hz
    nz, nx = kappa2.shape
    n = nz * nx
    X = np.asarray(X, np.float64)
    p = X.shape[1]
    rec = np.asarray(rec_idx)
    G = point_source_rhs((nz, nx), src_idx, hx, hz).reshape(len(src_idx), n)   # rows g_s
    q = X.T @ G                                          # encoded sources, [p][n]
    phi = 0.0
    grad = np.zeros(n)
    gam = np.asarray(gamma, np.float64).ravel()
    for f, (w, S) in enumerate(zip(omegas, _solvers(kappa2, gamma, omegas, hx, hz))):
        u = S.solve(q)                                   # H_f^{-1} G x_i, [p][n]
        dx = X.T @ np.asarray(dobs[f])                   # D_f x_i, [p][nrec]
        res = u[:, rec] - dx
        phi += 0.5 * float(np.sum(np.abs(res) ** 2)) / p
        src_adj = np.zeros_like(u)
        src_adj[:, rec] = res
        lam = np.conj(S.solve(np.conj(src_adj)))
        grad += np.sum(np.real(np.conj(lam) * (w ** 2) * (1.0 - 1j * gam) * u), axis=0) / p
    return phi, grad.reshape(nz, nx)


def gn_hessvec(kappa2, gamma, omegas, hx, src_idx, rec_idx, dm, hz=None):
    """Gauss-Newton Hessian times a model perturbation, Re(J^H J dm) (the
    misfit's Hessian without its second-order term, eq. 3.9-3.11), float64 [nz][nx]."""
    jdm = born(kappa2, gamma, omegas, hx, src_idx, rec_idx, dm, hz)
    return born_adjoint(kappa2, gamma, omegas, hx, src_idx, rec_idx, jdm, hz)


def nodal_grad(d, hx, hz):
    """Forward differences between neighbouring nodes: (gx [nz][nx-1], gz [nz-1][nx])."""
    d = np.asarray(d, np.float64)
    return (d[:, 1:] - d[:, :-1]) / hx, (d[1:, :] - d[:-1, :]) / hz


def nodal_grad_T(gx, gz, hx, hz):
    """Adjoint of nodal_grad: an edge difference (b - a)/h sends -1/h to a and +1/h to b."""
    nz, nx = gz.shape[0] + 1, gx.shape[1] + 1
    out = np.zeros((nz, nx))
    out[:, 1:] += gx / hx
    out[:, :-1] -= gx / hx
    out[1:, :] += gz / hz
    out[:-1, :] -= gz / hz
    return out


def reg_laplacian(d, hx, hz):
    """Lap_h d = -grad_h^T grad_h d (the 5-point Laplacian with the nodal-gradient closure)."""
    return -nodal_grad_T(*nodal_grad(d, hx, hz), hx, hz)


REG_NONE, REG_HIGH, REG_DIFF = 0, 1, 2


def regulariser(kind, m, m_ref, hx, hz=None):
    """(R(m), dR/dm) of eq. 5.1 (kind REG_HIGH) or eq. 5.2 (REG_DIFF); REG_NONE gives zeros."""
    hz = hx if hz is None else hz
    d = np.asarray(m, np.float64) - np.asarray(m_ref, np.float64)
    if kind == REG_NONE:
        return 0.0, np.zeros_like(d)
    if kind == REG_HIGH:
        ld = reg_laplacian(d, hx, hz)
        return float(np.sum(ld * ld)), 2.0 * reg_laplacian(ld, hx, hz)
    if kind == REG_DIFF:
        gx, gz = nodal_grad(d, hx, hz)
        return float(np.sum(gx * gx) + np.sum(gz * gz)), 2.0 * nodal_grad_T(gx, gz, hx, hz)
    raise ValueError(kind)


def reg_hessvec(kind, v, hx, hz=None):
    """nabla^2 R applied to v (R is quadratic: 2 Lap_h^2 v or 2 grad_h^T grad_h v)."""
    hz = hx if hz is None else hz
    if kind == REG_NONE:
        return np.zeros_like(np.asarray(v, np.float64))
    if kind == REG_HIGH:
        return 2.0 * reg_laplacian(reg_laplacian(v, hx, hz), hx, hz)
    if kind == REG_DIFF:
        return 2.0 * nodal_grad_T(*nodal_grad(v, hx, hz), hx, hz)
    raise ValueError(kind)


def gn_cg(kappa2, gamma, omegas, hx, src_idx, rec_idx, b, damping, iters, hz=None, reg=REG_NONE, alpha=0.0):
    """Conjugate gradients on the damped Gauss-Newton system
    (Re(J^H J) + alpha nabla^2 R + damping I) x = b from x = 0 (the inner solve of
    a Gauss-Newton step, Sec. 3.3, eq. 3.11), `iters` steps.
    Returns x (float64 [nz][nx]) and the residual norms ||b - A x_k||, k = 0..iters."""
    hz_ = hx if hz is None else hz
    A = lambda v: (gn_hessvec(kappa2, gamma, omegas, hx, src_idx, rec_idx, v, hz) + damping * v
                   + alpha * reg_hessvec(reg, v, hx, hz_))
    b = np.asarray(b, np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.sum(r * r))
    norms = [np.sqrt(rr)]
    for _ in range(iters):
        ap = A(p)
        step = rr / float(np.sum(p * ap))
        x = x + step * p
        r = r - step * ap
        rr_new = float(np.sum(r * r))
        norms.append(np.sqrt(rr_new))
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, np.array(norms)


def gn_step(kappa2, gamma, omegas, hx, src_idx, rec_idx, dobs, damping, cg_iters, mu, hz=None, reg=REG_NONE,
            alpha=0.0, m_ref=None):
    """One Gauss-Newton step (Sec. 3.3) on Phi(m) + alpha R(m): the data misfit
    Phi and the gradient g = dPhi/dm + alpha dR/dm at m, dm from cg_iters CG
    steps on (Re(J^H J) + alpha nabla^2 R + damping I) dm = -g, and m + mu dm.
    Returns (m_new, Phi(m), CG residual norms, R(m), g)."""
    phi, g = misfit_and_grad(kappa2, gamma, omegas, hx, src_idx, rec_idx, dobs, hz)
    rv = 0.0
    if reg != REG_NONE:
        rv, rg = regulariser(reg, kappa2, m_ref, hx, hz)
        g = g + alpha * rg
    dm, norms = gn_cg(kappa2, gamma, omegas, hx, src_idx, rec_idx, -g, damping, cg_iters, hz, reg, alpha)
    return kappa2 + mu * dm, phi, norms, rv, g


def frequency_continuation(kappa2, gamma, omegas, hx, src_idx, rec_idx, dobs, cycles, window, gn_iters, damping,
                           cg_iters, mu, hz=None, reg=REG_NONE, alpha=0.0, m_ref=None):
    """Alg. 1: for each cycle (i_start, i_end) (0-based, inclusive) and each
    i in it, gn_iters Gauss-Newton steps on the data of the frequencies
    omega_max(i - window, 0) .. omega_i, each cycle starting from the previous
    model.  dobs [nf][ns][nrec] for all frequencies; gamma is fixed; the
    regulariser (reg, alpha) keeps its reference model m_ref (default: the
    initial model) fixed.  Returns the final model and the misfit before every step."""
    m = np.asarray(kappa2, np.float64)
    m_ref = m.copy() if m_ref is None else np.asarray(m_ref, np.float64)
    history = []
    for i0, i1 in cycles:
        for i in range(i0, i1 + 1):
            lo = max(i - window, 0)
            for _ in range(gn_iters):
                m, phi, _, _, _ = gn_step(m, gamma, omegas[lo:i + 1], hx, src_idx, rec_idx, dobs[lo:i + 1], damping,
                                          cg_iters, mu, hz, reg, alpha, m_ref)
                history.append(phi)
    return m, np.array(history)


def resample_bilinear(f, mz, mx):
    """Bilinear interpolation of a nodal field [nz][nx] onto an mz x mx grid of
    the same extent (node I at coordinate I (nz-1)/(mz-1) of the input grid),
    by scipy's regular-grid linear interpolator: the grid the network is
    retrained on after a window of Alg. 1 (Sec. 5, retraining details)."""
    from scipy.interpolate import RegularGridInterpolator
    f = np.asarray(f, np.float64)
    nz, nx = f.shape
    it = RegularGridInterpolator((np.arange(nz, dtype=np.float64), np.arange(nx, dtype=np.float64)), f,
                                 method="linear")
    z = np.arange(mz) * (nz - 1) / max(mz - 1, 1)
    x = np.arange(mx) * (nx - 1) / max(mx - 1, 1)
    Z, X = np.meshgrid(z, x, indexing="ij")
    return it(np.stack([Z.ravel(), X.ravel()], axis=1)).reshape(mz, mx)
