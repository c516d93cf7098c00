"""Discrete Helmholtz operator (eq. 3.1 and 3.2) -- oracle, test infrastructure only.

H(m, omega) u = -Lap_h u - omega^2 m (1 - i gamma) u on an nz x nx node grid,
standard 5-point central differences, spacing hx along columns and hz along
rows.  Neighbours outside the grid are zero (Dirichlet-0 ghosts); this keeps
H complex symmetric (H^T = H), the property the adjoint-by-conjugation trick of
Sec. 4.3 relies on.

Everything here is FP64 / complex128.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def helmholtz_coef(kappa2, gamma, omega):
    """Per-node mass term omega^2 m (1 - i gamma) of eq. (3.1)."""
    return (omega ** 2) * np.asarray(kappa2, np.float64) * (1.0 - 1j * np.asarray(gamma, np.float64))


def shifted_coef(kappa2, gamma, omega, beta=0.5, with_gamma=True):
    """Per-node mass term of the shifted Laplacian, eq. (3.12) with alpha = 1:
    omega^2 m (1 - (gamma + beta) i)  (with_gamma=True, the reading used here)
    or the literal omega^2 m (1 - beta i)."""
    g = np.asarray(gamma, np.float64) if with_gamma else 0.0
    return (omega ** 2) * np.asarray(kappa2, np.float64) * (1.0 - 1j * (g + beta))


def laplacian_sparse(nz, nx, hx, hz):
    """-Lap_h as a sparse matrix (node n = i*nx + k, Dirichlet-0 ghosts)."""
    ex = np.ones(nx)
    ez = np.ones(nz)
    Dx = sp.diags([-ex[:-1], 2 * ex, -ex[:-1]], [-1, 0, 1], shape=(nx, nx)) / hx ** 2
    Dz = sp.diags([-ez[:-1], 2 * ez, -ez[:-1]], [-1, 0, 1], shape=(nz, nz)) / hz ** 2
    return (sp.kron(sp.identity(nz), Dx) + sp.kron(Dz, sp.identity(nx))).tocsr()


def assemble(coef, hx, hz):
    """Sparse -Lap_h - diag(coef), complex128 CSR."""
    nz, nx = coef.shape
    L = laplacian_sparse(nz, nx, hx, hz).astype(np.complex128)
    return (L - sp.diags(coef.ravel())).tocsr()


def assemble_helmholtz(kappa2, gamma, omega, hx, hz=None):
    hz = hx if hz is None else hz
    return assemble(helmholtz_coef(kappa2, gamma, omega), hx, hz)


def dense_bruteforce(coef, hx, hz):
    """Entry-by-entry dense matrix straight from the stencil definition (small grids)."""
    nz, nx = coef.shape
    n = nz * nx
    A = np.zeros((n, n), dtype=np.complex128)
    for i in range(nz):
        for k in range(nx):
            r = i * nx + k
            A[r, r] = 2.0 / hx ** 2 + 2.0 / hz ** 2 - coef[i, k]
            for di, dk, w in ((0, -1, hx), (0, 1, hx), (-1, 0, hz), (1, 0, hz)):
                ii, kk = i + di, k + dk
                if 0 <= ii < nz and 0 <= kk < nx:
                    A[r, ii * nx + kk] = -1.0 / w ** 2
    return A


def apply(coef, u, hx, hz):
    """Matrix-free stencil: (-Lap_h - diag(coef)) u for u of shape [..., nz, nx]."""
    u = np.asarray(u)
    p = np.zeros(u.shape[:-2] + (u.shape[-2] + 2, u.shape[-1] + 2), dtype=np.result_type(u, coef))
    p[..., 1:-1, 1:-1] = u
    lap = ((2 * u - p[..., 1:-1, :-2] - p[..., 1:-1, 2:]) / hx ** 2
           + (2 * u - p[..., :-2, 1:-1] - p[..., 2:, 1:-1]) / hz ** 2)
    return lap - coef * u


def apply_helmholtz(kappa2, gamma, omega, u, hx, hz=None):
    hz = hx if hz is None else hz
    return apply(helmholtz_coef(kappa2, gamma, omega), u, hx, hz)


class DirectSolver:
    """SuperLU factorisation of H, reused for many right-hand sides."""

    def __init__(self, A):
        self.lu = spla.splu(A.tocsc())
        self.n = A.shape[0]

    def solve(self, b, trans="N"):
        shape = np.shape(b)
        b2 = np.asarray(b, np.complex128).reshape(-1, self.n).T
        x = self.lu.solve(np.ascontiguousarray(b2), trans=trans)
        return x.T.reshape(shape)


def relres(coef, x, b, hx, hz):
    """||b - Hx||_2 / ||b||_2 per right-hand side (leading axis)."""
    r = np.asarray(b, np.complex128) - apply(coef, np.asarray(x, np.complex128), hx, hz)
    r = r.reshape(r.shape[0], -1) if r.ndim == 3 else r.reshape(1, -1)
    b2 = np.asarray(b, np.complex128).reshape(r.shape[0], -1)
    return np.linalg.norm(r, axis=1) / np.linalg.norm(b2, axis=1)
