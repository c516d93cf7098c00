"""Restarted GMRES and right-preconditioned flexible GMRES -- oracle, test infrastructure only.

Textbook FGMRES(m) (Saad's flexible variant: the preconditioned directions
z_j = M(v_j) are stored, x = x0 + Z y), modified Gram-Schmidt, complex Givens
rotations, FP64 / complex128 throughout.  With a linear M it is ordinary
right-preconditioned GMRES(m).  The stopping test is the true residual
||b - H x||_2 / ||b||_2 <= tol, recomputed at every restart; inside a cycle the
Givens residual estimate (equal to the true residual in exact arithmetic for
right preconditioning) ends the cycle early.  These are the readings the paper
leaves open (it says "GMRES" with a V-cycle or CNN preconditioner, tolerances
1e-6 / 1e-4 in Sec. 5.4 and a 300-iteration cap in Sec. 5.7).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class KrylovResult:
    x: np.ndarray
    iters: int
    relres: float
    converged: bool
    history: list = field(default_factory=list)


def fgmres(A, b, M=None, x0=None, restart=20, tol=1e-6, maxit=300, max_iters_exact=None):
    """Solve A x = b.  A, M: callables on flat complex128 vectors.

    max_iters_exact: if given, perform exactly that many Arnoldi iterations
    (no convergence test, no restart) -- the fixed-iteration GMRES of eq. (4.3)
    and Alg. 2."""
    b = np.asarray(b, np.complex128).ravel()
    n = b.size
    x = np.zeros(n, np.complex128) if x0 is None else np.asarray(x0, np.complex128).ravel().copy()
    M = (lambda v: v) if M is None else M
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return KrylovResult(np.zeros(n, np.complex128), 0, 0.0, True, hist)
    its = 0
    budget = maxit if max_iters_exact is None else max_iters_exact
    m_cycle = restart if max_iters_exact is None else max_iters_exact
    while True:
        r = b - A(x)
        beta = np.linalg.norm(r)
        rel = beta / bnorm
        hist.append(rel)
        if max_iters_exact is None and (rel <= tol or its >= budget):
            return KrylovResult(x, its, rel, rel <= tol, hist)
        if max_iters_exact is not None and its >= budget:
            return KrylovResult(x, its, rel, rel <= tol, hist)
        if beta == 0.0:
            return KrylovResult(x, its, 0.0, True, hist)
        m = min(m_cycle, budget - its)
        V = np.zeros((m + 1, n), np.complex128)
        Z = np.zeros((m, n), np.complex128)
        Hh = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m, np.complex128)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = np.asarray(M(V[j]), np.complex128).ravel()
            w = np.asarray(A(Z[j]), np.complex128).ravel()
            for i in range(j + 1):                 # modified Gram-Schmidt
                Hh[i, j] = np.vdot(V[i], w)
                w = w - Hh[i, j] * V[i]
            Hh[j + 1, j] = np.linalg.norm(w)
            breakdown = Hh[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / Hh[j + 1, j]
            for i in range(j):                     # previous rotations
                t = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                Hh[i + 1, j] = -np.conj(sn[i]) * Hh[i, j] + np.conj(cs[i]) * Hh[i + 1, j]
                Hh[i, j] = t
            a, c = Hh[j, j], Hh[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            # unitary [[cs, sn], [-conj(sn), conj(cs)]] maps (a, c) to (den, 0)
            if den == 0.0:
                cs[j], sn[j] = 1.0, 0.0
            else:
                cs[j], sn[j] = np.conj(a) / den, np.conj(c) / den
            t = cs[j] * Hh[j, j] + sn[j] * Hh[j + 1, j]
            Hh[j + 1, j] = 0.0
            Hh[j, j] = t
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            its += 1
            if breakdown:
                break
            if max_iters_exact is None and abs(g[j + 1]) / bnorm <= tol:
                break
        y = np.linalg.solve(np.triu(Hh[:k, :k]), g[:k])
        x = x + Z[:k].T @ y


def gmres(A, b, M=None, **kw):
    """Right-preconditioned GMRES = FGMRES with a linear M."""
    return fgmres(A, b, M=M, **kw)
