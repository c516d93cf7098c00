"""Shifted-Laplacian multigrid V-cycle (eq. 3.12, Sec. 3.4) -- oracle, test infrastructure only.

The paper fixes only the operator P = -Lap_h - omega^2 m (alpha - beta i) with
alpha = 1, beta = 0.5 and "levels = 3".  The cycle internals are this build's
reading (they make V_SL a fixed *linear* operator, as plain GMRES needs):
  * coarse node I of a level sits on node 2I+1 of the level above, so a level
    of n nodes has floor(n/2) coarse nodes and every level keeps the first
    boundary (the ghost row/column -1, i.e. the free surface and the left
    edge) exactly in place;
  * the far boundary (ghost n of the finest grid) then lies a distance
    delta = h (finest spacing) beyond the last node of every level; the last
    row/column of a level uses the non-uniform second difference
    -u'' ~ 2/(H+delta) [ (1/delta + 1/H) u - u_W / H ]   (H = level spacing),
    which is the ordinary 5-point stencil on the finest level (delta = H) and
    keeps the coarse operators consistent with the fine boundary.  Without it
    (coarse boundary one fine cell off) the 3-level cycle stops contracting;
  * P_l is rediscretised on level l from m and gamma restricted by normalised
    full weighting (weights over in-range fine nodes only);
  * residual restriction: full weighting, stencil (1/16)[1 2 1; 2 4 2; 1 2 1];
  * prolongation: bilinear interpolation (= 4 R^T);
  * smoother: damped Jacobi, weight 0.8, one pre- and one post-sweep;
  * coarsest level: a fixed GMRES polynomial of degree 20.  Damped Jacobi
    diverges on the coarse shifted Laplacian (its smooth modes have negative
    real part once k h exceeds 1), and an inner Krylov solve, as in the
    two-grid schemes the paper builds on, would make the cycle nonlinear.  The
    polynomial keeps the cycle linear: its roots are the harmonic Ritz values
    of a degree-20 Arnoldi run on the coarsest operator started from a fixed
    Philox-4x32 vector (key COARSE_KEY, entries uniform in the unit square,
    normalised; a smooth start vector would leave the oscillatory modes out of
    the polynomial), applied in Leja order as
    x <- x + r/theta, r <- r - P r/theta, so that p(P) f is what GMRES(20)
    would return for that start vector.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import operator as op
from . import philox

COARSE_KEY = (0x48454C4D, 0x5F534C31)   # fixed key of the coarse start vector

FW = np.array([0.25, 0.5, 0.25])


def coarse_shape(nz, nx):
    return nz // 2, nx // 2


def restrict_fw(r):
    """Full-weighting restriction of [..., nz, nx] onto the odd nodes (zero ghosts)."""
    nz, nx = r.shape[-2:]
    cz, cx = coarse_shape(nz, nx)
    p = np.zeros(r.shape[:-2] + (nz + 2, nx + 2), dtype=r.dtype)
    p[..., 1:-1, 1:-1] = r
    out = np.zeros(r.shape[:-2] + (cz, cx), dtype=r.dtype)
    for a in range(3):
        for b in range(3):
            # fine index 2I + 1 + (a-1) -> padded index 2I + 1 + a
            out += FW[a] * FW[b] * p[..., 1 + a:1 + a + 2 * cz:2, 1 + b:1 + b + 2 * cx:2]
    return out


def prolong_bilinear(ec, fine_shape):
    """Bilinear prolongation (4 R^T) of coarse [..., cz, cx] onto [..., nz, nx]."""
    nz, nx = fine_shape
    cz, cx = ec.shape[-2:]
    out = np.zeros(ec.shape[:-2] + (nz + 2, nx + 2), dtype=ec.dtype)
    for a in range(3):
        for b in range(3):
            w = 4.0 * FW[a] * FW[b]
            out[..., 1 + a:1 + a + 2 * cz:2, 1 + b:1 + b + 2 * cx:2] += w * ec
    return out[..., 1:nz + 1, 1:nx + 1]


def restrict_coef_field(f):
    """Normalised full weighting of a real coefficient field (m or gamma)."""
    num = restrict_fw(np.asarray(f, np.float64))
    den = restrict_fw(np.ones_like(f, dtype=np.float64))
    return num / den


@dataclass
class Level:
    """One level: mass term, spacings, and the distances from the last row /
    column to the far boundary (equal to the spacings on the finest level)."""
    coef: np.ndarray   # SL mass term omega^2 m (1 - (gamma + beta) i)
    hx: float
    hz: float
    dx: float = None
    dz: float = None

    def __post_init__(self):
        self.dx = self.hx if self.dx is None else self.dx
        self.dz = self.hz if self.dz is None else self.dz
        nz, nx = self.coef.shape
        self.cwx = np.full(nx, 1.0 / self.hx ** 2)      # coefficient of the west neighbour
        self.cex = np.full(nx, 1.0 / self.hx ** 2)      # coefficient of the east neighbour
        self.dgx = np.full(nx, 2.0 / self.hx ** 2)      # x part of the diagonal
        self.cnz = np.full(nz, 1.0 / self.hz ** 2)
        self.csz = np.full(nz, 1.0 / self.hz ** 2)
        self.dgz = np.full(nz, 2.0 / self.hz ** 2)
        H, d = self.hx, self.dx
        self.cwx[-1] = 2.0 / ((H + d) * H)
        self.dgx[-1] = 2.0 / (H + d) * (1.0 / d + 1.0 / H)
        H, d = self.hz, self.dz
        self.cnz[-1] = 2.0 / ((H + d) * H)
        self.dgz[-1] = 2.0 / (H + d) * (1.0 / d + 1.0 / H)

    @property
    def diag(self):
        return self.dgz[:, None] + self.dgx[None, :] - self.coef

    def apply(self, u):
        u = np.asarray(u)
        p = np.zeros(u.shape[:-2] + (u.shape[-2] + 2, u.shape[-1] + 2), dtype=np.complex128)
        p[..., 1:-1, 1:-1] = u
        return (self.diag * u - self.cwx[None, :] * p[..., 1:-1, :-2] - self.cex[None, :] * p[..., 1:-1, 2:]
                - self.cnz[:, None] * p[..., :-2, 1:-1] - self.csz[:, None] * p[..., 2:, 1:-1])


class VCycle:
    """V_SL(f): one 3-level V-cycle for P e = f from e = 0 (a linear map)."""

    def __init__(self, kappa2, gamma, omega, hx, hz=None, levels=3, beta=0.5,
                 jacobi_weight=0.8, pre=1, post=1, coarse_degree=20, with_gamma=True):
        hz = hx if hz is None else hz
        self.levels = []
        k2 = np.asarray(kappa2, np.float64)
        g = np.asarray(gamma, np.float64)
        nz0, nx0 = k2.shape
        for lvl in range(levels):
            cz, cxn = k2.shape
            # last node of level lvl sits on finest node 2^lvl * n_lvl - 1
            dz = (nz0 - (2 ** lvl * cz - 1)) * hz
            dx = (nx0 - (2 ** lvl * cxn - 1)) * hx
            self.levels.append(Level(op.shifted_coef(k2, g, omega, beta, with_gamma),
                                     hx * 2 ** lvl, hz * 2 ** lvl, dx, dz))
            if lvl + 1 < levels:
                k2 = restrict_coef_field(k2)
                g = restrict_coef_field(g)
        self.w = jacobi_weight
        self.pre, self.post = pre, post
        self.roots = coarse_roots(self.levels[-1], coarse_degree)

    def jacobi(self, L, e, f, sweeps):
        for _ in range(sweeps):
            e = e + self.w * (f - L.apply(e)) / L.diag
        return e

    def cycle(self, f, lvl=0):
        L = self.levels[lvl]
        e = np.zeros_like(f, dtype=np.complex128)
        if lvl == len(self.levels) - 1:
            return apply_root_polynomial(L, self.roots, f)
        e = self.jacobi(L, e, f, self.pre)
        r = f - L.apply(e)
        ec = self.cycle(restrict_fw(r), lvl + 1)
        e = e + prolong_bilinear(ec, f.shape[-2:])
        return self.jacobi(L, e, f, self.post)

    def __call__(self, f):
        return self.cycle(np.asarray(f, np.complex128))


def harmonic_ritz(L, degree):
    """Harmonic Ritz values of `degree` Arnoldi steps (modified Gram-Schmidt) on
    the level operator from the normalised Philox start vector.  They are the roots of the
    GMRES residual polynomial for that start vector."""
    shape = L.coef.shape
    n = L.coef.size
    degree = min(degree, n)          # the Krylov space has at most n dimensions
    V = np.zeros((degree + 1, n), np.complex128)
    Hh = np.zeros((degree + 1, degree), np.complex128)
    v0 = philox.complex_uniform(n, COARSE_KEY)
    V[0] = v0 / np.linalg.norm(v0)
    k = degree
    for j in range(degree):
        w = L.apply(V[j].reshape(shape)).ravel()
        w_norm = np.linalg.norm(w)
        for i in range(j + 1):
            Hh[i, j] = np.vdot(V[i], w)
            w = w - Hh[i, j] * V[i]
        Hh[j + 1, j] = np.linalg.norm(w)
        if Hh[j + 1, j] <= 1e-12 * w_norm:      # invariant subspace reached
            k = j + 1
            break
        V[j + 1] = w / Hh[j + 1, j]
    Hk = Hh[:k, :k]
    ek = np.zeros(k)
    ek[-1] = 1.0
    f = np.linalg.solve(Hk.conj().T, ek)
    T = Hk + abs(Hh[k, k - 1]) ** 2 * np.outer(f, ek)
    return np.linalg.eigvals(T)


def leja_order(theta):
    """Leja ordering: start from the largest modulus, then repeatedly take the
    point maximising the product of distances to those already taken (ties to
    the lowest index)."""
    theta = np.asarray(theta)
    k = theta.size
    first = int(np.argmax(np.abs(theta)))
    order = [first]
    rest = [i for i in range(k) if i != first]
    while rest:
        score = [np.prod(np.abs(theta[i] - theta[order])) for i in rest]
        best = rest[int(np.argmax(score))]
        order.append(best)
        rest.remove(best)
    return theta[order]


def coarse_roots(L, degree):
    return leja_order(harmonic_ritz(L, degree))


def apply_root_polynomial(L, roots, f):
    """x = p(P) f with 1 - z p(z) = prod (1 - z/theta_i)."""
    x = np.zeros_like(f, dtype=np.complex128)
    r = np.array(f, dtype=np.complex128)
    for t in roots:
        x = x + r / t
        r = r - L.apply(r) / t
    return x
