"""Training of the encoder-solver network (eq. 4.2-4.3, Alg. 2) -- oracle, test infrastructure only.

* loss (eq. 4.2): L = (1/B) sum_i || net(s_i r_i) - s_i e_i / (hx hz) ||_2^2 over both
  real channels and all pixels, with s_i = sqrt(N)/||r_i|| (the scaling of unet.py);
* Adam (the optimiser the paper names): beta = (0.9, 0.999), eps = 1e-8, bias
  corrected;
* data generation (eq. 4.3): x ~ CN(0,1), b = H x, x~ = GMRES(H, M = V-cycle, b,
  x0 = 0, k iterations), k uniform on {1..10}; r = b - H x~, e = x - x~;
* light-weight retraining (Alg. 2): each of the first data_epochs epochs,
  after training on D, every pair of a snapshot of D spawns
  e_new = M_net(r), e~ = one GMRES iteration on H e = r from x0 = e_new (V-cycle
  preconditioner), r~ = H e~, and (r~, e~) is appended, so D doubles per epoch.
The random draws come from Philox-4x32-10 (philox.py):
  x of sample i: complex normal stream i under key (seed, 0xDA7A);
  k of sample i: 1 + floor(10 u) with u from word 0 of counter (i, 0x7FFFFFFF, 0, 0).
"""
from __future__ import annotations

import numpy as np

from . import krylov as kr
from . import operator as op
from . import philox
from . import unet as U

DATA_KEY1 = 0xDA7A
K_STREAM = 0x7FFFFFFF


def sample_k(i, seed):
    w = philox.philox4x32(np.array([i & 0xFFFFFFFF, K_STREAM, 0, 0], dtype=np.uint64), (seed, DATA_KEY1))
    u = philox.uniform01(w)[0]
    return 1 + int(np.floor(10.0 * u))


def sample_x(i, n, seed):
    return philox.complex_normal(n, (seed, DATA_KEY1), stream_id=i)


def make_pairs(coef, hx, hz, vcycle, shape, npairs, seed, first=0):
    """(r, e) pairs of eq. 4.3 for one medium; returns r, e complex [npairs][nz][nx] and the k's."""
    nz, nx = shape
    n = nz * nx
    A = lambda v: op.apply(coef, v.reshape(nz, nx), hx, hz).ravel()
    M = lambda v: vcycle(v.reshape(nz, nx)).ravel()
    R = np.zeros((npairs, nz, nx), np.complex128)
    E = np.zeros_like(R)
    ks = []
    for t in range(npairs):
        i = first + t
        x = sample_x(i, n, seed)
        k = sample_k(i, seed)
        b = A(x)
        res = kr.fgmres(A, b, M=M, max_iters_exact=k)
        xt = res.x
        R[t] = (b - A(xt)).reshape(nz, nx)
        E[t] = (x - xt).reshape(nz, nx)
        ks.append(k)
    return R, E, ks


def mse_loss_and_grad(out, target):
    """L = (1/B) sum ||out - target||^2 and dL/dout."""
    B = out.shape[0]
    d = out - target
    return float((d * d).sum() / B), 2.0 * d / B


def scaled_pair(r, e, hx, hz):
    """Network input s r and target s e / (hx hz) as [B][H][W][2] real arrays."""
    B = r.shape[0]
    N = r[0].size
    s = np.sqrt(N) / np.linalg.norm(r.reshape(B, -1), axis=1)
    rin = np.stack([r.real, r.imag], axis=-1) * s[:, None, None, None]
    tgt = np.stack([e.real, e.imag], axis=-1) * (s / (hx * hz))[:, None, None, None]
    return rin, tgt


def loss_and_grad(theta, enc_in, r, e, hx, hz, w=U.WIDTHS, down_res=2):
    rin, tgt = scaled_pair(r, e, hx, hz)
    out, st = U.network_forward(theta, enc_in, rin, w, down_res)
    L, g = mse_loss_and_grad(out, tgt)
    return L, U.network_backward(st, g, w)


class Adam:
    def __init__(self, n, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)


def alg2_new_pairs(theta, coef, hx, hz, vcycle, kappa2, gamma, omega, R, E, w=U.WIDTHS, down_res=2):
    """One data epoch of Alg. 2 on a snapshot (R, E): the appended pairs."""
    nz, nx = R.shape[1:]
    A = lambda v: op.apply(coef, v.reshape(nz, nx), hx, hz).ravel()
    M = lambda v: vcycle(v.reshape(nz, nx)).ravel()
    e_new = U.cnn_precond(theta, kappa2, gamma, omega, hx, hz, R, w, down_res)
    Rn = np.zeros_like(R)
    En = np.zeros_like(E)
    for t in range(R.shape[0]):
        res = kr.fgmres(A, R[t].ravel(), M=M, x0=e_new[t].ravel(), max_iters_exact=1)
        En[t] = res.x.reshape(nz, nx)
        Rn[t] = A(res.x).reshape(nz, nx)
    return Rn, En
