"""Frequency continuation (Alg. 1) over the library's Gauss-Newton steps, with
the network's light-weight retraining (Alg. 2) after every window.

Orchestration only: for each cycle (i_start, i_end) of frequency indices
(0-based, inclusive) and each i in it, the operators of the window
omega_max(i - window, 0) .. omega_i are set up with the current model and
gn_iters steps of fwi_gn_step update it (objective: data misfit + alpha R
with the regulariser of eq. 5.1 or 5.2 around a fixed reference model); a
cycle starts from the model the previous one ended with.  After each window,
when a network is given, it is retrained on the model just reached, on the
grid with 10 points per wavelength at the window's highest frequency (Sec. 5,
"Retraining details").  Every arithmetic step (set-up, resampling, solves,
gradient, CG, model update, training) runs in the library.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib as L
from . import api


def training_grid(nz: int, nx: int, h: float, omega: float, c_min: float, ppw: float = 10.0, multiple: int = 8):
    """Grid of the same physical extent with about `ppw` points per minimum
    wavelength at omega (never finer than the inversion grid), sides rounded
    to a multiple of `multiple` (the network needs multiples of 8).  Returns
    (nz_t, nx_t, hx_t, hz_t)."""
    h_t = max(2 * math.pi * c_min / (ppw * omega), h)
    rnd = lambda n: max(multiple, int(round(n * h / h_t / multiple)) * multiple)
    nz_t, nx_t = min(rnd(nz), nz - nz % multiple), min(rnd(nx), nx - nx % multiple)
    return nz_t, nx_t, h * (nx - 1) / (nx_t - 1), h * (nz - 1) / (nz_t - 1)


def retrain_on_window(net, m: torch.Tensor, gamma: torch.Tensor, omega: float, h: float, ppw: float = 10.0,
                      seed: int = 0, alg2: bool = True, **train_kw):
    """Retraining of `net` on the medium m at frequency omega, on the grid with
    `ppw` points per wavelength at omega (model and attenuation resampled
    bilinearly by the library): Alg. 2 (the paper's defaults: 128 pairs, 3 data
    epochs, 30 epochs, lr 1e-4) or, with alg2=False, plain retraining on 2000
    fresh eq. (4.3) pairs for 200 steps at lr 1e-4.  train_kw override
    cnn_precond_train's arguments.  Returns (loss history, dataset size,
    training grid)."""
    nz, nx = m.shape
    c_min = 1.0 / math.sqrt(float(m.max()))
    nz_t, nx_t, hx_t, hz_t = training_grid(nz, nx, h, omega, c_min, ppw)
    if (nz_t, nx_t) == (nz, nx):
        mt, gt = m, gamma
    else:
        mt = api.helm_resample(m, nz_t, nx_t)
        gt = api.helm_resample(gamma, nz_t, nx_t)
    if alg2:
        kw = dict(npairs=128, batch=16, steps=10 ** 6, lr=1e-4, alg2_initial=128, alg2_data_epochs=3, alg2_epochs=30)
    else:
        kw = dict(npairs=2000, batch=16, steps=200, lr=1e-4)
    kw.update(train_kw)
    op = api.helm_setup(mt, gt, omega, hx_t, hz=hz_t)
    try:
        hist, dsz = api.cnn_precond_train(net, op, seed=seed, **kw)
    finally:
        op.close()
    return hist, dsz, (nz_t, nx_t, hx_t, hz_t)


def frequency_continuation(kappa2: torch.Tensor, gamma: torch.Tensor, omegas, h: float, src_idx, rec_idx,
                           dobs: torch.Tensor, cycles, window: int, gn_iters: int, damping: float, cg_iters: int,
                           mu: float = 1.0, reg: str = "none", alpha: float = 0.0, m_ref: torch.Tensor | None = None,
                           tol: float = 1e-6, tol_sens: float = 0.0, retrain=None, allow_not_converged=False,
                           log=None, **solve_kw):
    """kappa2, gamma float32 [nz][nx] and dobs complex64 [nf][ns][nrec] on the
    GPU.  reg / alpha / m_ref: the regulariser ("high": eq. 5.1, "diff":
    eq. 5.2) around m_ref (default: the initial model, kept fixed).
    retrain: None, or a callable retrain(m, i) run after the window that ends
    at frequency index i (e.g. retrain_on_window with the solve's network).
    A step whose solves missed their tolerance raises unless
    allow_not_converged; a non-finite solve always raises.  log: optional
    callable given a one-line summary after every step.  Returns the final
    model and, per step, a dict: window (lo, hi), misfit (data misfit before
    the step), reg (R before the step), norms (CG residual norms), iters
    (solver iterations of every batch of the step, [2 + 2 cg_iters][nfreq][nsrc]),
    code."""
    m = kappa2.to(torch.float32).contiguous().clone()
    m_ref = m.clone() if m_ref is None else m_ref.to(torch.float32).contiguous()
    nxt = torch.empty_like(m)
    history = []
    for i0, i1 in cycles:
        for i in range(i0, i1 + 1):
            lo = max(i - window, 0)
            for _ in range(gn_iters):
                ops = [api.helm_setup(m, gamma, w, h) for w in omegas[lo:i + 1]]
                try:
                    out = api.fwi_gn_step(ops, src_idx, rec_idx, dobs[lo:i + 1], m, damping, cg_iters, mu=mu,
                                          tol=tol, tol_sens=tol_sens, reg=reg, alpha=alpha, m_ref=m_ref, m_new=nxt,
                                          **solve_kw)
                finally:
                    for o in ops:
                        o.close()
                code = out["code"]
                if code != L.HELM_OK and not (allow_not_converged and code == L.HELM_NOT_CONVERGED):
                    raise L.HelmError(code, f"Gauss-Newton step in window {lo}..{i}: some solves missed their "
                                            f"tolerance (pass allow_not_converged=True to continue)")
                m, nxt = nxt, m
                history.append({"window": (lo, i), "misfit": out["misfit"], "reg": out["reg"],
                                "norms": out["norms"], "iters": out["iters"], "code": code})
                if log:
                    log(f"Gauss-Newton step on window {lo}..{i}: misfit {out['misfit']:.6g}, "
                        f"{int(out['iters'].sum())} solver iterations, code {code}")
            if retrain is not None:
                retrain(m, i)
    return m, history
