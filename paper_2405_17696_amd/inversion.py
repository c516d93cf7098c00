"""Frequency continuation (Alg. 1) over the library's Gauss-Newton steps.

Orchestration only: for each cycle (i_start, i_end) of frequency indices
(0-based, inclusive) and each i in it, the operators of the window
omega_max(i - window, 0) .. omega_i are set up with the current model and
gn_iters steps of fwi_gn_step update it; a cycle starts from the model the
previous one ended with.  Every arithmetic step (set-up, solves, gradient,
CG, model update) runs in the library.
"""
from __future__ import annotations

import torch

from . import api


def frequency_continuation(kappa2: torch.Tensor, gamma: torch.Tensor, omegas, h: float, src_idx, rec_idx,
                           dobs: torch.Tensor, cycles, window: int, gn_iters: int, damping: float, cg_iters: int,
                           mu: float = 1.0, **solve_kw):
    """kappa2, gamma float32 [nz][nx] and dobs complex64 [nf][ns][nrec] on the
    GPU.  Returns the final model and, per step, (window (lo, hi), misfit
    before the step, CG residual norms)."""
    m = kappa2.to(torch.float32).contiguous().clone()
    nxt = torch.empty_like(m)
    history = []
    for i0, i1 in cycles:
        for i in range(i0, i1 + 1):
            lo = max(i - window, 0)
            for _ in range(gn_iters):
                ops = [api.helm_setup(m, gamma, w, h) for w in omegas[lo:i + 1]]
                try:
                    _, phi, _, norms, _ = api.fwi_gn_step(ops, src_idx, rec_idx, dobs[lo:i + 1], m, damping, cg_iters,
                                                          mu=mu, m_new=nxt, **solve_kw)
                finally:
                    for o in ops:
                        o.close()
                m, nxt = nxt, m
                history.append(((lo, i), phi, norms))
    return m, history
