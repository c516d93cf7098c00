"""Host logic of the frequency-continuation driver (Alg. 1), with the library
calls replaced by recording stand-ins: the sequence of frequency windows, the
hand-over of the model from step to step, the release of every operator, the
handling of the steps' return codes, the per-step iteration record, the
regulariser's fixed reference model, and retraining after every window."""
import numpy as np
import pytest
import torch

from paper_2405_17696_amd import _lib as L
from paper_2405_17696_amd import api, inversion


class FakeOp:
    def __init__(self, log, m, w):
        self.log, self.m, self.w, self.closed = log, m, w, False

    def close(self):
        self.closed = True


def _patch(monkeypatch, codes=None):
    log, ops_made, refs = [], [], []

    def setup(m, gamma, w, h):
        op = FakeOp(log, m.clone(), w)
        ops_made.append(op)
        return op

    def gn_step(ops, src, rec, dobs, m, damping, cg_iters, mu=1.0, m_new=None, m_ref=None, **kw):
        assert all(torch.equal(o.m, m) for o in ops)           # operators built from the current model
        assert dobs.shape[0] == len(ops)
        refs.append(m_ref.clone())
        log.append(([o.w for o in ops], float(m[0, 0])))
        m_new.copy_(m + mu)                                     # stand-in update: +mu everywhere
        code = codes[len(log) - 1] if codes else 0
        its = np.full((2 + 2 * cg_iters, len(ops), len(src)), len(log))
        return {"m_new": m_new, "misfit": 10.0 - len(log), "reg": 0.0, "grad": None,
                "norms": np.zeros(cg_iters + 1), "iters": its, "code": code}

    monkeypatch.setattr(api, "helm_setup", setup)
    monkeypatch.setattr(api, "fwi_gn_step", gn_step)
    return log, ops_made, refs


def test_windows_model_handover_and_cleanup(monkeypatch):
    log, ops_made, refs = _patch(monkeypatch)
    omegas = [1.0, 2.0, 3.0, 4.0]
    m0 = torch.zeros((4, 4))
    dobs = torch.zeros((4, 2, 3), dtype=torch.complex64)
    retrained = []
    m, hist = inversion.frequency_continuation(m0, None, omegas, 1.0, [0, 1], [2, 3, 4], dobs,
                                               cycles=[(0, 3), (2, 3)], window=1, gn_iters=2, damping=0.0,
                                               cg_iters=2, mu=0.5,
                                               retrain=lambda mm, i: retrained.append((i, float(mm[0, 0]))))
    windows = [h["window"] for h in hist]
    assert windows == [(0, 0)] * 2 + [(0, 1)] * 2 + [(1, 2)] * 2 + [(2, 3)] * 2 + [(1, 2)] * 2 + [(2, 3)] * 2
    assert [f for f, _ in log][:4] == [[1.0], [1.0], [1.0, 2.0], [1.0, 2.0]]
    # each step starts from the previous step's model, across cycles too
    assert [v for _, v in log] == [0.5 * k for k in range(12)]
    assert float(m[0, 0]) == 6.0 and torch.equal(m0, torch.zeros((4, 4)))
    assert all(o.closed for o in ops_made)
    # the regulariser's reference stays the initial model
    assert all(torch.equal(r, m0) for r in refs)
    # retraining after every window, on the model the window ended with
    assert retrained == [(0, 1.0), (1, 2.0), (2, 3.0), (3, 4.0), (2, 5.0), (3, 6.0)]
    # per-step iteration record and misfit
    assert hist[3]["iters"].shape == (6, 2, 2) and int(hist[3]["iters"].max()) == 4
    assert [h["misfit"] for h in hist][:3] == [9.0, 8.0, 7.0]


def test_step_codes_raise_unless_allowed(monkeypatch):
    omegas = [1.0, 2.0]
    m0 = torch.zeros((4, 4))
    dobs = torch.zeros((2, 2, 3), dtype=torch.complex64)
    kw = dict(cycles=[(0, 1)], window=1, gn_iters=1, damping=0.0, cg_iters=1)
    _patch(monkeypatch, codes=[0, L.HELM_NOT_CONVERGED])
    with pytest.raises(L.HelmError):
        inversion.frequency_continuation(m0, None, omegas, 1.0, [0, 1], [2, 3, 4], dobs, **kw)
    _patch(monkeypatch, codes=[0, L.HELM_NOT_CONVERGED])
    m, hist = inversion.frequency_continuation(m0, None, omegas, 1.0, [0, 1], [2, 3, 4], dobs,
                                               allow_not_converged=True, **kw)
    assert [h["code"] for h in hist] == [0, L.HELM_NOT_CONVERGED]
    _patch(monkeypatch, codes=[L.HELM_ENAN, 0])
    with pytest.raises(L.HelmError):
        inversion.frequency_continuation(m0, None, omegas, 1.0, [0, 1], [2, 3, 4], dobs, allow_not_converged=True,
                                         **kw)


def test_training_grid_ten_points_per_wavelength():
    # 512 nodes at 13.5 points per wavelength -> about 379 at 10, rounded to a multiple of 8
    import math
    c, h = 1.5, 0.0125
    w = 2 * math.pi * c / (13.5 * h)
    nz, nx, hx, hz = inversion.training_grid(512, 512, h, w, c)
    assert (nz, nx) == (376, 376) or (nz, nx) == (384, 384)
    assert abs(2 * math.pi * c / (w * hx) - 10.0) < 0.2
    assert abs(hx * (nx - 1) - h * 511) < 1e-12            # same extent
    # a window already at or below 10 points per wavelength keeps the grid
    w10 = 2 * math.pi * c / (8.0 * h)
    assert inversion.training_grid(512, 512, h, w10, c)[:2] == (512, 512)
