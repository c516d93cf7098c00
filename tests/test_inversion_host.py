"""Host logic of the frequency-continuation driver (Alg. 1), with the library
calls replaced by recording stand-ins: the sequence of frequency windows, the
hand-over of the model from step to step and the release of every operator."""
import numpy as np
import torch

from paper_2405_17696_amd import api, inversion


class FakeOp:
    def __init__(self, log, m, w):
        self.log, self.m, self.w, self.closed = log, m, w, False

    def close(self):
        self.closed = True


def test_windows_model_handover_and_cleanup(monkeypatch):
    log, ops_made = [], []

    def setup(m, gamma, w, h):
        op = FakeOp(log, m.clone(), w)
        ops_made.append(op)
        return op

    def gn_step(ops, src, rec, dobs, m, damping, cg_iters, mu=1.0, m_new=None, **kw):
        assert all(torch.equal(o.m, m) for o in ops)           # operators built from the current model
        assert dobs.shape[0] == len(ops)
        log.append(([o.w for o in ops], float(m[0, 0])))
        m_new.copy_(m + mu)                                     # stand-in update: +mu everywhere
        return m_new, 10.0 - len(log), None, np.zeros(cg_iters + 1), 0

    monkeypatch.setattr(api, "helm_setup", setup)
    monkeypatch.setattr(api, "fwi_gn_step", gn_step)
    omegas = [1.0, 2.0, 3.0, 4.0]
    m0 = torch.zeros((4, 4))
    dobs = torch.zeros((4, 2, 3), dtype=torch.complex64)
    m, hist = inversion.frequency_continuation(m0, None, omegas, 1.0, [0, 1], [2, 3, 4], dobs,
                                               cycles=[(0, 3), (2, 3)], window=1, gn_iters=2, damping=0.0,
                                               cg_iters=2, mu=0.5)
    windows = [w for w, _, _ in hist]
    assert windows == [(0, 0)] * 2 + [(0, 1)] * 2 + [(1, 2)] * 2 + [(2, 3)] * 2 + [(1, 2)] * 2 + [(2, 3)] * 2
    assert [f for f, _ in log][:4] == [[1.0], [1.0], [1.0, 2.0], [1.0, 2.0]]
    # each step starts from the previous step's model, across cycles too
    assert [v for _, v in log] == [0.5 * k for k in range(12)]
    assert float(m[0, 0]) == 6.0 and torch.equal(m0, torch.zeros((4, 4)))
    assert all(o.closed for o in ops_made)
