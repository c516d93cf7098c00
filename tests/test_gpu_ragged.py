"""Ragged batches at the shape of the uneven-batch workload: three grids
(256 x 512, 384 x 768, 512 x 1024) sampling one faulted model, three
frequencies each (5, 8 and 12 points per wavelength), all systems in one
masked FGMRES launch.  Each system's result must not depend on the batch it
rides in (bit-identical to solving it alone), graph replay must match eager
launches, and every returned residual is recomputed by the oracle's FP64
operator."""
import numpy as np
import pytest
import torch

from oracle import operator as op
from paper_2405_17696_amd import api, synth

pytestmark = pytest.mark.gpu

NSRC = 2
MAXIT = 300


@pytest.fixture(scope="module")
def batch(gpu):
    items = synth.config3_media(nsrc=NSRC)
    ops, rhs, rhs_op, meds = [], [], [], []
    for k, (med, src) in enumerate(items):
        k2 = torch.tensor(med.kappa2, dtype=torch.float32, device="cuda")
        g = torch.tensor(med.gamma, dtype=torch.float32, device="cuda")
        ops.append(api.helm_setup(k2, g, med.omega, med.h))
        rhs.append(src.reshape(src.shape[0], -1))
        rhs_op += [k] * src.shape[0]
        meds.append(med)
    b = torch.tensor(np.concatenate([r.ravel() for r in rhs]), dtype=torch.complex64, device="cuda")
    return ops, b, rhs_op, meds, rhs


def split(flat, rhs_op, ops):
    out, o = [], 0
    for k in rhs_op:
        n = ops[k].n
        out.append(flat[o:o + n])
        o += n
    return out


@pytest.mark.parametrize("precond", ["mg", "cnn_vu"])
def test_ragged_batch_equals_per_system_solves(batch, precond):
    ops, b, rhs_op, meds, rhs = batch
    net = api.cnn_create(seed=5) if precond != "mg" else None
    maxit = MAXIT if precond == "mg" else 60
    print("ragged", precond, len(rhs_op), "systems", flush=True)
    x, it, rr, st, code = api.helm_solve(ops, b, tol=1e-6, rhs_op=rhs_op, precond=precond, maxit=maxit, net=net,
                                         restart=20)
    xs = split(x, rhs_op, ops)
    bs = split(b, rhs_op, ops)
    for k in range(len(ops)):
        sel = [i for i, o in enumerate(rhs_op) if o == k]
        bk = torch.cat([bs[i] for i in sel])
        xk, itk, rrk, stk, _ = api.helm_solve(ops[k], bk, tol=1e-6, precond=precond, maxit=maxit, net=net,
                                              restart=20)
        print("op", k, meds[k].kappa2.shape, "its", itk.tolist(), flush=True)
        assert np.array_equal(itk, it[sel]) and np.array_equal(stk, st[sel])
        assert np.array_equal(rrk, rr[sel])
        assert torch.equal(xk, torch.cat([xs[i] for i in sel]))


def test_ragged_graph_replay_and_oracle_residuals(batch):
    ops, b, rhs_op, meds, rhs = batch
    x, it, rr, st, code = api.helm_solve(ops, b, tol=1e-6, rhs_op=rhs_op, precond="mg", maxit=MAXIT, restart=20)
    xg, itg, rrg, stg, _ = api.helm_solve(ops, b, tol=1e-6, rhs_op=rhs_op, precond="mg", maxit=MAXIT, restart=20,
                                          use_graph=True)
    assert np.array_equal(it, itg) and torch.equal(x, xg)
    xs = split(x.cpu().numpy(), rhs_op, ops)
    for i, k in enumerate(rhs_op):
        med = meds[k]
        coef = op.helmholtz_coef(med.kappa2.astype(np.float32).astype(np.float64),
                                 med.gamma.astype(np.float32).astype(np.float64), med.omega)
        nz, nx = med.kappa2.shape
        bi = rhs[k][i - rhs_op.index(k)].astype(np.complex128).reshape(nz, nx)
        r = op.relres(coef, xs[i].reshape(1, nz, nx), bi.reshape(1, nz, nx), med.h, med.h)[0]
        assert abs(r - rr[i]) <= 1e-6 * max(r, 1e-12) + 1e-12, (i, r, rr[i])
        if st[i] == 0:
            assert r <= 1e-6
        assert it[i] <= MAXIT
