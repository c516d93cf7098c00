"""Shared test inputs: seeded media rounded to float32 exactly as the GPU
library stores them, so the oracle and the library define the same operator."""
from __future__ import annotations

import numpy as np

from paper_2405_17696_amd import synth


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def medium(nz, nx, seed=7, ppw=10.0, kind="grf", h=synth.H_DEFAULT):
    rng = np.random.default_rng(seed)
    if kind == "grf":
        c = synth.velocity_grf(nz, nx, rng)
    elif kind == "layered":
        c = synth.velocity_layered(nz, nx, rng)
    else:
        c = np.full((nz, nx), 1.5)
    med = synth.medium_from_velocity(c, ppw=ppw, h=h)
    med.kappa2 = f32(med.kappa2)
    med.gamma = f32(med.gamma)
    return med


def rand_c(shape, seed):
    return synth.random_complex(shape, np.random.default_rng(seed))


def relerr(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
