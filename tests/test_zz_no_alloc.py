"""The allocation-free V-cycle entry point against helm_vcycle, through the C
ABI: the same kernels on the same inputs give the same bits, on two calls in a
row (the second with fewer right-hand sides, on another grid, so that the
fixed scratch array holds the first call's values when the second starts), and
a request beyond the fixed scratch size is refused."""
import ctypes as C

import numpy as np
import pytest
import torch

from helpers import medium, rand_c
from paper_2405_17696_amd import _lib as L
from paper_2405_17696_amd import api

pytestmark = pytest.mark.gpu


def setup(med):
    return api.helm_setup(torch.tensor(med.kappa2, dtype=torch.float32, device="cuda"),
                          torch.tensor(med.gamma, dtype=torch.float32, device="cuda"), med.omega, med.h)


def noalloc(op, f):
    e = torch.full_like(f, float("nan"))
    code = L.load().helm_vcycle_noalloc(op.handle, C.c_void_p(f.data_ptr()), C.c_void_p(e.data_ptr()),
                                        f.numel() // op.n, C.c_void_p(torch.cuda.current_stream().cuda_stream))
    L.check(code)
    torch.cuda.synchronize()
    return e


def test_noalloc_vcycle_equals_vcycle(gpu):
    lib = L.load()
    assert lib.helm_vcycle_noalloc_max_bytes() == 32 << 20
    big = medium(256, 256, seed=71, kind="layered")
    small = medium(96, 64, seed=72)
    Hb, Hs = setup(big), setup(small)
    fb = torch.tensor(rand_c((24, 256, 256), 73).astype(np.complex64), device="cuda")
    fs = torch.tensor(rand_c((5, 96, 64), 74).astype(np.complex64), device="cuda")
    for H, f in ((Hb, fb), (Hs, fs), (Hb, fb[:3].contiguous())):
        print("noalloc vcycle", tuple(f.shape), flush=True)
        ref = api.helm_vcycle(H, f)
        got = noalloc(H, f)
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref)
    # beyond the fixed scratch: 65 right-hand sides of 256 x 256 need 32.5 MiB
    f65 = torch.zeros((65, 256, 256), dtype=torch.complex64, device="cuda")
    e65 = torch.empty_like(f65)
    code = lib.helm_vcycle_noalloc(Hb.handle, C.c_void_p(f65.data_ptr()), C.c_void_p(e65.data_ptr()), 65,
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code == L.HELM_EINVAL and b"scratch" in lib.helm_last_error()
    # an empty batch is a no-op
    assert lib.helm_vcycle_noalloc(Hb.handle, None, None, 0, None) == 0
    Hb.close()
    Hs.close()
