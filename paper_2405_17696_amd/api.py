"""Python binding of libhelm with the C entry-point names.

Argument marshalling only: tensors must already be on the GPU (torch supplies
device memory and the current stream); every step runs in the library's HIP
kernels.  Complex tensors are torch.complex64 / torch.complex128 laid out
[nrhs][nz][nx] (or flat, back to back, for ragged batches).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("libhelm takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libhelm takes contiguous tensors")
    return C.c_void_p(t.data_ptr())


class HelmOp:
    """Owning wrapper of a helm_op_t handle."""

    def __init__(self, handle, nz, nx, omega, hx, hz):
        self.handle = handle
        self.nz, self.nx, self.omega, self.hx, self.hz = nz, nx, omega, hx, hz

    @property
    def n(self):
        return self.nz * self.nx

    def close(self):
        if self.handle:
            L.load().helm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def helm_setup(kappa2: torch.Tensor, gamma: torch.Tensor, omega: float, h: float, hz: float | None = None,
               sl_beta: float = 0.5, sl_no_gamma: bool = False, mg_levels: int = 3, coarse_degree: int = 20,
               jacobi_weight: float = 0.8) -> HelmOp:
    lib = L.load()
    k2 = kappa2.to(device="cuda", dtype=torch.float32).contiguous()
    g = gamma.to(device="cuda", dtype=torch.float32).contiguous()
    nz, nx = k2.shape
    o = L.SetupOpts(hz or 0.0, sl_beta, int(sl_no_gamma), mg_levels, coarse_degree, jacobi_weight)
    out = C.c_void_p()
    L.check(lib.helm_setup(_ptr(k2), _ptr(g), nz, nx, float(omega), float(h), C.byref(o), _stream(), C.byref(out)))
    torch.cuda.current_stream().synchronize()
    return HelmOp(out, nz, nx, float(omega), float(h), float(hz or h))


def helm_matvec(op: HelmOp, u: torch.Tensor, v: torch.Tensor | None = None, adjoint: bool = False) -> torch.Tensor:
    if u.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("helm_matvec takes complex64 or complex128")
    if u.numel() % op.n:
        raise ValueError("u size is not a multiple of the grid size")
    v = torch.empty_like(u) if v is None else v
    if v.dtype != u.dtype or v.numel() != u.numel():
        raise ValueError("v must match u")
    dt = L.HELM_C64 if u.dtype == torch.complex64 else L.HELM_C128
    L.check(L.load().helm_matvec(op.handle, _ptr(u), _ptr(v), u.numel() // op.n, dt, int(adjoint), _stream()))
    return v


def helm_vcycle(op: HelmOp, f: torch.Tensor, e: torch.Tensor | None = None) -> torch.Tensor:
    if f.dtype != torch.complex64:
        raise TypeError("helm_vcycle takes complex64")
    if f.numel() % op.n:
        raise ValueError("f size is not a multiple of the grid size")
    e = torch.empty_like(f) if e is None else e
    L.check(L.load().helm_vcycle(op.handle, _ptr(f), _ptr(e), f.numel() // op.n, _stream()))
    return e


def helm_coarse_roots(op: HelmOp):
    import numpy as np
    lib = L.load()
    n = C.c_int()
    L.check(lib.helm_coarse_roots(op.handle, None, C.byref(n)))
    buf = (C.c_double * (2 * n.value))()
    L.check(lib.helm_coarse_roots(op.handle, buf, C.byref(n)))
    a = np.frombuffer(buf, dtype=np.float64)
    return a[0::2] + 1j * a[1::2]


def helm_solve(ops, rhs: torch.Tensor, x: torch.Tensor | None = None, tol: float = 1e-6, rhs_op=None,
               precond: str = "mg", restart: int = 0, maxit: int = 300, adjoint: bool = False,
               krylov_dtype: str = "c64", x0_given: bool = False, use_graph: bool = False,
               reorth: bool = False, net=None):
    """Solve H x = b for a batch.  ops: HelmOp or list; rhs complex64, x complex128.
    Returns (x, iters, relres, status, code)."""
    import numpy as np
    lib = L.load()
    if isinstance(ops, HelmOp):
        ops = [ops]
    if rhs.dtype != torch.complex64:
        raise TypeError("rhs must be complex64")
    if rhs_op is None:
        if rhs.numel() % ops[0].n:
            raise ValueError("rhs size is not a multiple of the grid size")
        rhs_op = [0] * (rhs.numel() // ops[0].n)
    nrhs = len(rhs_op)
    ntot = sum(ops[k].n for k in rhs_op)
    if rhs.numel() != ntot:
        raise ValueError(f"rhs has {rhs.numel()} entries, operators need {ntot}")
    if x is None:
        x = torch.empty(rhs.shape, dtype=torch.complex128, device=rhs.device)
    if x.dtype != torch.complex128 or x.numel() != ntot:
        raise ValueError("x must be complex128 with the size of rhs")
    handles = (C.c_void_p * len(ops))(*[o.handle for o in ops])
    ro = (C.c_int * nrhs)(*rhs_op)
    o = L.SolveOpts(L.PRECOND[precond], restart, maxit, int(adjoint),
                    L.HELM_C64 if krylov_dtype == "c64" else L.HELM_C128, int(x0_given), int(use_graph),
                    int(reorth), C.c_void_p(net.handle.value if net is not None else None))
    it = (C.c_int * nrhs)()
    rr = (C.c_double * nrhs)()
    stt = (C.c_int * nrhs)()
    code = lib.helm_solve(handles, len(ops), ro, _ptr(rhs), _ptr(x), nrhs, float(tol), C.byref(o), it, rr, stt,
                          _stream())
    L.check(code, soft_ok=True)
    return (x, np.array(it[:], dtype=np.int64), np.array(rr[:], dtype=np.float64),
            np.array(stt[:], dtype=np.int64), code)
