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


def helm_resample(f: torch.Tensor, mz: int, mx: int) -> torch.Tensor:
    """Bilinear resampling of a float32 [nz][nx] device field onto [mz][mx] (same extent)."""
    if f.dtype != torch.float32 or f.dim() != 2:
        raise TypeError("helm_resample takes a float32 [nz][nx] tensor")
    f = f.contiguous()
    out = torch.empty((mz, mx), dtype=torch.float32, device=f.device)
    L.check(L.load().helm_resample(_ptr(f), f.shape[0], f.shape[1], _ptr(out), int(mz), int(mx), _stream()))
    return out


def helm_vcycle_noalloc(op: HelmOp, f: torch.Tensor, e: torch.Tensor) -> torch.Tensor:
    """e = V_SL(f) without any allocation in the library (fixed scratch array); e must be given."""
    if f.dtype != torch.complex64 or e.dtype != torch.complex64 or e.numel() != f.numel():
        raise TypeError("helm_vcycle_noalloc takes complex64 f and e of one size")
    if f.numel() % op.n:
        raise ValueError("f size is not a multiple of the grid size")
    L.check(L.load().helm_vcycle_noalloc(op.handle, _ptr(f), _ptr(e), f.numel() // op.n, _stream()))
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
               reorth: bool = False, net=None, streams: int = 1):
    """Solve H x = b for a batch.  ops: HelmOp or list; rhs complex64, x complex128.
    streams=2 applies a CNN preconditioner to the two halves of each operator's
    batch on two streams.  Returns (x, iters, relres, status, code)."""
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
                    int(reorth), C.c_void_p(net.handle.value if net is not None else None), int(streams))
    it = (C.c_int * nrhs)()
    rr = (C.c_double * nrhs)()
    stt = (C.c_int * nrhs)()
    code = lib.helm_solve(handles, len(ops), ro, _ptr(rhs), _ptr(x), nrhs, float(tol), C.byref(o), it, rr, stt,
                          _stream())
    L.check(code, soft_ok=True)
    return (x, np.array(it[:], dtype=np.int64), np.array(rr[:], dtype=np.float64),
            np.array(stt[:], dtype=np.int64), code)


def helm_autotune(enable: int = -1) -> int:
    """Convolution kernel autotuning: 1 on, 0 off, 2 forget tuned shapes, -1 query.
    Returns the number of shapes tuned so far."""
    n = C.c_int()
    L.check(L.load().helm_autotune(int(enable), C.byref(n)))
    return n.value


def helm_conv_force(kernel: int = -1) -> int:
    """Pin the convolution kernel (an id below the returned count) wherever it
    applies, or remove the pin with -1.  Returns the number of kernel kinds."""
    n = C.c_int()
    L.check(L.load().helm_conv_force(int(kernel), C.byref(n)))
    return n.value


def helm_autotune_file(path, save: bool):
    """Save the tuned convolution kernel choices to, or merge them from, a text file."""
    L.check(L.load().helm_autotune_file(str(path).encode(), int(save)))


# ---------------------------------------------------------------- encoder-solver network
class CnnNet:
    """Owning wrapper of a cnn_net_t handle."""

    def __init__(self, handle):
        self.handle = handle

    @property
    def nparams(self):
        n = C.c_long()
        L.check(L.load().cnn_num_params(self.handle, C.byref(n)))
        return n.value

    def close(self):
        if self.handle:
            L.load().cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cnn_create(widths=(32, 64, 128, 256), seed=0, down_res=2) -> CnnNet:
    a = L.CnnArch((C.c_int * 4)(*widths), down_res)
    out = C.c_void_p()
    L.check(L.load().cnn_create(C.byref(a), int(seed), C.byref(out)))
    return CnnNet(out)


def cnn_load(path) -> CnnNet:
    out = C.c_void_p()
    L.check(L.load().cnn_load(str(path).encode(), C.byref(out)))
    return CnnNet(out)


def cnn_save(net: CnnNet, path):
    L.check(L.load().cnn_save(net.handle, str(path).encode()))


def cnn_get_params(net: CnnNet):
    import numpy as np
    a = np.empty(net.nparams, np.float32)
    L.check(L.load().cnn_get_params(net.handle, a.ctypes.data_as(C.c_void_p)))
    return a


def cnn_set_params(net: CnnNet, theta):
    import numpy as np
    a = np.ascontiguousarray(theta, dtype=np.float32)
    if a.size != net.nparams:
        raise ValueError(f"expected {net.nparams} parameters, got {a.size}")
    L.check(L.load().cnn_set_params(net.handle, a.ctypes.data_as(C.c_void_p)))


def cnn_get_grad(net: CnnNet):
    import numpy as np
    a = np.empty(net.nparams, np.float32)
    L.check(L.load().cnn_get_grad(net.handle, a.ctypes.data_as(C.c_void_p)))
    return a


def cnn_zero_grad(net: CnnNet):
    L.check(L.load().cnn_zero_grad(net.handle))


def cnn_forward(net: CnnNet, op: HelmOp, rin: torch.Tensor) -> torch.Tensor:
    """Raw network on scaled inputs rin [B][nz][nx][2] float32 (device)."""
    if rin.dtype != torch.float32 or rin.shape[1:] != (op.nz, op.nx, 2):
        raise ValueError("rin must be float32 [B][nz][nx][2]")
    out = torch.empty_like(rin)
    L.check(L.load().cnn_forward(net.handle, op.handle, _ptr(rin), _ptr(out), rin.shape[0], _stream()))
    return out


def cnn_precond_apply(net: CnnNet, op: HelmOp, r: torch.Tensor) -> torch.Tensor:
    if r.dtype != torch.complex64 or r.numel() % op.n:
        raise ValueError("r must be complex64 [nrhs][nz][nx]")
    e = torch.empty_like(r)
    L.check(L.load().cnn_precond_apply(net.handle, op.handle, _ptr(r), _ptr(e), r.numel() // op.n, _stream()))
    return e


def cnn_loss_grad(net: CnnNet, op: HelmOp, r: torch.Tensor, e: torch.Tensor) -> float:
    if r.dtype != torch.complex64 or e.dtype != torch.complex64 or r.shape != e.shape:
        raise ValueError("r, e must be complex64 of the same shape")
    loss = C.c_double()
    L.check(L.load().cnn_loss_grad(net.handle, op.handle, _ptr(r), _ptr(e), r.numel() // op.n, C.byref(loss),
                                   _stream()))
    return loss.value


def cnn_adam_step(net: CnnNet, lr=1e-4):
    L.check(L.load().cnn_adam_step(net.handle, float(lr), _stream()))


def cnn_make_pairs(op: HelmOp, first: int, npairs: int, seed: int):
    r = torch.empty((npairs, op.nz, op.nx), dtype=torch.complex64, device="cuda")
    e = torch.empty_like(r)
    L.check(L.load().cnn_make_pairs(op.handle, int(first), int(npairs), int(seed), _ptr(r), _ptr(e), _stream()))
    return r, e


def cnn_alg2_epoch(net: CnnNet, op: HelmOp, r: torch.Tensor, e: torch.Tensor, npairs: int):
    """r, e hold 2*npairs slots; the pairs spawned by the first npairs fill the rest."""
    if r.shape[0] < 2 * npairs or e.shape[0] < 2 * npairs:
        raise ValueError("r, e need room for 2*npairs pairs")
    L.check(L.load().cnn_alg2_epoch(net.handle, op.handle, _ptr(r), _ptr(e), int(npairs), _stream()))


def cnn_precond_train(net: CnnNet, op: HelmOp, npairs=2000, batch=16, steps=200, lr=1e-4, seed=0,
                      alg2_initial=0, alg2_data_epochs=0, alg2_epochs=0):
    import numpy as np
    done = C.c_int()
    dsz = C.c_int()
    o = L.TrainOpts(npairs, batch, steps, lr, alg2_initial, alg2_data_epochs, alg2_epochs, C.pointer(done),
                    C.pointer(dsz))
    hist = (C.c_float * (steps if steps > 0 else 200))()     # the library's default step count is 200
    L.check(L.load().cnn_precond_train(net.handle, op.handle, C.byref(o), int(seed), hist, _stream()))
    return np.array(hist[:done.value], dtype=np.float64), dsz.value


def _f32(a):
    import numpy as np
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def _vp(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def cnn_layer_resblock(x, w1, b1, w2, b2):
    """Fused 32-channel residual block through the library kernel; host float arrays, NHWC."""
    import numpy as np
    x = _f32(x)
    B, H, Wd, Cc = x.shape
    if Cc != 32:
        raise ValueError("the fused residual block takes 32 channels")
    out = np.empty_like(x)
    L.check(L.load().cnn_layer_resblock(B, H, Wd, _vp(x), _vp(_f32(w1)), _vp(_f32(b1)), _vp(_f32(w2)),
                                        _vp(_f32(b2)), _vp(out)))
    return out


def cnn_layer_forward(kind, stride, x1, w, b, x2=None, bcast2=False, resid=None, relu=True):
    """One layer through the library kernels; host float arrays, NHWC."""
    import numpy as np
    x1, x2, w, b, resid = _f32(x1), _f32(x2), _f32(w), _f32(b), _f32(resid)
    B, H, Wd, c1 = x1.shape
    c2 = 0 if x2 is None else x2.shape[-1]
    cout = w.shape[0] if kind == 0 else w.shape[2]
    Ho, Wo = ((H + stride - 1) // stride, (Wd + stride - 1) // stride) if kind == 0 else (2 * H, 2 * Wd)
    out = np.empty((B, Ho, Wo, cout), np.float32)
    L.check(L.load().cnn_layer_forward(kind, stride, B, H, Wd, c1, c2, int(bcast2), cout, _vp(x1), _vp(x2), _vp(w),
                                       _vp(b), _vp(resid), int(relu), _vp(out)))
    return out


def cnn_layer_backward(kind, stride, x1, w, y, gout, x2=None, bcast2=False, relu=True):
    import numpy as np
    x1, x2, w, y, gout = _f32(x1), _f32(x2), _f32(w), _f32(y), _f32(gout)
    B, H, Wd, c1 = x1.shape
    c2 = 0 if x2 is None else x2.shape[-1]
    cout = w.shape[0] if kind == 0 else w.shape[2]
    gx1 = np.empty_like(x1)
    gx2 = None if x2 is None else np.empty((B,) + x2.shape[1:], np.float32)
    gw = np.empty_like(w)
    gb = np.empty(cout, np.float32)
    L.check(L.load().cnn_layer_backward(kind, stride, B, H, Wd, c1, c2, int(bcast2), cout, _vp(x1), _vp(x2), _vp(w),
                                        _vp(y), int(relu), _vp(gout), _vp(gx1), _vp(gx2), _vp(gw), _vp(gb)))
    return gx1, gx2, gw, gb


# ---------------------------------------------------------------- FWI misfit and gradient
def fwi_misfit_grad(ops, src_idx, rec_idx, dobs: torch.Tensor, tol: float = 1e-6, precond: str = "mg",
                    restart: int = 0, maxit: int = 300, krylov_dtype: str = "c64", use_graph: bool = False,
                    reorth: bool = False, net=None, grad: torch.Tensor | None = None, streams: int = 1):
    """Misfit 1/2 sum |R u - d|^2 over frequencies (one op each) and sources, and its
    gradient w.r.t. the squared slowness.  src_idx / rec_idx: flat node indices;
    dobs complex64 [nfreq][nsrc][nrec] on the GPU.  Returns (misfit, grad float32
    [nz][nx], iters [2][nfreq][nsrc], code)."""
    import numpy as np
    lib = L.load()
    if isinstance(ops, HelmOp):
        ops = [ops]
    src = [int(v) for v in np.asarray(src_idx).ravel()]
    rec = [int(v) for v in np.asarray(rec_idx).ravel()]
    nf, ns, nr = len(ops), len(src), len(rec)
    if dobs.dtype != torch.complex64 or tuple(dobs.shape) != (nf, ns, nr):
        raise ValueError(f"dobs must be complex64 of shape {(nf, ns, nr)}")
    dobs = dobs.contiguous()
    if grad is None:
        grad = torch.empty((ops[0].nz, ops[0].nx), dtype=torch.float32, device=dobs.device)
    if grad.dtype != torch.float32 or grad.numel() != ops[0].n:
        raise ValueError("grad must be float32 [nz][nx]")
    handles = (C.c_void_p * nf)(*[o.handle for o in ops])
    o = L.SolveOpts(L.PRECOND[precond], restart, maxit, 0,
                    L.HELM_C64 if krylov_dtype == "c64" else L.HELM_C128, 0, int(use_graph),
                    int(reorth), C.c_void_p(net.handle.value if net is not None else None), int(streams))
    phi = C.c_double()
    its = (C.c_int * (2 * nf * ns))()
    code = lib.fwi_misfit_grad(handles, nf, (C.c_int * ns)(*src), ns, (C.c_int * nr)(*rec), nr, _ptr(dobs),
                               float(tol), C.byref(o), C.byref(phi), _ptr(grad), its, _stream())
    L.check(code, soft_ok=True)
    return phi.value, grad, np.array(its[:], dtype=np.int64).reshape(2, nf, ns), code


def fwi_misfit_grad_encoded(ops, src_idx, X, rec_idx, dobs: torch.Tensor, tol: float = 1e-6, precond: str = "mg",
                            restart: int = 0, maxit: int = 300, krylov_dtype: str = "c64", use_graph: bool = False,
                            reorth: bool = False, net=None, grad: torch.Tensor | None = None, streams: int = 1):
    """Simultaneous-source misfit 1/2 (1/p) sum |R H^{-1} G x_i - D x_i|^2 and its
    gradient (Sec. 3.2); X real [nsrc][p] (host), dobs the unencoded data,
    complex64 [nfreq][nsrc][nrec] on the GPU.  Returns (misfit, grad float32
    [nz][nx], iters [2][nfreq][p], code)."""
    import numpy as np
    lib = L.load()
    if isinstance(ops, HelmOp):
        ops = [ops]
    src = [int(v) for v in np.asarray(src_idx).ravel()]
    rec = [int(v) for v in np.asarray(rec_idx).ravel()]
    nf, ns, nr = len(ops), len(src), len(rec)
    Xh = np.ascontiguousarray(np.asarray(X, dtype=np.float32))
    if Xh.ndim != 2 or Xh.shape[0] != ns:
        raise ValueError(f"X must be [nsrc={ns}][p]")
    p = Xh.shape[1]
    if dobs.dtype != torch.complex64 or tuple(dobs.shape) != (nf, ns, nr):
        raise ValueError(f"dobs must be complex64 of shape {(nf, ns, nr)}")
    dobs = dobs.contiguous()
    if grad is None:
        grad = torch.empty((ops[0].nz, ops[0].nx), dtype=torch.float32, device=dobs.device)
    if grad.dtype != torch.float32 or grad.numel() != ops[0].n:
        raise ValueError("grad must be float32 [nz][nx]")
    handles = (C.c_void_p * nf)(*[o.handle for o in ops])
    o = L.SolveOpts(L.PRECOND[precond], restart, maxit, 0,
                    L.HELM_C64 if krylov_dtype == "c64" else L.HELM_C128, 0, int(use_graph),
                    int(reorth), C.c_void_p(net.handle.value if net is not None else None), int(streams))
    phi = C.c_double()
    its = (C.c_int * (2 * nf * p))()
    code = lib.fwi_misfit_grad_encoded(handles, nf, (C.c_int * ns)(*src), ns,
                                       Xh.ctypes.data_as(C.POINTER(C.c_float)), p, (C.c_int * nr)(*rec), nr,
                                       _ptr(dobs), float(tol), C.byref(o), C.byref(phi), _ptr(grad), its, _stream())
    L.check(code, soft_ok=True)
    return phi.value, grad, np.array(its[:], dtype=np.int64).reshape(2, nf, p), code


def _fwi_lin(name, ops, src_idx, rec_idx, x: torch.Tensor, tol, precond, restart, maxit, krylov_dtype, use_graph,
             reorth, net, streams=1):
    """Shared marshalling of fwi_born / fwi_born_adjoint / fwi_gn_hessvec."""
    import numpy as np
    lib = L.load()
    if isinstance(ops, HelmOp):
        ops = [ops]
    src = [int(v) for v in np.asarray(src_idx).ravel()]
    rec = [int(v) for v in np.asarray(rec_idx).ravel()]
    nf, ns, nr = len(ops), len(src), len(rec)
    if name == "fwi_born_adjoint":
        if x.dtype != torch.complex64 or tuple(x.shape) != (nf, ns, nr):
            raise ValueError(f"dd must be complex64 of shape {(nf, ns, nr)}")
        out = torch.empty((ops[0].nz, ops[0].nx), dtype=torch.float32, device=x.device)
    else:
        if x.dtype != torch.float32 or x.numel() != ops[0].n:
            raise ValueError("dm must be float32 [nz][nx]")
        out = (torch.empty((nf, ns, nr), dtype=torch.complex64, device=x.device) if name == "fwi_born" else
               torch.empty((ops[0].nz, ops[0].nx), dtype=torch.float32, device=x.device))
    x = x.contiguous()
    handles = (C.c_void_p * nf)(*[o.handle for o in ops])
    o = L.SolveOpts(L.PRECOND[precond], restart, maxit, 0,
                    L.HELM_C64 if krylov_dtype == "c64" else L.HELM_C128, 0, int(use_graph),
                    int(reorth), C.c_void_p(net.handle.value if net is not None else None), int(streams))
    nb = 3 if name == "fwi_gn_hessvec" else 2
    its = (C.c_int * (nb * nf * ns))()
    code = getattr(lib, name)(handles, nf, (C.c_int * ns)(*src), ns, (C.c_int * nr)(*rec), nr, _ptr(x), float(tol),
                              C.byref(o), _ptr(out), its, _stream())
    L.check(code, soft_ok=True)
    return out, np.array(its[:], dtype=np.int64).reshape(nb, nf, ns), code


def fwi_born(ops, src_idx, rec_idx, dm: torch.Tensor, tol: float = 1e-6, precond: str = "mg", restart: int = 0,
             maxit: int = 300, krylov_dtype: str = "c64", use_graph: bool = False, reorth: bool = False, net=None,
             streams: int = 1):
    """J dm: linearised data, complex64 [nfreq][nsrc][nrec].  Returns (jdm, iters [2][nfreq][nsrc], code)."""
    return _fwi_lin("fwi_born", ops, src_idx, rec_idx, dm, tol, precond, restart, maxit, krylov_dtype, use_graph,
                    reorth, net, streams)


def fwi_born_adjoint(ops, src_idx, rec_idx, dd: torch.Tensor, tol: float = 1e-6, precond: str = "mg",
                     restart: int = 0, maxit: int = 300, krylov_dtype: str = "c64", use_graph: bool = False,
                     reorth: bool = False, net=None, streams: int = 1):
    """Re(J^H dd), float32 [nz][nx].  Returns (out, iters [2][nfreq][nsrc], code)."""
    return _fwi_lin("fwi_born_adjoint", ops, src_idx, rec_idx, dd, tol, precond, restart, maxit, krylov_dtype,
                    use_graph, reorth, net, streams)


def fwi_gn_hessvec(ops, src_idx, rec_idx, dm: torch.Tensor, tol: float = 1e-6, precond: str = "mg",
                   restart: int = 0, maxit: int = 300, krylov_dtype: str = "c64", use_graph: bool = False,
                   reorth: bool = False, net=None, streams: int = 1):
    """Re(J^H J dm), the Gauss-Newton Hessian applied to dm, float32 [nz][nx].
    Returns (out, iters [3][nfreq][nsrc], code)."""
    return _fwi_lin("fwi_gn_hessvec", ops, src_idx, rec_idx, dm, tol, precond, restart, maxit, krylov_dtype,
                    use_graph, reorth, net, streams)


def _gn_opts(damping, cg_iters, tol_sens, reg, alpha, m_ref):
    if reg not in L.FWI_REG:
        raise ValueError(f"reg must be one of {sorted(L.FWI_REG)}")
    if reg != "none":
        if m_ref is None:
            raise ValueError("the regulariser needs m_ref")
        if m_ref.dtype != torch.float32 or not m_ref.is_contiguous():
            raise ValueError("m_ref must be a contiguous float32 tensor")
    return L.GnOpts(float(damping), int(cg_iters), float(tol_sens), L.FWI_REG[reg], float(alpha),
                    C.c_void_p(m_ref.data_ptr() if m_ref is not None else None))


def fwi_gn_cg(ops, src_idx, rec_idx, b: torch.Tensor, damping: float = 0.0, cg_iters: int = 10, tol: float = 1e-6,
              tol_sens: float = 0.0, reg: str = "none", alpha: float = 0.0, m_ref: torch.Tensor | None = None,
              precond: str = "mg", restart: int = 0, maxit: int = 300, krylov_dtype: str = "c64",
              use_graph: bool = False, reorth: bool = False, net=None, streams: int = 1):
    """cg_iters CG steps on (Re(J^H J) + alpha nabla^2 R + damping I) x = b from
    x = 0; b float32 [nz][nx] on the GPU; the point-source fields at tol, the
    Born and adjoint solves at tol_sens (<= 0: tol).  Returns (x float32
    [nz][nx], residual norms [cg_iters + 1], iters [cg_iters][2][nfreq][nsrc], code)."""
    import numpy as np
    lib = L.load()
    if isinstance(ops, HelmOp):
        ops = [ops]
    src = [int(v) for v in np.asarray(src_idx).ravel()]
    rec = [int(v) for v in np.asarray(rec_idx).ravel()]
    nf, ns, nr = len(ops), len(src), len(rec)
    if b.dtype != torch.float32 or b.numel() != ops[0].n:
        raise ValueError("b must be float32 [nz][nx]")
    b = b.contiguous()
    x = torch.empty((ops[0].nz, ops[0].nx), dtype=torch.float32, device=b.device)
    handles = (C.c_void_p * nf)(*[o.handle for o in ops])
    g = _gn_opts(damping, cg_iters, tol_sens, reg, alpha, m_ref)
    o = L.SolveOpts(L.PRECOND[precond], restart, maxit, 0,
                    L.HELM_C64 if krylov_dtype == "c64" else L.HELM_C128, 0, int(use_graph),
                    int(reorth), C.c_void_p(net.handle.value if net is not None else None), int(streams))
    norms = (C.c_double * (cg_iters + 1))()
    its = (C.c_int * max(1, 2 * cg_iters * nf * ns))()
    code = lib.fwi_gn_cg(handles, nf, (C.c_int * ns)(*src), ns, (C.c_int * nr)(*rec), nr, _ptr(b), C.byref(g),
                         float(tol), C.byref(o), _ptr(x), norms, its, _stream())
    L.check(code, soft_ok=True)
    it = np.array(its[:2 * cg_iters * nf * ns], dtype=np.int64).reshape(cg_iters, 2, nf, ns)
    return x, np.array(norms[:], dtype=np.float64), it, code


def fwi_gn_step(ops, src_idx, rec_idx, dobs: torch.Tensor, m: torch.Tensor, damping: float, cg_iters: int,
                mu: float = 1.0, tol: float = 1e-6, tol_sens: float = 0.0, reg: str = "none", alpha: float = 0.0,
                m_ref: torch.Tensor | None = None, precond: str = "mg", restart: int = 0, maxit: int = 300,
                krylov_dtype: str = "c64", use_graph: bool = False, reorth: bool = False, net=None,
                m_new: torch.Tensor | None = None, streams: int = 1):
    """One Gauss-Newton step m + mu dm on Phi + alpha R, dm from CG on
    (Re(J^H J) + alpha nabla^2 R + damping I) dm = -grad; ops must be set up
    with m.  Returns a dict: m_new, misfit (data misfit at m), reg (R(m)),
    grad (dPhi/dm + alpha dR/dm), norms (CG residual norms), iters
    [2 + 2 cg_iters][nfreq][nsrc], code."""
    import numpy as np
    lib = L.load()
    if isinstance(ops, HelmOp):
        ops = [ops]
    src = [int(v) for v in np.asarray(src_idx).ravel()]
    rec = [int(v) for v in np.asarray(rec_idx).ravel()]
    nf, ns, nr = len(ops), len(src), len(rec)
    if dobs.dtype != torch.complex64 or tuple(dobs.shape) != (nf, ns, nr):
        raise ValueError(f"dobs must be complex64 of shape {(nf, ns, nr)}")
    if m.dtype != torch.float32 or m.numel() != ops[0].n:
        raise ValueError("m must be float32 [nz][nx]")
    dobs, m = dobs.contiguous(), m.contiguous()
    m_new = torch.empty_like(m) if m_new is None else m_new
    grad = torch.empty_like(m)
    handles = (C.c_void_p * nf)(*[o.handle for o in ops])
    g = _gn_opts(damping, cg_iters, tol_sens, reg, alpha, m_ref)
    o = L.SolveOpts(L.PRECOND[precond], restart, maxit, 0,
                    L.HELM_C64 if krylov_dtype == "c64" else L.HELM_C128, 0, int(use_graph),
                    int(reorth), C.c_void_p(net.handle.value if net is not None else None), int(streams))
    phi = C.c_double()
    rv = C.c_double()
    norms = (C.c_double * (cg_iters + 1))()
    nb = 2 + 2 * cg_iters
    its = (C.c_int * (nb * nf * ns))()
    code = lib.fwi_gn_step(handles, nf, (C.c_int * ns)(*src), ns, (C.c_int * nr)(*rec), nr, _ptr(dobs), _ptr(m),
                           C.byref(g), float(mu), float(tol), C.byref(o), _ptr(m_new), C.byref(phi), C.byref(rv),
                           _ptr(grad), norms, its, _stream())
    L.check(code, soft_ok=True)
    return {"m_new": m_new, "misfit": phi.value, "reg": rv.value, "grad": grad,
            "norms": np.array(norms[:], dtype=np.float64),
            "iters": np.array(its[:], dtype=np.int64).reshape(nb, nf, ns), "code": code}


def fwi_release_workspace():
    """Free the FWI entry points' device workspace pool."""
    L.check(L.load().fwi_release_workspace())


class FwiMisfit(torch.autograd.Function):
    """Phi(m) = 1/2 sum_{f,s} |R H_f(m)^{-1} g_s - d_fs|^2 as a differentiable function
    of the squared slowness m (float32 [nz][nx] on the GPU).  The forward pass runs
    the forward and adjoint solve batches in the library and keeps dPhi/dm; the
    backward pass scales it by the incoming gradient.

        phi = FwiMisfit.apply(m, gamma, omegas, h, src_idx, rec_idx, dobs, solve_kw)
    """

    @staticmethod
    def forward(ctx, m, gamma, omegas, h, src_idx, rec_idx, dobs, solve_kw=None):
        kw = dict(solve_kw or {})
        ops = [helm_setup(m.detach(), gamma, float(w), h) for w in omegas]
        try:
            phi, grad, its, code = fwi_misfit_grad(ops, src_idx, rec_idx, dobs, **kw)
        finally:
            for o in ops:
                o.close()
        ctx.save_for_backward(grad)
        ctx.mdtype = m.dtype
        ctx.iters = its
        ctx.code = code
        return torch.tensor(phi, dtype=torch.float64, device=m.device)

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return ((gout.to(torch.float64) * grad.to(torch.float64)).to(ctx.mdtype),
                None, None, None, None, None, None, None)


def fwi_misfit(m, gamma, omegas, h, src_idx, rec_idx, dobs, **solve_kw):
    """Differentiable misfit; see FwiMisfit."""
    return FwiMisfit.apply(m, gamma, omegas, h, src_idx, rec_idx, dobs, solve_kw)
