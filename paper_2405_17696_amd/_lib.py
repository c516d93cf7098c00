"""ctypes loader for libhelm.so (argument marshalling only; all compute is in the library).

The library is loaded from the package directory.  There is no fallback: if
the shared object is missing or cannot be loaded, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libhelm.so"

HELM_OK = 0
HELM_NOT_CONVERGED = 1
HELM_EINVAL = -1
HELM_ENOMEM = -2
HELM_EHIP = -3
HELM_ENAN = -4
HELM_C64 = 0
HELM_C128 = 1
PRECOND = {"mg": 0, "none": 1, "cnn": 2, "cnn_vu": 3}


class HelmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libhelm error {code}: {msg}")
        self.code = code


class SetupOpts(C.Structure):
    _fields_ = [("hz", C.c_double), ("sl_beta", C.c_double), ("sl_no_gamma", C.c_int),
                ("mg_levels", C.c_int), ("coarse_degree", C.c_int), ("jacobi_weight", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("precond", C.c_int), ("restart", C.c_int), ("maxit", C.c_int), ("adjoint", C.c_int),
                ("krylov_dtype", C.c_int), ("x0_given", C.c_int), ("use_graph", C.c_int),
                ("reorth", C.c_int), ("net", C.c_void_p), ("streams", C.c_int)]


class CnnArch(C.Structure):
    _fields_ = [("widths", C.c_int * 4), ("down_res", C.c_int)]


class TrainOpts(C.Structure):
    _fields_ = [("npairs", C.c_int), ("batch", C.c_int), ("steps", C.c_int), ("lr", C.c_double),
                ("alg2_initial", C.c_int), ("alg2_data_epochs", C.c_int), ("alg2_epochs", C.c_int),
                ("steps_done", C.POINTER(C.c_int)), ("dataset_size", C.POINTER(C.c_int))]


class GnOpts(C.Structure):
    _fields_ = [("damping", C.c_double), ("cg_iters", C.c_int), ("tol_sens", C.c_double), ("reg", C.c_int),
                ("alpha", C.c_double), ("m_ref", C.c_void_p)]


FWI_REG = {"none": 0, "high": 1, "diff": 2}

_lib = None

# name -> (restype, argtypes); every exported symbol of include/*.h is listed here
SIGNATURES = {
    "helm_setup": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double,
                             C.POINTER(SetupOpts), C.c_void_p, C.POINTER(C.c_void_p)]),
    "helm_destroy": (None, [C.c_void_p]),
    "helm_op_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double),
                               C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "helm_matvec": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]),
    "helm_solve": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.c_void_p, C.c_void_p,
                             C.c_int, C.c_double, C.POINTER(SolveOpts), C.POINTER(C.c_int),
                             C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p]),
    "helm_vcycle": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "helm_resample": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_void_p, C.c_int, C.c_int, C.c_void_p]),
    "helm_vcycle_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "helm_vcycle_noalloc_max_bytes": (C.c_size_t, []),
    "helm_coarse_roots": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    "cnn_create": (C.c_int, [C.POINTER(CnnArch), C.c_uint64, C.POINTER(C.c_void_p)]),
    "cnn_destroy": (None, [C.c_void_p]),
    "cnn_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "cnn_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_void_p)]),
    "cnn_num_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_long)]),
    "cnn_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "cnn_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "cnn_get_grad": (C.c_int, [C.c_void_p, C.c_void_p]),
    "cnn_zero_grad": (C.c_int, [C.c_void_p]),
    "cnn_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "cnn_precond_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "cnn_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                C.c_void_p]),
    "cnn_adam_step": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p]),
    "cnn_make_pairs": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "cnn_alg2_epoch": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p]),
    "cnn_layer_resblock": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "helm_autotune": (C.c_int, [C.c_int, C.POINTER(C.c_int)]),
    "helm_autotune_file": (C.c_int, [C.c_char_p, C.c_int]),
    "helm_conv_force": (C.c_int, [C.c_int, C.POINTER(C.c_int)]),
    "fwi_misfit_grad": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.c_int,
                                  C.POINTER(C.c_int), C.c_int, C.c_void_p, C.c_double, C.POINTER(SolveOpts),
                                  C.POINTER(C.c_double), C.c_void_p, C.POINTER(C.c_int), C.c_void_p]),
    "fwi_misfit_grad_encoded": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.c_int,
                                          C.POINTER(C.c_float), C.c_int, C.POINTER(C.c_int), C.c_int, C.c_void_p,
                                          C.c_double, C.POINTER(SolveOpts), C.POINTER(C.c_double), C.c_void_p,
                                          C.POINTER(C.c_int), C.c_void_p]),
    "fwi_born": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int), C.c_int,
                           C.c_void_p, C.c_double, C.POINTER(SolveOpts), C.c_void_p, C.POINTER(C.c_int), C.c_void_p]),
    "fwi_born_adjoint": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int),
                                   C.c_int, C.c_void_p, C.c_double, C.POINTER(SolveOpts), C.c_void_p,
                                   C.POINTER(C.c_int), C.c_void_p]),
    "fwi_gn_hessvec": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int),
                                 C.c_int, C.c_void_p, C.c_double, C.POINTER(SolveOpts), C.c_void_p,
                                 C.POINTER(C.c_int), C.c_void_p]),
    "fwi_gn_cg": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int), C.c_int,
                            C.c_void_p, C.POINTER(GnOpts), C.c_double, C.POINTER(SolveOpts), C.c_void_p,
                            C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p]),
    "fwi_gn_step": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int),
                              C.c_int, C.c_void_p, C.c_void_p, C.POINTER(GnOpts), C.c_double, C.c_double,
                              C.POINTER(SolveOpts), C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p]),
    "fwi_release_workspace": (C.c_int, []),
    "cnn_precond_train": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(TrainOpts), C.c_uint64,
                                    C.POINTER(C.c_float), C.c_void_p]),
    "cnn_layer_forward": (C.c_int, [C.c_int] * 9 + [C.c_void_p] * 5 + [C.c_int, C.c_void_p]),
    "cnn_layer_backward": (C.c_int, [C.c_int] * 9 + [C.c_void_p] * 4 + [C.c_int] + [C.c_void_p] * 5),
    "helm_ktimer_start": (C.c_int, [C.c_char_p]),
    "helm_ktimer_sample": (C.c_int, [C.c_int]),
    "helm_ktimer_sample_steps": (C.c_int, [C.c_int]),
    "helm_ktimer_count": (C.c_int, [C.POINTER(C.c_longlong)]),
    "helm_ktimer_read": (C.c_int, [C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "helm_ktimer_busy": (C.c_int, [C.POINTER(C.c_double)]),
    "helm_last_error": (C.c_char_p, []),
    "helm_version": (C.c_char_p, []),
}


def load():
    """Load libhelm.so (once).  Raises if it is missing: there is no CPU fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise HelmError(HELM_EINVAL, f"{LIB_PATH} not built; run __graft_entry__.build()")
    lib = C.CDLL(str(LIB_PATH))
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code, soft_ok=False):
    if code == HELM_OK or (soft_ok and code == HELM_NOT_CONVERGED):
        return code
    msg = load().helm_last_error().decode(errors="replace")
    raise HelmError(code, msg)
