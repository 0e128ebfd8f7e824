"""ctypes declarations of the C-ABI in include/gkb.h (argument marshalling
only; every step of the solver runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgkb.so")

GKB_OK, GKB_MAXIT = 0, 1
GKB_EINVAL, GKB_ENOMEM, GKB_EHIP, GKB_ENAN, GKB_EINNER = -1, -2, -3, -4, -5
DIRICHLET, NATURAL = 0, 1
FP64, MIXED = 0, 1
INNER = {"jacobi": 0, "mg": 1, "learned": 2}
OPS = {"W": 0, "A": 1, "AT": 2, "M": 3, "diag": 4}
KERNELS = {"smooth": 0, "apply": 1, "resid": 2, "smooth_prolong": 3, "smooth_zero": 4}
SMOOTHERS = {"jacobi": 0, "hybrid": 1}
KRYLOV = {"cg": 0, "fgmres": 1}
METHODS = {"solver": 0, "precond": 1}
TRANSFERS = {"auto": 0, "div": 1, "smooth": 2}
SCALE_NONE, SCALE_CENTRAL = 0, 1

class Grid(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("h", C.c_double),
                ("bc", C.c_int * 6), ("pin_cell", C.c_int)]


class Csr(C.Structure):
    _fields_ = [("m", C.c_int), ("n", C.c_int),
                ("w_rowptr", C.POINTER(C.c_int)), ("w_col", C.POINTER(C.c_int)),
                ("w_val", C.POINTER(C.c_double)),
                ("a_rowptr", C.POINTER(C.c_int)), ("a_col", C.POINTER(C.c_int)),
                ("a_val", C.POINTER(C.c_double))]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("inner", C.c_int), ("mg_levels", C.c_int),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("inner_tol", C.c_double),
                ("inner_maxit", C.c_int), ("maxit", C.c_int), ("refine_tol", C.c_double),
                ("max_sweeps", C.c_int), ("check_every", C.c_int), ("use_graphs", C.c_int),
                ("stencil", C.c_int), ("smoother", C.c_int),
                ("hip_stream", C.c_void_p), ("max_workspace_bytes", C.c_size_t),
                ("krylov", C.c_int), ("fgmres_restart", C.c_int), ("method", C.c_int),
                ("outer_restart", C.c_int), ("cnn_weights", C.c_char_p),
                ("learned_min_gain", C.c_double), ("mg_transfer", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("sweeps", C.c_int), ("outer_iterations", C.c_int),
                ("inner_iterations", C.c_long), ("inner_solves", C.c_int),
                ("fallbacks", C.c_int), ("learned_solves", C.c_int), ("residual", C.c_double),
                ("error_estimate", C.c_double), ("seconds_solve", C.c_double),
                ("history_len", C.c_int), ("zeta", C.c_double * 512),
                ("estimate", C.c_double * 512), ("workspace_bytes", C.c_size_t),
                ("mg_levels", C.c_int), ("omega", C.c_double * 16),
                ("omega_edge", C.c_double * 16), ("learned_gain", C.c_double),
                ("learned_fallback_reason", C.c_int), ("learned_fallback_iteration", C.c_int),
                ("outer_krylov_iterations", C.c_int), ("mg_transfer", C.c_int)]


_lib = None


def lib():
    """Load libgkb.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python __graft_entry__.py build` (hipcc, gfx950)")
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    ctxp = C.c_void_p
    L.gkb_default_options.argtypes = [C.POINTER(Options)]
    L.gkb_default_options.restype = None
    L.gkb_setup.argtypes = [C.POINTER(Grid), P, C.c_double, C.POINTER(Options), C.POINTER(ctxp)]
    L.gkb_setup.restype = C.c_int
    L.gkb_solve.argtypes = [ctxp, P, P, C.c_double, C.c_int, P, P, C.POINTER(C.c_int),
                            C.POINTER(C.c_double)]
    L.gkb_solve.restype = C.c_int
    L.gkb_stats.argtypes = [ctxp, C.POINTER(Stats)]
    L.gkb_stats.restype = C.c_int
    L.gkb_sizes.argtypes = [ctxp] + [C.POINTER(C.c_long)] * 4
    L.gkb_sizes.restype = C.c_int
    L.gkb_strerror.argtypes = [C.c_int]
    L.gkb_strerror.restype = C.c_char_p
    L.gkb_destroy.argtypes = [ctxp]
    L.gkb_destroy.restype = None
    L.gkb_apply.argtypes = [ctxp, C.c_int, C.c_int, P, P]
    L.gkb_apply.restype = C.c_int
    L.gkb_precondition.argtypes = [ctxp, C.c_int, P, P]
    L.gkb_precondition.restype = C.c_int
    L.gkb_inner_solve.argtypes = [ctxp, P, P, C.c_double, C.POINTER(C.c_int)]
    L.gkb_inner_solve.restype = C.c_int
    L.gkb_residual.argtypes = [ctxp, P, P, P, P, P, P, P]
    L.gkb_residual.restype = C.c_int
    L.gkb_time_kernel.argtypes = [ctxp, C.c_int, C.c_int, C.POINTER(C.c_double)]
    L.gkb_time_kernel.restype = C.c_int
    L.gkb_setup_csr.argtypes = [C.POINTER(Csr), C.c_double, C.c_int, C.POINTER(Options),
                                C.POINTER(ctxp)]
    L.gkb_setup_csr.restype = C.c_int
    L.gkb_residual_noalloc.argtypes = [C.POINTER(Grid), P, P, P, P, P, P, P, P]
    L.gkb_residual_noalloc.restype = C.c_int
    _declare_cnn(L)
    _lib = L
    return L


def _declare_cnn(L):
    P = C.c_void_p
    I = C.c_int
    L.gkb_cnn_create.argtypes = [I, I, C.POINTER(I), C.c_uint, C.POINTER(P)]
    L.gkb_cnn_create.restype = I
    L.gkb_cnn_destroy.argtypes = [P]
    L.gkb_cnn_destroy.restype = None
    L.gkb_cnn_param_count.argtypes = [P]
    L.gkb_cnn_param_count.restype = C.c_long
    L.gkb_cnn_set_params.argtypes = [P, P]
    L.gkb_cnn_set_params.restype = I
    L.gkb_cnn_get_params.argtypes = [P, P]
    L.gkb_cnn_get_params.restype = I
    L.gkb_cnn_forward.argtypes = [P, I, I, I, I, P, P]
    L.gkb_cnn_forward.restype = I
    L.gkb_cnn_backward.argtypes = [P, I, I, I, I, P, P, P, P]
    L.gkb_cnn_backward.restype = I
    L.gkb_cnn_adam_step.argtypes = [P, P, C.c_double, C.c_double, C.c_double, C.c_double]
    L.gkb_cnn_adam_step.restype = I
    L.gkb_cnn_train.argtypes = [P, P, P, I, I, I, I, I, I, I, C.c_double, C.c_uint, P]
    L.gkb_cnn_train.restype = I
    L.gkb_cnn_eval.argtypes = [P, P, P, I, I, I, I, C.POINTER(C.c_double)]
    L.gkb_cnn_eval.restype = I
    L.gkb_cnn_save.argtypes = [P, C.c_char_p]
    L.gkb_cnn_save.restype = I
    L.gkb_cnn_load.argtypes = [C.c_char_p, C.POINTER(P)]
    L.gkb_cnn_load.restype = I
    L.gkb_attach_cnn.argtypes = [P, P]
    L.gkb_attach_cnn.restype = I
    L.gkb_set_capture.argtypes = [P, P, P, I, I, P]
    L.gkb_set_capture.restype = I
    L.gkb_capture_count.argtypes = [P, C.POINTER(I)]
    L.gkb_capture_count.restype = I


def check(rc: int, what: str = "gkb"):
    if rc < 0:
        msg = lib().gkb_strerror(rc).decode()
        raise RuntimeError(f"{what} failed: {msg} (code {rc})")
    return rc
