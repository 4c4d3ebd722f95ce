"""ctypes binding of ``include/jfnk.h``: argument marshalling only.

Device memory comes from torch tensors (``tensor.data_ptr()``) and the stream
from ``torch.cuda.current_stream().cuda_stream``; every computation runs in the
HIP library.  Loading fails loudly if ``libjfnk.so`` has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjfnk.so")

JFNK_OK, JFNK_NOT_CONVERGED, JFNK_ERR_ARG, JFNK_ERR_HIP, JFNK_ERR_NONFINITE = 0, 1, -1, -2, -3
F64, F32 = 0, 1
PC_NONE, PC_PHYSICS, PC_LEARNED = 0, 1, 2
JV_STABLE, JV_LITERAL, JV_ANALYTIC = 0, 1, 2
ORTHO_CGS2, ORTHO_ONE_REDUCTION = 0, 1
NET_LOSS_SOLUTION, NET_LOSS_REST_JACOBIAN = 0, 1
KC_JV, KC_RESIDUAL, KC_PC, KC_ARNOLDI, KC_VEC, KC_NET = range(6)

EXPORTS = ["jfnk_create", "jfnk_destroy", "jfnk_last_error", "jfnk_set_stream", "jfnk_rhs",
           "jfnk_residual", "jfnk_apply_F", "jfnk_jv", "jfnk_precond_apply", "jfnk_gmres",
           "jfnk_newton_step", "jfnk_norm", "jfnk_timing_enable", "jfnk_timing_read",
           "jfnk_net_init", "jfnk_net_set_params", "jfnk_net_get_params", "jfnk_net_apply",
           "jfnk_nlpc_residual", "jfnk_nlpc_step", "jfnk_net_set_loss", "jfnk_net_loss_grad", "jfnk_net_train_step", "jfnk_tune", "jfnk_set_variant",
           "jfnk_batch_create", "jfnk_batch_destroy", "jfnk_batch_size", "jfnk_batch_apply_F",
           "jfnk_batch_newton_step", "jfnk_batch_tune", "jfnk_jv_noalloc"]


class Problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double), ("dt", C.c_double),
                ("theta0", C.c_double), ("g", C.c_double), ("cp", C.c_double), ("cv", C.c_double),
                ("rgas", C.c_double), ("p_ref", C.c_double), ("kappa_div", C.c_double),
                ("n_bv", C.c_double), ("closure", C.c_int32), ("cs", C.c_double), ("pr_t", C.c_double),
                ("k_m", C.c_double), ("k_h", C.c_double), ("bc_lateral", C.c_int32),
                ("bc_vertical", C.c_int32), ("h0", C.c_double), ("strip_width", C.c_double),
                ("strip_center", C.c_double), ("strip_shape", C.c_int32), ("strip_xi", C.c_double),
                ("convection", C.c_int32), ("energy_test", C.c_int32), ("dd_p", C.c_int32)]


class GmresOpts(C.Structure):
    _fields_ = [("m", C.c_int32), ("max_restarts", C.c_int32), ("tol", C.c_double), ("pc", C.c_int32),
                ("jv", C.c_int32), ("sweeps", C.c_int32), ("max_iters", C.c_int32), ("ortho", C.c_int32),
                ("no_judge", C.c_int32)]


class GmresInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("res0", C.c_double), ("res_est", C.c_double), ("h_out", C.POINTER(C.c_double)),
                ("fallback", C.c_int32), ("res_true", C.c_double)]


class NewtonOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol_factor", C.c_double), ("max_newton", C.c_int32),
                ("inner", C.c_int32), ("gm", GmresOpts), ("forcing", C.c_int32), ("eta", C.c_double),
                ("eta_floor", C.c_double), ("rec_r", C.c_void_p), ("rec_du", C.c_void_p),
                ("rec_cap", C.c_int32), ("rec_count", C.POINTER(C.c_int32)), ("rec_krylov", C.c_int32)]


class NewtonInfo(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("gmres_iters_total", C.c_int32), ("converged", C.c_int32),
                ("fallbacks", C.c_int32), ("res0", C.c_double), ("res_final", C.c_double)]


_lib = None


def lib_available() -> bool:
    return os.path.exists(LIB_PATH)


def load():
    """Load the HIP library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2007_10411_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.jfnk_create.argtypes = [C.POINTER(Problem), C.c_int32, vp, C.POINTER(vp)]
    L.jfnk_destroy.argtypes = [vp]
    L.jfnk_last_error.restype = C.c_char_p
    L.jfnk_set_stream.argtypes = [vp, vp]
    L.jfnk_rhs.argtypes = [vp, vp, vp]
    L.jfnk_residual.argtypes = [vp, vp, vp, vp]
    L.jfnk_apply_F.argtypes = [vp, C.c_int, C.c_int32, vp, vp, vp]
    L.jfnk_jv.argtypes = [vp, C.c_int, C.c_int, vp, vp, C.c_double, vp]
    L.jfnk_precond_apply.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, C.c_int32]
    L.jfnk_gmres.argtypes = [vp, C.c_int, vp, vp, vp, C.POINTER(GmresOpts), C.POINTER(GmresInfo)]
    L.jfnk_newton_step.argtypes = [vp, vp, vp, C.POINTER(NewtonOpts), C.POINTER(NewtonInfo)]
    L.jfnk_norm.argtypes = [vp, C.c_int, vp, C.c_int64, C.POINTER(C.c_double)]
    L.jfnk_timing_enable.argtypes = [vp, C.c_int32]
    L.jfnk_timing_read.argtypes = [vp, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]
    L.jfnk_net_init.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
    L.jfnk_net_set_params.argtypes = [vp, vp, C.c_int64]
    L.jfnk_net_get_params.argtypes = [vp, vp, C.c_int64]
    L.jfnk_net_apply.argtypes = [vp, C.c_int32, vp, vp]
    L.jfnk_net_set_loss.argtypes = [vp, C.c_int32]
    L.jfnk_nlpc_residual.argtypes = [vp, vp, vp, vp, C.c_int32]
    L.jfnk_nlpc_step.argtypes = [vp, vp, vp, C.POINTER(NewtonOpts), C.c_int32, C.POINTER(NewtonInfo)]
    L.jfnk_net_loss_grad.argtypes = [vp, vp, vp, C.c_int32, C.POINTER(C.c_double), vp]
    L.jfnk_net_train_step.argtypes = [vp, vp, vp, C.c_int32, C.POINTER(C.c_int32), C.c_float, C.POINTER(C.c_double)]
    L.jfnk_tune.argtypes = [vp, C.POINTER(C.c_int32)]
    L.jfnk_set_variant.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    L.jfnk_batch_create.argtypes = [C.POINTER(Problem), C.c_int32, C.c_int32, vp, C.POINTER(vp)]
    L.jfnk_batch_destroy.argtypes = [vp]
    L.jfnk_batch_size.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.jfnk_batch_apply_F.argtypes = [vp, C.c_int32, vp, vp, vp]
    L.jfnk_batch_newton_step.argtypes = [vp, vp, vp, C.POINTER(NewtonOpts), C.POINTER(NewtonInfo), C.c_int32]
    L.jfnk_batch_tune.argtypes = [vp, C.POINTER(C.c_int32)]
    L.jfnk_jv_noalloc.argtypes = [C.POINTER(Problem), C.c_int, C.c_int, vp, vp, C.c_double, vp, vp]
    for name in EXPORTS:
        if name != "jfnk_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


class JfnkError(RuntimeError):
    def __init__(self, code, where):
        msg = load().jfnk_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with code {code}: {msg}")
        self.code = code


def check(code, where, soft_ok=True):
    if code == JFNK_OK or (soft_ok and code == JFNK_NOT_CONVERGED):
        return code
    raise JfnkError(code, where)


def problem_struct(p) -> Problem:
    s = Problem()
    for name, _ in Problem._fields_:
        setattr(s, name, getattr(p, name))
    return s
