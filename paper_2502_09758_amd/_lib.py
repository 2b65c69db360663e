"""ctypes binding of libmaid.so (argument marshalling only).

Every function here checks shapes, dtypes and devices of torch tensors and
passes raw device pointers and the current HIP stream to the C ABI declared
in include/maid.h; all computation happens in the HIP kernels.  If the
library is missing the import of the functions fails loudly: there is no
fallback path.
"""
from __future__ import annotations

import ctypes as ct
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmaid.so")

MAID_F32, MAID_F64 = 0, 1
MAID_BOUNDARY_ZERO, MAID_BOUNDARY_PERIODIC = 0, 1
MAID_REG_TV, MAID_REG_TV_CHANNELWISE, MAID_REG_QUADRATIC = 0, 1, 2
OK, MAXITER, ACCURACY_FLOOR = 0, 1, 2
EINVAL, ENOMEM, EHIP, NOT_SPD, NONFINITE = -1, -2, -3, -4, -5
CODE_NAMES = {OK: "OK", MAXITER: "MAXITER", ACCURACY_FLOOR: "ACCURACY_FLOOR", EINVAL: "EINVAL",
              ENOMEM: "ENOMEM", EHIP: "EHIP", NOT_SPD: "NOT_SPD", NONFINITE: "NONFINITE"}

# every entry point declared in include/maid.h
EXPORTS = ("maid_create", "maid_destroy", "maid_last_error", "maid_config_string",
           "maid_set_tile_rows", "maid_set_team", "maid_set_one_pass_cg", "maid_set_mfma", "maid_set_one_pass", "maid_one_pass_forms", "maid_lower_solve", "maid_upper_value_grad",
           "maid_adjoint_solve", "maid_hypergrad", "maid_apply_operator", "maid_sobolev_value", "maid_step",
           "maid_profile", "maid_profile_read", "maid_profile_name",
           "maid_create_batch", "maid_batch_size", "maid_batch_lower_solve", "maid_batch_adjoint_solve",
           "maid_batch_step", "maid_autotune", "maid_batch_upper_value_grad", "maid_batch_hypergrad",
           "maid_set_step_trace", "maid_step_trace_length", "maid_lower_solve_refined",
           "maid_upper_value_grad_noalloc", "maid_batch_create", "maid_batch_steps",
           "maid_gd_solve", "maid_hessian_apply", "maid_ift_step", "maid_lista_step",
           "maid1d_create", "maid1d_destroy", "maid1d_last_error", "maid1d_lower_solve", "maid1d_upper_value_grad",
           "maid1d_adjoint_solve", "maid1d_hypergrad", "maid1d_step")
PROF_KINDS = 12


class maid_desc(ct.Structure):
    _fields_ = [("H", ct.c_int32), ("W", ct.c_int32), ("C", ct.c_int32), ("K", ct.c_int32),
                ("dtype", ct.c_int32), ("boundary", ct.c_int32), ("reg", ct.c_int32), ("kc", ct.c_int32),
                ("alpha", ct.c_double),
                ("eps_tv", ct.c_double), ("beta", ct.c_double), ("h1_w0", ct.c_double)]


class maid_solve_info(ct.Structure):
    _fields_ = [("iters", ct.c_int32), ("backtracks", ct.c_int32), ("status", ct.c_int32),
                ("res_norm", ct.c_double), ("obj", ct.c_double), ("L", ct.c_double)]


class maid_refine_info(ct.Structure):
    _fields_ = [("newton_steps", ct.c_int32), ("cg_iters", ct.c_int32), ("status", ct.c_int32),
                ("rel_step", ct.c_double), ("grad_norm", ct.c_double)]


class maid_hparams(ct.Structure):
    _fields_ = [("rho_lo", ct.c_double), ("rho_hi", ct.c_double), ("nu_lo", ct.c_double),
                ("nu_hi", ct.c_double), ("lambda_", ct.c_double), ("mu", ct.c_double),
                ("L_g", ct.c_double), ("eps_min", ct.c_double), ("max_bt", ct.c_int32),
                ("max_lower_iter", ct.c_int32), ("max_cg_iter", ct.c_int32)]


class maid1d_desc(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("batch", ct.c_int32), ("alpha1", ct.c_double), ("alpha2", ct.c_double)]


class maid1d_sched(ct.Structure):
    _fields_ = [("eps", ct.c_double), ("delta", ct.c_double), ("step", ct.c_double), ("k", ct.c_int32)]


class maid_state(ct.Structure):
    _fields_ = [("theta", ct.c_void_p), ("x", ct.c_void_p), ("q", ct.c_void_p),
                ("eps", ct.c_double), ("delta", ct.c_double), ("step", ct.c_double),
                ("L", ct.c_double), ("k", ct.c_int32)]


class maid_step_info(ct.Structure):
    _fields_ = [("accepted", ct.c_int32), ("trials", ct.c_int32), ("retries", ct.c_int32),
                ("lower_iters", ct.c_int32), ("cg_iters", ct.c_int32), ("status", ct.c_int32),
                ("psi", ct.c_double), ("ell_k", ct.c_double), ("ell_next", ct.c_double),
                ("znorm", ct.c_double), ("lower_status", ct.c_int32), ("cg_status", ct.c_int32)]


_lib = None


class MaidError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib():
    """Load libmaid.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_09758_amd.build`")
    L = ct.CDLL(LIB_PATH)
    P = ct.c_void_p
    d = ct.c_double
    dp = ct.POINTER(ct.c_double)
    i32 = ct.c_int32
    L.maid_create.argtypes = [ct.POINTER(maid_desc), ct.POINTER(P)]
    L.maid_create.restype = ct.c_int
    L.maid_destroy.argtypes = [P]
    L.maid_destroy.restype = None
    L.maid_last_error.argtypes = [P]
    L.maid_last_error.restype = ct.c_char_p
    L.maid_config_string.argtypes = [P]
    L.maid_config_string.restype = ct.c_char_p
    L.maid_set_tile_rows.argtypes = [P, i32]
    L.maid_set_tile_rows.restype = ct.c_int
    L.maid_set_team.argtypes = [P, i32]
    L.maid_set_team.restype = ct.c_int
    L.maid_set_one_pass_cg.argtypes = [P, i32]
    L.maid_set_one_pass_cg.restype = ct.c_int
    L.maid_set_mfma.argtypes = [P, i32]
    L.maid_set_mfma.restype = ct.c_int
    L.maid_set_one_pass.argtypes = [P, i32]
    L.maid_set_one_pass.restype = ct.c_int
    L.maid_one_pass_forms.argtypes = [P, ct.POINTER(i32)]
    L.maid_one_pass_forms.restype = ct.c_int
    L.maid_lower_solve.argtypes = [P, P, P, P, d, i32, dp, ct.POINTER(maid_solve_info), ct.POINTER(i32), P]
    L.maid_lower_solve.restype = ct.c_int
    L.maid_lower_solve_refined.argtypes = [P, P, P, P, d, i32, d, i32, i32, dp, ct.POINTER(maid_solve_info),
                                           ct.POINTER(maid_refine_info), P]
    L.maid_lower_solve_refined.restype = ct.c_int
    L.maid_upper_value_grad.argtypes = [P, P, P, P, P, dp, dp, P]
    L.maid_upper_value_grad.restype = ct.c_int
    L.maid_upper_value_grad_noalloc.argtypes = [ct.POINTER(maid_desc), P, P, P, P, dp, dp,
                                                ct.POINTER(ct.c_char_p), P]
    L.maid_upper_value_grad_noalloc.restype = ct.c_int
    L.maid_adjoint_solve.argtypes = [P, P, P, P, P, d, i32, ct.POINTER(maid_solve_info), P]
    L.maid_adjoint_solve.restype = ct.c_int
    L.maid_hypergrad.argtypes = [P, P, P, P, P, P, i32, P, dp, P]
    L.maid_hypergrad.restype = ct.c_int
    L.maid_apply_operator.argtypes = [P, P, P, P, i32, P]
    L.maid_apply_operator.restype = ct.c_int
    L.maid_sobolev_value.argtypes = [P, P, P, dp, P]
    L.maid_sobolev_value.restype = ct.c_int
    L.maid_step.argtypes = [P, P, P, ct.POINTER(maid_state), ct.POINTER(maid_hparams),
                            ct.POINTER(maid_step_info), P]
    L.maid_step.restype = ct.c_int
    L.maid_profile.argtypes = [P, i32]
    L.maid_profile.restype = ct.c_int
    L.maid_profile_read.argtypes = [P, i32, ct.POINTER(ct.c_int64), ct.POINTER(ct.c_int64), dp]
    L.maid_profile_read.restype = ct.c_int
    L.maid_profile_name.argtypes = [i32]
    L.maid_profile_name.restype = ct.c_char_p
    PP = ct.POINTER(P)
    L.maid_create_batch.argtypes = [ct.POINTER(maid_desc), i32, ct.POINTER(P)]
    L.maid_create_batch.restype = ct.c_int
    L.maid_batch_size.argtypes = [P]
    L.maid_batch_size.restype = i32
    L.maid_batch_lower_solve.argtypes = [P, PP, PP, PP, dp, i32, dp, ct.POINTER(maid_solve_info), P]
    L.maid_batch_lower_solve.restype = ct.c_int
    L.maid_batch_adjoint_solve.argtypes = [P, PP, PP, PP, PP, dp, i32, ct.POINTER(maid_solve_info), P]
    L.maid_batch_adjoint_solve.restype = ct.c_int
    L.maid_batch_step.argtypes = [P, PP, PP, ct.POINTER(maid_state), ct.POINTER(maid_hparams),
                                  ct.POINTER(maid_step_info), P]
    L.maid_batch_step.restype = ct.c_int
    L.maid_batch_steps.argtypes = [P, PP, PP, ct.POINTER(maid_state), ct.POINTER(maid_hparams),
                                   ct.POINTER(maid_step_info), i32, P]
    L.maid_batch_steps.restype = ct.c_int
    L.maid_batch_create.argtypes = [ct.POINTER(maid_desc), i32, ct.POINTER(P)]
    L.maid_batch_create.restype = ct.c_int
    L.maid_gd_solve.argtypes = [P, P, P, P, d, i32, d, P, ct.POINTER(maid_solve_info), P]
    L.maid_gd_solve.restype = ct.c_int
    L.maid_hessian_apply.argtypes = [P, P, P, P, P, P]
    L.maid_hessian_apply.restype = ct.c_int
    L.maid_ift_step.argtypes = [P, P, P, ct.POINTER(maid_state), i32, d, d, i32, ct.POINTER(maid_step_info), P]
    L.maid_ift_step.restype = ct.c_int
    L.maid_lista_step.argtypes = [P, P, P, ct.POINTER(maid_state), i32, d, ct.POINTER(maid_step_info), P]
    L.maid_lista_step.restype = ct.c_int
    SI = ct.POINTER(maid_solve_info)
    L.maid1d_create.argtypes = [ct.POINTER(maid1d_desc), ct.POINTER(P)]
    L.maid1d_create.restype = ct.c_int
    L.maid1d_destroy.argtypes = [P]
    L.maid1d_destroy.restype = None
    L.maid1d_last_error.argtypes = [P]
    L.maid1d_last_error.restype = ct.c_char_p
    L.maid1d_lower_solve.argtypes = [P, P, P, P, d, dp, i32, SI, P]
    L.maid1d_lower_solve.restype = ct.c_int
    L.maid1d_upper_value_grad.argtypes = [P, P, P, P, P, dp, dp, P]
    L.maid1d_upper_value_grad.restype = ct.c_int
    L.maid1d_adjoint_solve.argtypes = [P, P, P, P, P, dp, i32, SI, P]
    L.maid1d_adjoint_solve.restype = ct.c_int
    L.maid1d_hypergrad.argtypes = [P, P, P, P, P, P, dp, P]
    L.maid1d_hypergrad.restype = ct.c_int
    L.maid1d_step.argtypes = [P, P, P, P, P, P, ct.POINTER(maid1d_sched), ct.POINTER(maid_hparams), d,
                              ct.POINTER(maid_step_info), P]
    L.maid1d_step.restype = ct.c_int
    L.maid_batch_upper_value_grad.argtypes = [P, PP, PP, PP, PP, dp, dp, P]
    L.maid_batch_upper_value_grad.restype = ct.c_int
    L.maid_batch_hypergrad.argtypes = [P, PP, PP, PP, PP, PP, i32, PP, dp, P]
    L.maid_batch_hypergrad.restype = ct.c_int
    L.maid_set_step_trace.argtypes = [P, i32, ct.POINTER(i32), i32, dp, i32]
    L.maid_set_step_trace.restype = ct.c_int
    L.maid_step_trace_length.argtypes = [P, ct.POINTER(i32), ct.POINTER(i32)]
    L.maid_step_trace_length.restype = ct.c_int
    L.maid_autotune.argtypes = [P, PP, PP, i32, ct.POINTER(i32), P]
    L.maid_autotune.restype = ct.c_int
    _lib = L
    return L


def create(desc: maid_desc) -> int:
    h = ct.c_void_p()
    rc = lib().maid_create(ct.byref(desc), ct.byref(h))
    if rc != OK:
        raise MaidError(rc, lib().maid_last_error(None).decode())
    return h.value


def create_batch(descs) -> int:
    arr = (maid_desc * len(descs))(*descs)
    h = ct.c_void_p()
    rc = lib().maid_create_batch(arr, len(descs), ct.byref(h))
    if rc != OK:
        raise MaidError(rc, lib().maid_last_error(None).decode())
    return h.value


def last_error(handle) -> str:
    return lib().maid_last_error(handle).decode()
