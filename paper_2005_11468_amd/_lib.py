"""ctypes declarations of the C ABI in include/psr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsr.so")

PSR_OK, PSR_EINVAL, PSR_ENOMEM, PSR_EDEVICE, PSR_EUNSUPPORTED = 0, 1, 2, 3, 4
PSR_FP64, PSR_MIXED = 0, 1
PSR_PLAIN, PSR_PERSISTENT = 0, 1
STATUS_NAMES = {0: "CONVERGED", 1: "MAXITER", 2: "TS_FAILED", 3: "NONFINITE", 4: "SINGULAR"}

dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p


class SootDesc(C.Structure):
    _fields_ = [("precursor", C.c_int32), ("growth", C.c_int32), ("carbon", C.c_int32),
                ("A_nuc", C.c_double), ("beta_nuc", C.c_double), ("E_nuc", C.c_double),
                ("A_grow", C.c_double), ("beta_grow", C.c_double), ("E_grow", C.c_double),
                ("site_density", C.c_double), ("soot_density", C.c_double),
                ("coag_scale", C.c_double)]


class MechDesc(C.Structure):
    _fields_ = [("n_elements", C.c_int32), ("n_species", C.c_int32), ("n_reactions", C.c_int32),
                ("elem_weight", dp), ("species_elems", ip), ("nasa7", dp),
                ("t_low", C.c_double), ("t_high", C.c_double),
                ("reac_idx", ip), ("reac_nu", ip), ("prod_idx", ip), ("prod_nu", ip),
                ("A", dp), ("beta", dp), ("Ea", dp), ("soot", C.POINTER(SootDesc))]


class Conditions(C.Structure):
    _fields_ = [("n_reactors", C.c_int64), ("energy", C.c_int32),
                ("P", vp), ("tau", vp), ("T_in", vp), ("Y_in", vp)]


class SolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("scheduler", C.c_int32),
                ("rtol", C.c_double), ("atol_Y", C.c_double), ("atol_T", C.c_double),
                ("ftol", C.c_double), ("lambda_min", C.c_double),
                ("T_min", C.c_double), ("T_max", C.c_double),
                ("ts_rtol", C.c_double), ("ts_atol_Y", C.c_double), ("ts_atol_T", C.c_double),
                ("ts_neg_tol", C.c_double), ("h0", C.c_double), ("h_max", C.c_double),
                ("h_min", C.c_double), ("nw_h_ratio", C.c_double),
                ("nw_max_it", C.c_int32), ("nw_every", C.c_int32), ("max_lin", C.c_int32),
                ("max_refine", C.c_int32), ("engine", C.c_int32),
                ("use_graph", C.c_int32), ("refine_tol", C.c_double),
                ("atol_lnM", C.c_double), ("ts_atol_lnM", C.c_double),
                ("rpw", C.c_int32), ("grid_per_cu", C.c_int32),
                ("lnM_step", C.c_double), ("ct_ratio", C.c_double),
                ("ct_tau_min", C.c_double), ("ct_min_step", C.c_double),
                ("order", C.c_int32), ("mixed_max_n", C.c_int32)]


class Group(C.Structure):
    _fields_ = [("mech", vp), ("cond", Conditions), ("x_inout", vp), ("status", vp), ("n_lin", vp)]


class SolveStats(C.Structure):
    _fields_ = [("reactors", C.c_int64), ("converged", C.c_int64), ("lin_total", C.c_int64),
                ("lin_max", C.c_int64), ("jac_total", C.c_int64), ("fp64_fallbacks", C.c_int64),
                ("rounds", C.c_int32), ("kernel_ms", C.c_double)]


class TuneResult(C.Structure):
    _fields_ = [("engine", C.c_int32), ("rpw", C.c_int32), ("grid_per_cu", C.c_int32),
                ("candidates", C.c_int32), ("ms", C.c_double), ("solves_per_s", C.c_double),
                ("default_ms", C.c_double)]


SYMBOLS = {
    "psr_create_mechanism": ([C.POINTER(MechDesc), C.POINTER(vp)], C.c_int),
    "psr_destroy_mechanism": ([vp], C.c_int),
    "psr_num_unknowns": ([vp, C.c_int32], C.c_int32),
    "psr_residual": ([vp, C.POINTER(Conditions), vp, vp, vp, vp], C.c_int),
    "psr_jacobian": ([vp, C.POINTER(Conditions), vp, vp, vp], C.c_int),
    "psr_jacobian_fd": ([vp, C.POINTER(Conditions), vp, vp, vp, vp], C.c_int),
    "psr_jacobian_fd_noalloc": ([vp, C.POINTER(Conditions), vp, vp, vp], C.c_int),
    "psr_soot_outputs": ([vp, C.c_int64, vp, vp, vp], C.c_int),
    "psr_lu_factor_batch": ([C.c_int32, C.c_int64, C.c_int32, vp, vp, vp, vp], C.c_int),
    "psr_lu_solve_batch": ([C.c_int32, C.c_int64, vp, vp, vp, vp], C.c_int),
    "psr_default_opts": ([C.POINTER(SolveOpts)], None),
    "psr_workspace_bytes": ([C.POINTER(Group), C.c_int32, C.POINTER(SolveOpts)], C.c_size_t),
    "psr_solve_batch": ([C.POINTER(Group), C.c_int32, C.POINTER(SolveOpts), vp, C.c_size_t,
                         C.POINTER(SolveStats), vp], C.c_int),
    "psr_autotune": ([C.POINTER(Group), C.c_int32, C.POINTER(SolveOpts), C.c_int64, C.c_char_p,
                      C.POINTER(TuneResult), vp], C.c_int),
    "psr_sweep_batch": ([C.POINTER(Group), C.c_int32, C.c_int32, vp, C.POINTER(SolveOpts), vp,
                         C.c_size_t, vp, vp, C.POINTER(SolveStats), vp], C.c_int),
    "psr_last_error": ([], C.c_char_p),
}

_lib = None


def load() -> C.CDLL:
    """Load libpsr.so; raise if it is missing (there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2005_11468_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (args, res) in SYMBOLS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


class PSRError(RuntimeError):
    pass


def check(status: int, what: str):
    if status != PSR_OK:
        msg = load().psr_last_error().decode()
        raise PSRError(f"{what}: status {status}: {msg}")
