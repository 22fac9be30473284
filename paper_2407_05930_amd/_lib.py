"""ctypes binding of libmsp.so (argument marshalling only).

The library must have been built (``python -m paper_2407_05930_amd.build``);
there is no fallback: importing this module raises if the shared object is
missing.  When torch is importable it is imported first so that the library
binds to the same HIP runtime instance as torch's tensors.
"""
from __future__ import annotations

import ctypes
import os

try:  # share one HIP runtime with torch (same soname, loaded once)
    import torch  # noqa: F401
except Exception:  # pragma: no cover - torch is part of the image
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmsp.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2407_05930_amd.build`")

lib = ctypes.CDLL(LIB_PATH)

MSP_OK = 0
MSP_NOT_CONVERGED = 1
STATUS = {
    0: "MSP_OK", 1: "MSP_NOT_CONVERGED", -1: "MSP_ERR_ARG", -2: "MSP_ERR_NOT_SYMMETRIC", -3: "MSP_ERR_BAD_MAP",
    -4: "MSP_ERR_BREAKDOWN", -5: "MSP_ERR_HIP", -6: "MSP_ERR_OOM", -7: "MSP_ERR_NOT_SPD",
    -8: "MSP_ERR_UNSUPPORTED",
}
PRECISION = {"fp64": 0, "mixed": 1, "mixed_bf16g": 2, "mixed_bf16": 3}
PC = {"amgr": 0, "fsai": 1, "none": 2, "amgr_sub": 3, "amgs": 4}


class msp_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rowptr", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32)), ("val", ctypes.POINTER(ctypes.c_double))]


class msp_symmap(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int32), ("n_b", ctypes.c_int64), ("img", ctypes.POINTER(ctypes.c_int64))]


class msp_copies(ctypes.Structure):
    _fields_ = [("copies", ctypes.c_int32), ("n_b", ctypes.c_int64), ("sub", ctypes.POINTER(ctypes.c_int64))]


class msp_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("pc", ctypes.c_int32), ("lrc_k", ctypes.c_int32),
                ("dist", ctypes.c_int32), ("theta", ctypes.c_double), ("jacobi0", ctypes.c_int32),
                ("jacobi", ctypes.c_int32), ("coarse_max", ctypes.c_int32), ("max_levels", ctypes.c_int32),
                ("max_ratio", ctypes.c_double), ("tol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("device", ctypes.c_int32), ("seed", ctypes.c_uint64), ("trunc0", ctypes.c_double),
                ("coarse64", ctypes.c_int32), ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32),
                ("amgs_light", ctypes.c_int32), ("schur_tau", ctypes.c_double), ("true_residual", ctypes.c_int32),
                ("afsai_nnz", ctypes.c_int32), ("emin_steps", ctypes.c_int32)]


class msp_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("relres_rec", ctypes.c_double * 64),
                ("nlev", ctypes.c_int32), ("rows", ctypes.c_int64 * 32), ("nnz", ctypes.c_int64 * 32),
                ("op_complexity", ctypes.c_double), ("c_rat", ctypes.c_double), ("avg_nnzr", ctypes.c_double),
                ("t_setup_s", ctypes.c_double), ("t_solve_s", ctypes.c_double),
                ("relres_true", ctypes.c_double * 64), ("t_vcycle_s", ctypes.c_double),
                ("split_drift", ctypes.c_int64), ("split_drift1", ctypes.c_int64)]


class msp_faces(ctypes.Structure):
    _fields_ = [("nf", ctypes.c_int64), ("cell_a", ctypes.POINTER(ctypes.c_int64)),
                ("cell_b", ctypes.POINTER(ctypes.c_int64)), ("kind", ctypes.POINTER(ctypes.c_int8)),
                ("axis", ctypes.POINTER(ctypes.c_int8)), ("area", ctypes.POINTER(ctypes.c_double)),
                ("dist_a", ctypes.POINTER(ctypes.c_double)), ("dist_b", ctypes.POINTER(ctypes.c_double))]


_P = ctypes.POINTER
_vp = ctypes.c_void_p
SIGNATURES = {
    "msp_default_opts": (ctypes.c_int, [_P(msp_opts)]),
    "msp_setup": (ctypes.c_int, [_P(msp_csr), _P(msp_symmap), _P(msp_opts), _P(_vp)]),
    "msp_setup_copies": (ctypes.c_int, [_P(msp_csr), _P(msp_copies), _P(msp_opts), _P(_vp)]),
    "msp_refresh": (ctypes.c_int, [_vp, _vp, _vp]),
    "msp_rebuild_below": (ctypes.c_int, [_vp, _vp, _vp, _P(_vp)]),
    "msp_export_amgs": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int64), _P(ctypes.c_int64),
                                       _P(ctypes.c_int64), _vp, _vp, _vp]),
    "msp_solve_device": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _P(msp_stats)]),
    "msp_solve": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _P(msp_stats)]),
    "msp_solve_device_noalloc": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _P(msp_stats)]),
    "msp_get_stats": (ctypes.c_int, [_vp, _P(msp_stats)]),
    "msp_num_levels": (ctypes.c_int, [_vp, _P(ctypes.c_int32)]),
    "msp_level_sizes": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int64), _P(ctypes.c_int64),
                                       _P(ctypes.c_int64), _P(ctypes.c_int64)]),
    "msp_export_level": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                        _P(ctypes.c_double)]),
    "msp_export_outer": (ctypes.c_int, [_vp, _vp, _vp]),
    "msp_export_sub_level": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp, _vp, _vp]),
    "msp_export_lrc": (ctypes.c_int, [_vp, _vp, _vp]),
    "msp_set_timing": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
    "msp_reset_timing": (ctypes.c_int, [_vp]),
    "msp_get_timing": (ctypes.c_int, [_vp, ctypes.c_int32, _P(ctypes.c_int64), _P(ctypes.c_double),
                                      _P(ctypes.c_double)]),
    "msp_get_timing_kernel": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32]),
    "msp_batch_setup": (ctypes.c_int, [ctypes.c_int32, _P(msp_csr), _P(msp_symmap), _P(msp_opts), _P(_vp)]),
    "msp_batch_solve": (ctypes.c_int, [_vp, _P(ctypes.c_int32), _P(_vp), _P(_vp), _vp, _P(msp_stats)]),
    "msp_batch_size": (ctypes.c_int, [_vp, _P(ctypes.c_int32)]),
    "msp_batch_set_chunk": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "msp_batch_last_launches": (ctypes.c_int, [_vp, _P(ctypes.c_int32)]),
    "msp_batch_free": (None, [_vp]),
    "msp_fv_create": (ctypes.c_int, [_P(msp_faces), _P(msp_symmap), ctypes.c_int32, _P(_vp)]),
    "msp_fv_nnz": (ctypes.c_int, [_vp, _P(ctypes.c_int64)]),
    "msp_fv_assemble": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "msp_fv_assemble_device": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "msp_fv_kappa_grad": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp]),
    "msp_fv_free": (None, [_vp]),
    "msp_free": (None, [_vp]),
    "msp_last_error": (ctypes.c_char_p, []),
}

for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


class MspError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def check(status: int) -> int:
    if status < 0:
        raise MspError(status, lib.msp_last_error().decode(errors="replace"))
    return status
