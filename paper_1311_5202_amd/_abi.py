"""ctypes declarations of the C ABI in include/fdbem.h (argument marshalling only)."""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdbem.so")

FDA_OK = 0
FDA_EINVAL = -1
FDA_ENOMEM = -2
FDA_EHIP = -3
FDA_NOT_CONVERGED = -4
FDA_NONFINITE = -5
FDA_EBREAKDOWN = -6
FDA_ENOTSUP = -7

OPS = {"RAW_H": 0, "RAW_G": 1, "RAW_T1": 2, "BM_H": 3, "BM_G": 4}
FDA_OP_FP32 = 0x100
PREC = {"fp64": 0, "fp32": 1, "both": 2}

EXPORTS = ("fda_default_opts", "bem_nystrom_nodes", "bem_near_correction", "fda_build", "fda_matvec", "bm_solve", "fda_rhs_plane_wave",
           "fda_stats", "fda_set_timing", "fda_phase_times", "fda_destroy", "fda_last_error", "fda_net_num_params",
           "fda_net_create", "fda_net_destroy", "fda_net_get_params", "fda_net_set_params", "fda_net_loss_grad",
           "fda_net_train_step", "fda_net_attach", "fda_net_loss_grad_raw", "fda_set_graph", "fda_batch_create",
           "fda_batch_matvec", "fda_batch_solve", "fda_batch_destroy", "fda_rhs_neumann", "fda_matvec_noalloc", "fda_analyze", "fda_net_weight_blocks")


class FdaGeometry(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("pts", ctypes.c_void_p), ("nrm", ctypes.c_void_p),
                ("w", ctypes.c_void_p), ("n_elem", ctypes.c_int64), ("elem", ctypes.c_void_p)]


class FdaOpts(ctypes.Structure):
    _fields_ = [("svd_eps", ctypes.c_double), ("lowrank_eps", ctypes.c_double), ("leaf_cap", ctypes.c_int),
                ("leaf_rule", ctypes.c_int), ("c_d", ctypes.c_double), ("far_field", ctypes.c_int),
                ("lf_grid", ctypes.c_int), ("precision", ctypes.c_int), ("corrections", ctypes.c_int),
                ("verbose", ctypes.c_int), ("wedge_factor", ctypes.c_int), ("m2l_tile", ctypes.c_int),
                ("p2p_threshold", ctypes.c_double),
                ("coupling", ctypes.c_double),
                ("autotune", ctypes.c_int),
                ("slab_mb", ctypes.c_int),
                ("hf_template", ctypes.c_int),
                ("original", ctypes.c_int),
                ("serial_slabs", ctypes.c_int),
                ("chunk_kernel", ctypes.c_int)]


class FdaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fdbem error {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load libfdbem.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1311_5202_amd.build_ext.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dbl, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_int
    L.fda_default_opts.argtypes = [ctypes.POINTER(FdaOpts)]
    L.bem_nystrom_nodes.argtypes = [i64, vp, vp, vp, vp]
    L.bem_near_correction.argtypes = [i64, vp, vp, vp, vp, dbl, ci, dbl, ctypes.POINTER(i64), vp, vp, vp]
    L.fda_build.argtypes = [ctypes.POINTER(FdaGeometry), dbl, dbl, ctypes.POINTER(FdaOpts), ctypes.POINTER(vp)]
    L.fda_matvec.argtypes = [vp, ci, vp, vp, vp]
    L.bm_solve.argtypes = [vp, ci, vp, dbl, ci, ci, ci, vp, ctypes.POINTER(ci), ctypes.POINTER(dbl), vp, vp]
    L.fda_rhs_plane_wave.argtypes = [vp, ctypes.POINTER(dbl), vp, vp]
    L.fda_stats.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
    L.fda_set_timing.argtypes = [vp, ci]
    L.fda_phase_times.argtypes = [vp, ctypes.POINTER(dbl), ci]
    L.fda_net_num_params.argtypes = []
    L.fda_net_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(vp)]
    L.fda_net_destroy.argtypes = [vp]
    L.fda_net_destroy.restype = None
    L.fda_net_get_params.argtypes = [vp, vp]
    L.fda_net_set_params.argtypes = [vp, vp]
    L.fda_net_loss_grad.argtypes = [vp, vp, ctypes.POINTER(dbl), vp]
    L.fda_net_train_step.argtypes = [vp, vp, dbl, ctypes.POINTER(dbl)]
    L.fda_net_attach.argtypes = [vp, vp]
    L.fda_net_loss_grad_raw.argtypes = [vp, ci, vp, vp, vp, vp, vp, i64, vp, vp, vp, vp, ctypes.POINTER(dbl), vp]
    L.fda_net_weight_blocks.argtypes = [vp, vp, ci]
    L.fda_set_graph.argtypes = [vp, ci]
    L.fda_batch_create.argtypes = [vp, ci, ctypes.POINTER(vp)]
    L.fda_batch_matvec.argtypes = [vp, ci, vp, vp, vp]
    L.fda_batch_solve.argtypes = [vp, ci, vp, dbl, ci, ci, ci, vp, vp, vp, vp]
    L.fda_batch_destroy.argtypes = [vp]
    L.fda_batch_destroy.restype = None
    L.fda_rhs_neumann.argtypes = [vp, vp, vp, vp]
    L.fda_matvec_noalloc.argtypes = [vp, ci, vp, vp, vp]
    L.fda_analyze.argtypes = [ctypes.POINTER(FdaGeometry), dbl, dbl, ctypes.POINTER(FdaOpts), ctypes.c_char_p,
                              ctypes.c_size_t]
    L.fda_destroy.argtypes = [vp]
    L.fda_destroy.restype = None
    L.fda_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("fda_destroy", "fda_last_error", "fda_net_destroy", "fda_batch_destroy"):
            getattr(L, name).restype = ci
    _lib = L
    return L


def check(code: int) -> int:
    if code != FDA_OK:
        raise FdaError(code, lib().fda_last_error().decode())
    return code
