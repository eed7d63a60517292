"""ctypes binding of ``libccmi.so`` (the C ABI declared in ``include/cc.h``).

Argument marshalling only: every step of the residual path runs in the
library's HIP kernels.  PyTorch supplies device memory and the stream.
Loading fails loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import pathlib

_HERE = pathlib.Path(__file__).resolve().parent
LIB_PATH = _HERE / "libccmi.so"

CC_OK, CC_EINVAL, CC_ENOMEM, CC_EDEVICE, CC_ENOTCONV, CC_EDIVERGED, CC_EUNSUPPORTED, CC_EINTERNAL = \
    0, -1, -2, -3, -4, -5, -6, -7
CC_CCD, CC_CCSD = 0, 1
CC_R64, CC_C128 = 0, 1
CC_PREC_F64, CC_PREC_F32, CC_PREC_BF16X3 = 0, 1, 2
CC_GUESS_GIVEN, CC_GUESS_MP2, CC_GUESS_MLP = 0, 1, 2

# Every symbol declared in include/cc.h.
EXPORTS = (
    "cc_create", "cc_destroy", "cc_last_error", "cc_status_string",
    "cc_plan_create", "cc_plan_destroy", "cc_plan_workspace_bytes", "cc_plan_residual",
    "cc_plan_step", "cc_plan_scalars", "cc_residual", "cc_energy", "cc_iterate", "cc_gemm",
    "cc_permute", "cc_plan_describe", "cc_plan_describe_dry", "cc_plan_flops", "cc_plan_profile",
    "cc_plan_profile_table", "cc_plan_autotune", "cc_plan_set_precision", "cc_plan_set_correction", "cc_gemm_tile_count", "cc_gemm_tile_count_c128", "cc_gemm_noalloc", "cc_plan_create_ops", "cc_plan_describe_ops_dry", "cc_plan_set_triples", "cc_plan_create2", "cc_batch_create",
    "cc_batch_destroy", "cc_batch_step", "cc_batch_scalars", "cc_batch_autotune", "cc_batch_iterate",
    "cc_batch_profile", "cc_batch_profile_table", "cc_batch_flops", "cc_mlp_num_params",
    "cc_mlp_num_samples", "cc_mlp_features", "cc_mlp_targets", "cc_mlp_moments", "cc_mlp_forward",
    "cc_mlp_loss_grad", "cc_mlp_train", "cc_guess_mlp", "cc_mlp_standardise",
)


class CCSystemStruct(C.Structure):
    _fields_ = [("o", C.c_int32), ("v", C.c_int32), ("scalar", C.c_int32)] + [
        (n, C.c_void_p) for n in ("f_oo", "f_ov", "f_vv", "oooo", "ooov", "oovv", "ovvo", "ovvv", "vvvv")
    ]


class CCAmps(C.Structure):
    _fields_ = [("t1", C.c_void_p), ("t2", C.c_void_p)]


class CCIterOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("prec", C.c_int32),
                ("level_shift", C.c_double), ("refine_tol", C.c_double), ("use_graph", C.c_int32),
                ("check_every", C.c_int32), ("diverge_window", C.c_int32), ("dressed", C.c_int32),
                ("autotune", C.c_int32), ("correction", C.c_int32), ("packed", C.c_int32),
                ("guess", C.c_int32), ("mlp_prec", C.c_int32), ("mlp_params", C.c_void_p),
                ("mlp_stats", C.c_void_p)]


class CCIterReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("rnorm", C.c_double),
                ("e_re", C.c_double), ("e_im", C.c_double), ("seconds", C.c_double),
                ("setup_seconds", C.c_double), ("lowp_iters", C.c_int32), ("corr_iters", C.c_int32),
                ("hist_rnorm", C.POINTER(C.c_double)),
                ("hist_e", C.POINTER(C.c_double)), ("hist_cap", C.c_int32), ("guess_used", C.c_int32),
                ("guess_rnorm_mlp", C.c_double), ("guess_rnorm_mp2", C.c_double), ("guess_seconds", C.c_double)]


class CCMlpStats(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("sx", "mD", "sD", "me", "se", "st")]


class CCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


_lib = None


def load() -> C.CDLL:
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
    lib = C.CDLL(str(LIB_PATH))
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "cc_create": (C.c_int, [P(vp), C.c_int, vp]),
        "cc_destroy": (C.c_int, [vp]),
        "cc_last_error": (C.c_char_p, [vp]),
        "cc_status_string": (C.c_char_p, [C.c_int]),
        "cc_plan_create": (C.c_int, [vp, P(CCSystemStruct), C.c_int, C.c_int, P(vp)]),
        "cc_plan_destroy": (C.c_int, [vp]),
        "cc_plan_workspace_bytes": (C.c_size_t, [vp]),
        "cc_plan_residual": (C.c_int, [vp, P(CCAmps), P(CCAmps), P(dbl)]),
        "cc_plan_step": (C.c_int, [vp, P(CCAmps), dbl, C.c_int]),
        "cc_plan_scalars": (C.c_int, [vp, P(dbl), P(dbl), P(dbl)]),
        "cc_residual": (C.c_int, [vp, P(CCSystemStruct), C.c_int, C.c_int, P(CCAmps), P(CCAmps), P(dbl)]),
        "cc_energy": (C.c_int, [vp, P(CCSystemStruct), C.c_int, P(CCAmps), P(dbl), P(dbl)]),
        "cc_iterate": (C.c_int, [vp, P(CCSystemStruct), C.c_int, P(CCIterOpts), P(CCAmps), P(CCIterReport)]),
        "cc_gemm": (C.c_int, [vp, C.c_int, C.c_int, i64, i64, i64, dbl, vp, i64, i64, vp, i64, i64, dbl, vp, i64]),
        "cc_permute": (C.c_int, [vp, C.c_int, C.c_int, P(i64), P(i32), dbl, vp, dbl, vp]),
        "cc_plan_describe": (C.c_char_p, [vp]),
        "cc_plan_describe_dry": (C.c_char_p, [C.c_int, C.c_int, C.c_int, C.c_int]),
        "cc_plan_flops": (dbl, [vp, C.c_int]),
        "cc_plan_profile": (C.c_int, [vp, C.c_int]),
        "cc_plan_autotune": (C.c_int, [vp, P(CCAmps), C.c_int]),
        "cc_plan_set_precision": (C.c_int, [vp, C.c_int]),
        "cc_plan_set_correction": (C.c_int, [vp, C.c_int, C.c_int]),
        "cc_gemm_tile_count": (C.c_int, [C.c_int]),
        "cc_gemm_tile_count_c128": (C.c_int, []),
        "cc_gemm_noalloc": (C.c_int, [vp, C.c_int, i64, i64, i64, dbl, vp, i64, i64, vp, i64, i64, dbl, vp, i64]),
        "cc_plan_create_ops": (C.c_int, [vp, P(CCSystemStruct), C.c_int, C.c_int, C.c_char_p, P(vp)]),
        "cc_plan_describe_ops_dry": (C.c_char_p, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_char_p]),
        "cc_plan_set_triples": (C.c_int, [vp, vp, vp]),
        "cc_plan_create2": (C.c_int, [vp, P(CCSystemStruct), C.c_int, C.c_int, C.c_int, P(vp)]),
        "cc_batch_create": (C.c_int, [vp, C.c_int, P(CCSystemStruct), C.c_int, C.c_int, P(CCAmps), P(vp)]),
        "cc_batch_destroy": (C.c_int, [vp]),
        "cc_batch_step": (C.c_int, [vp, dbl, C.c_int]),
        "cc_batch_scalars": (C.c_int, [vp, P(dbl), P(dbl), P(dbl)]),
        "cc_batch_autotune": (C.c_int, [vp, C.c_int]),
        "cc_batch_iterate": (C.c_int, [vp, P(CCIterOpts), P(CCIterReport), P(i32)]),
        "cc_batch_profile": (C.c_int, [vp, C.c_int]),
        "cc_batch_profile_table": (C.c_char_p, [vp]),
        "cc_batch_flops": (dbl, [vp]),
        "cc_mlp_num_params": (i64, []),
        "cc_mlp_num_samples": (i64, [C.c_int, C.c_int]),
        "cc_mlp_features": (C.c_int, [vp, P(CCSystemStruct), P(CCMlpStats), vp]),
        "cc_mlp_targets": (C.c_int, [vp, C.c_int, C.c_int, vp, dbl, vp]),
        "cc_mlp_moments": (C.c_int, [vp, vp, vp, i64, P(dbl)]),
        "cc_mlp_forward": (C.c_int, [vp, C.c_int, vp, vp, i64, vp]),
        "cc_mlp_standardise": (C.c_int, [vp, vp, vp, i64, P(CCMlpStats), vp, vp]),
        "cc_mlp_loss_grad": (C.c_int, [vp, C.c_int, vp, vp, vp, i64, P(dbl), vp]),
        "cc_mlp_train": (C.c_int, [vp, C.c_int, vp, vp, vp, vp, vp, i64, vp, i64, i32, dbl, P(i64), P(dbl), i32]),
        "cc_guess_mlp": (C.c_int, [vp, P(CCSystemStruct), C.c_int, vp, P(CCMlpStats), P(CCAmps)]),
        "cc_plan_profile_table": (C.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().cc_status_string(status).decode()
