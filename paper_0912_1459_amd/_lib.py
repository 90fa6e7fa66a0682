"""ctypes declarations of libcdsigma.so (the C ABI in include/cdsigma.h).

Loading fails loudly when the library has not been built: there is no CPU
fallback for any step of the path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdsigma.so")

CDS_OK, CDS_EINVAL, CDS_ENOMEM, CDS_EDEVICE, CDS_ENOTPSD, CDS_ECAP, CDS_ESTATE = 0, -1, -2, -3, -4, -5, -6
PREC_FP64, PREC_FP32, PREC_BF16X3 = 0, 1, 2
CD_CONVERGED, CD_CAP, CD_FULLRANK, CD_NOTPSD = 0, 1, 2, -4
QP_CONVERGED, QP_MAX_ITER, QP_NONFINITE = 0, 1, 2
QP_RECOMPUTE, QP_RESIDUES = 0, 1

ERROR_NAMES = {CDS_EINVAL: "EINVAL", CDS_ENOMEM: "ENOMEM", CDS_EDEVICE: "EDEVICE",
               CDS_ENOTPSD: "ENOTPSD", CDS_ECAP: "ECAP", CDS_ESTATE: "ESTATE"}

# every symbol the header declares (checked by the CPU test-suite)
EXPORTS = [
    "cds_create", "cds_destroy", "cds_last_error", "cds_get_stats", "cds_reset_stats",
    "cds_set_kernel_timing", "cds_set_cd_lookahead", "cds_set_cd_large_path", "cds_set_cd_speculate", "cds_set_cd_mailbox", "cds_set_transform_fp64", "cds_set_target_chunk", "cds_version", "cds_eri_columns", "cds_cholesky_sgauss", "cds_cholesky_sgauss_subset",
    "cds_cholesky_dense", "cds_transform", "cds_cholesky_transform_sgauss", "cds_restride_blocks", "cds_sigma2", "cds_sigma2_noalloc", "cds_qp_solve", "cds_qp_adjoint",
    "cds_transform_adjoint", "cds_mp2", "cds_workspace_bytes", "cds_sigma2_matrix", "cds_dyson_solve",
]


class Stats(ctypes.Structure):
    _fields_ = [
        ("t_cd_ms", ctypes.c_double), ("t_cd_kernel_ms", ctypes.c_double),
        ("t_transform_ms", ctypes.c_double), ("t_contract_ms", ctypes.c_double),
        ("t_epilogue_ms", ctypes.c_double), ("t_newton_ms", ctypes.c_double),
        ("t_adjoint_ms", ctypes.c_double), ("bytes_cd", ctypes.c_double),
        ("flops_contract", ctypes.c_double), ("n_cd_steps", ctypes.c_int64),
        ("n_contract", ctypes.c_int64), ("n_newton_iter", ctypes.c_int64),
        ("t_cd_pass_ms", ctypes.c_double), ("bytes_cd_pass", ctypes.c_double),
        ("n_cd_pass", ctypes.c_int64), ("n_cd_miss", ctypes.c_int64),
        ("flops_cd_pass", ctypes.c_double), ("bytes_cd_step", ctypes.c_double),
        ("n_cd_step_launch", ctypes.c_int64), ("n_cd_pass_launch", ctypes.c_int64),
        ("t_mp2_ms", ctypes.c_double), ("flops_mp2", ctypes.c_double), ("t_dyson_ms", ctypes.c_double),
        ("t_cd_spec_ms", ctypes.c_double), ("n_cd_spec", ctypes.c_int64), ("n_cd_spec_block", ctypes.c_int64),
        ("n_cd_state_read", ctypes.c_int64), ("flops_cd_pass_method", ctypes.c_double),
        ("flops_cd_block_method", ctypes.c_double),
    ]


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_0912_1459_amd.build` "
                           "(the HIP library is required; there is no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    ip = ctypes.c_int
    sig = {
        "cds_create": (ip, [ip, P, ctypes.POINTER(P)]),
        "cds_destroy": (None, [P]),
        "cds_last_error": (ctypes.c_char_p, [P]),
        "cds_get_stats": (ip, [P, ctypes.POINTER(Stats)]),
        "cds_reset_stats": (ip, [P]),
        "cds_set_kernel_timing": (ip, [P, i32]),
        "cds_set_cd_lookahead": (ip, [P, i32]),
        "cds_set_cd_large_path": (ip, [P, i32]),
        "cds_set_cd_speculate": (ip, [P, i32]),
        "cds_set_cd_mailbox": (ip, [P, i32]),
        "cds_set_transform_fp64": (ip, [P, i32]),
        "cds_set_target_chunk": (ip, [P, i32]),
        "cds_version": (ctypes.c_char_p, []),
        "cds_eri_columns": (ip, [P, i32, P, P, i64, P, P]),
        "cds_cholesky_sgauss": (ip, [P, i32, P, P, d, d, d, i64, P, i64, P, P, i64, P, P, P]),
        "cds_cholesky_dense": (ip, [P, i64, P, i64, d, d, d, i64, P, i64, P, P, i64, P, P, P]),
        "cds_cholesky_sgauss_subset": (ip, [P, i32, P, P, P, d, d, d, i64, P, i64, P, P, i64, P, P, P]),
        "cds_transform": (ip, [P, i32, i32, i64, P, i64, P, i32, i32, i32, P, i64, P, P]),
        "cds_cholesky_transform_sgauss": (ip, [P, i32, P, P, d, d, d, i64, P, i64, P, P, i32, P, i32, i32, i32, P,
                                               i64, P, P, P, P, P]),
        "cds_restride_blocks": (ip, [P, i32, i64, i64, i64, P]),
        "cds_sigma2": (ip, [P, i32, i64, i64, i32, i32, i32, P, P, P, P, i32, P, P, P]),
        "cds_sigma2_noalloc": (ip, [P, i32, i64, i64, i32, i32, i32, P, P, P, P, i32, P, P, P]),
        "cds_qp_solve": (ip, [P, i32, i64, i64, i32, i32, i32, P, P, P, P, P, d, i32, i32, P, P, P, P]),
        "cds_qp_adjoint": (ip, [P, i32, i64, i64, i32, i32, i32, P, P, P, P, P, P, P, P, P]),
        "cds_transform_adjoint": (ip, [P, i32, i32, i64, P, i64, P, i32, i32, i32, P, i64, P, P, P]),
        "cds_mp2": (ip, [P, i32, i64, i64, i32, i32, P, P, P]),
        "cds_sigma2_matrix": (ip, [P, i32, i64, i64, i32, i32, i32, P, P, P, P, i32, P, P, P]),
        "cds_dyson_solve": (ip, [P, i32, i64, i64, i32, i32, i32, P, P, P, P, d, i32, P, P, P, P, P]),
        "cds_workspace_bytes": (ip, [P, ctypes.POINTER(ctypes.c_size_t)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L
