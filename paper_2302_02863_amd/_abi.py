"""ctypes declarations of the C ABI in include/fpde.h (argument marshalling only).

Loading fails loudly if libfpde.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfpde.so")

FPDE_OK, FPDE_EINVAL, FPDE_EDOMAIN, FPDE_ENOMEM, FPDE_EDEVICE, FPDE_ENOCONV, FPDE_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "FPDE_OK", -1: "FPDE_EINVAL", -2: "FPDE_EDOMAIN", -3: "FPDE_ENOMEM", -4: "FPDE_EDEVICE",
                -5: "FPDE_ENOCONV", -6: "FPDE_ESTATE"}
PREC_FP64, PREC_MIXED = 0, 1
F64, F32 = 0, 1
FLAG_PLAN_ONLY = 0x1
FLAG_JACOBI = 0x2
PART_B, PART_M, PART_KNEAR, PART_KFAR, PART_ALL, PART_FP64 = 0x1, 0x2, 0x4, 0x8, 0xF, 0x10

EXPORT = dict(CSR_ROWPTR=1, CSR_COLS=2, CSR_B=3, CSR_M=4, K_PERM=5, K_LEAFPTR=6, K_FAR=7, K_NEAR=8,
              RHO_PERM=9, RHO_FAR=10, RHO_NEAR=11, RHO=12, PAIRS=13, K_BOXES=14, RHO_BOXES=15)
EXPORT_IS_FLOAT = {"CSR_B", "CSR_M", "RHO", "K_BOXES", "RHO_BOXES"}


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_nodes", C.c_int64), ("n_dofs", C.c_int64),
                ("coords", C.POINTER(C.c_double)), ("n_cells", C.c_int64),
                ("cells", C.POINTER(C.c_int32)), ("cell_interior", C.POINTER(C.c_uint8)),
                ("exterior_radius", C.c_double)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("leaf_size", C.c_int32), ("leaf_size_rho", C.c_int32),
                ("cheb_p", C.c_int32), ("eta", C.c_double), ("nq_sing", C.c_int32), ("nq_reg", C.c_int32),
                ("s_bar", C.c_double), ("s_exterior", C.c_double), ("kappa_exterior", C.c_double),
                ("n_theta", C.c_int32), ("a_scale", C.c_double), ("flags", C.c_uint64),
                ("max_device_bytes", C.c_uint64), ("recompress_tol", C.c_double)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_int64) for n in (
        "n_dofs", "n_nodes", "n_cells", "n_fields", "n_pairs_identical", "n_pairs_edge", "n_pairs_vertex",
        "csr_nnz", "k_clusters", "k_levels", "k_leaves", "k_far", "k_near", "k_rank", "k_leaf_cap",
        "rho_points", "rho_clusters", "rho_levels", "rho_far", "rho_near", "device_bytes")] + \
        [(n, C.c_double) for n in ("t_plan_ms", "t_singular_ms", "t_near_blocks_ms", "t_bases_ms", "t_rho_ms",
                                    "t_mass_ms", "t_total_ms")] + \
        [(n, C.c_int64) for n in ("apply_bytes_near", "apply_bytes_csr", "apply_bytes_bases",
                                  "k_rank_rc", "k_rank_rc_min")] + \
        [(n, C.c_double) for n in ("k_rank_rc_mean", "t_recompress_ms")]


class Profile(C.Structure):
    _fields_ = [("n_applies", C.c_int64), ("ms_gather", C.c_double), ("ms_far", C.c_double),
                ("ms_out", C.c_double), ("ms_far_out", C.c_double), ("ms_total", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("rel_residual", C.c_double), ("converged", C.c_int32),
                ("refinements", C.c_int32), ("cond_estimate", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_02863_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.fpde_opts_default.argtypes = [C.POINTER(Opts)]
        L.fpde_gauss_legendre.argtypes = [C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.fpde_build.argtypes = [C.POINTER(Mesh), C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                 C.POINTER(Opts), C.POINTER(vp)]
        L.fpde_apply.argtypes = [vp, C.c_int32, vp, vp, C.c_int64, vp]
        L.fpde_apply_parts.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, C.c_int64, vp]
        L.fpde_apply_noalloc.argtypes = [vp, C.c_int32, vp, vp, C.c_int64, vp]
        L.fpde_load_vector.argtypes = [vp, vp, vp, vp]
        L.fpde_solve.argtypes = [vp, vp, vp, C.c_int64, C.c_double, C.c_int32, C.POINTER(SolveInfo), vp]
        L.fpde_apply_adjoint.argtypes = [vp, C.c_double, vp, vp, C.c_int64, vp, vp, vp]
        L.fpde_stats.argtypes = [vp, C.POINTER(Stats)]
        L.fpde_export.argtypes = [vp, C.c_int32, C.c_int32, vp, C.POINTER(C.c_int64)]
        L.fpde_profile.argtypes = [vp, C.c_int32, C.POINTER(Profile)]
        L.fpde_destroy.argtypes = [vp]
        L.fpde_destroy.restype = None
        L.fpde_last_error.restype = C.c_char_p
        for n in ("fpde_opts_default", "fpde_gauss_legendre", "fpde_build", "fpde_apply", "fpde_apply_parts",
                  "fpde_apply_noalloc",
                  "fpde_load_vector", "fpde_solve", "fpde_apply_adjoint", "fpde_stats", "fpde_export",
                  "fpde_profile"):
            getattr(L, n).restype = C.c_int32
        _lib = L
    return _lib


class FpdeError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().fpde_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")


def check(status: int, where: str):
    if status != FPDE_OK:
        raise FpdeError(status, where)
