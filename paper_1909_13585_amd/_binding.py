"""ctypes binding of the C ABI in ``include/mlb.h`` (argument marshalling only).

Every function here forwards to the HIP library ``libmlb.so``; no step of the
analysis runs in Python.  Loading fails loudly if the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlb.so")

MLB_OK = 0
MLB_EINVAL = -1
MLB_ESTATE = -2
MLB_ENOMEM = -3
MLB_EDEVICE = -4
MLB_ENOTCONV = -5
MLB_ENOPOS = -6
MLB_EBREAKDOWN = -7
MLB_FP64 = 0
MLB_ELEM_CONFORMING = 0
MLB_ELEM_INCOMPATIBLE = 1
MLB_MIXED = 1
MLB_WARM_NONE = 0
MLB_WARM_COARSE = 1
MLB_WARM_STATIC = 2

STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ESTATE", -3: "ENOMEM", -4: "EDEVICE", -5: "ENOTCONV",
                -6: "ENOPOS", -7: "EBREAKDOWN"}


class MlbDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("nel", C.c_int * 3), ("E1", C.c_double), ("E0", C.c_double),
                ("nu", C.c_double), ("penal", C.c_double), ("mg_levels", C.c_int), ("eig_level", C.c_int),
                ("precision", C.c_int), ("device", C.c_int), ("element", C.c_int)]


class MlbOpts(C.Structure):
    _fields_ = [("smooth_steps", C.c_int), ("jacobi_omega", C.c_double), ("eig_guard", C.c_int),
                ("eig_max_it", C.c_int), ("check_every", C.c_int), ("seed", C.c_uint64), ("cycle", C.c_int),
                ("block_cg", C.c_int), ("eig_sweeps", C.c_int), ("graphs", C.c_int), ("pinvit_steps", C.c_int),
                ("refine_sweeps", C.c_int), ("coarse_sweeps", C.c_int), ("pinvit_shift", C.c_int),
                ("refine_fine", C.c_int)]


class MlbSolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("converged", C.c_int), ("rel_residual", C.c_double),
                ("true_rel_residual", C.c_double), ("seconds", C.c_double)]


class MlbEigInfo(C.Structure):
    _fields_ = [("coarse_iterations", C.c_int), ("coarse_residual", C.c_double), ("coarse_gap", C.c_double),
                ("fine_iterations", C.c_int), ("fine_true_residual", C.c_double), ("seconds_coarse", C.c_double),
                ("seconds_fine", C.c_double), ("seconds_ritz", C.c_double), ("coarse_warm_used", C.c_int),
                ("pinvit_steps", C.c_int), ("lambda1_before_pinvit", C.c_double), ("seconds_pinvit", C.c_double),
                ("refine_levels", C.c_int), ("refine_lambda1", C.c_double * 8), ("seconds_refine", C.c_double),
                ("coarse_guard_fired", C.c_int)]


class MlbTuneInfo(C.Structure):
    _fields_ = [("wht_zchunk", C.c_int), ("stencil_cols", C.c_int), ("wht_ms", C.c_float * 5),
                ("stencil_ms", C.c_float * 5), ("wht_variant", C.c_int), ("wht_lds_ms", C.c_float * 5),
                ("wht_nopf_ms", C.c_float * 5), ("wht64_zchunk", C.c_int), ("wht64_variant", C.c_int),
                ("wht64_ms", C.c_float * 5), ("wht64_lds_ms", C.c_float * 5), ("wht64_nopf_ms", C.c_float * 5),
                ("wht_v3_ms", C.c_float * 5), ("wht64_v3_ms", C.c_float * 5), ("wht_score_ms", C.c_float * 20),
                ("wht64_score_ms", C.c_float * 20)]


class MlbBatchDesc(C.Structure):
    _fields_ = [("ninst", C.c_int), ("nel", C.c_int * 128), ("E1", C.c_double), ("E0", C.c_double),
                ("nu", C.c_double), ("penal", C.c_double), ("precision", C.c_int), ("device", C.c_int),
                ("max_coarse_dofs", C.c_int)]


class MlbBatchOpts(C.Structure):
    _fields_ = [("smooth_steps", C.c_int), ("jacobi_omega", C.c_double), ("queue", C.c_int), ("graphs", C.c_int),
                ("check_every", C.c_int), ("refine_steps", C.c_int)]


class MlbBatchInfo(C.Structure):
    _fields_ = [("max_iterations", C.c_int), ("total_iterations", C.c_int), ("batch_iterations", C.c_int),
                ("converged", C.c_int), ("worst_true_rel_res", C.c_double), ("setup_s", C.c_double),
                ("solve_s", C.c_double), ("refine_steps", C.c_int), ("misses", C.c_int),
                ("worst_floor", C.c_double), ("worst_refined_rel_res", C.c_double)]



class MlbMmaOpts(C.Structure):
    _fields_ = [("xmin", C.c_double), ("xmax", C.c_double), ("move", C.c_double), ("asyinit", C.c_double),
                ("asyincr", C.c_double), ("asydecr", C.c_double), ("c", C.c_double), ("d", C.c_double)]


class MlbMmaInfo(C.Structure):
    _fields_ = [("dual_iterations", C.c_int), ("dual_evaluations", C.c_int), ("proj_grad", C.c_double),
                ("dual_value", C.c_double), ("lam", C.c_double * 32), ("y", C.c_double * 32),
                ("seconds", C.c_double)]

_P = C.c_void_p
_I = C.c_int
_D = C.c_double
_SIGS = {
    "mlb_create": (_I, [C.POINTER(MlbDesc), C.POINTER(_P)]),
    "mlb_destroy": (None, [_P]),
    "mlb_last_error": (C.c_char_p, [_P]),
    "mlb_set_opts": (_I, [_P, C.POINTER(MlbOpts)]),
    "mlb_level_size": (_I, [_P, _I, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "mlb_set_bc": (_I, [_P, _P]),
    "mlb_set_bc_dev": (_I, [_P, _P, _P]),
    "mlb_set_loads": (_I, [_P, _I, _P]),
    "mlb_set_loads_dev": (_I, [_P, _I, _P, _P]),
    "mlb_set_density": (_I, [_P, _P]),
    "mlb_set_density_dev": (_I, [_P, _P, _P]),
    "mlb_solve_static": (_I, [_P, _D, _I, _P, _P, C.POINTER(MlbSolveInfo)]),
    "mlb_solve_static_dev": (_I, [_P, _D, _I, _P, _P, C.POINTER(MlbSolveInfo), _P]),
    "mlb_buckling": (_I, [_P, _I, _I, _D, _P, _P, C.POINTER(MlbEigInfo)]),
    "mlb_buckling_dev": (_I, [_P, _I, _I, _D, _P, _P, C.POINTER(MlbEigInfo), _P]),
    "mlb_eig_residuals": (_I, [_P, _P]),
    "mlb_eig_residuals_dev": (_I, [_P, _P, _P]),
    "mlb_sensitivities": (_I, [_P, _P, _P, C.POINTER(MlbSolveInfo)]),
    "mlb_sensitivities_dev": (_I, [_P, _P, _P, C.POINTER(MlbSolveInfo), _P]),
    "mlb_sensitivities_consistent": (_I, [_P, _P, C.POINTER(MlbSolveInfo)]),
    "mlb_sensitivities_consistent_dev": (_I, [_P, _P, C.POINTER(MlbSolveInfo), _P]),
    "mlb_set_warm_start": (_I, [_P, _I, _I, _P]),
    "mlb_set_warm_start_dev": (_I, [_P, _I, _I, _P, _P]),
    "mlb_apply_K_dev": (_I, [_P, _I, _I, _P, _P, _P]),
    "mlb_apply_G_dev": (_I, [_P, _I, _I, _P, _P, _P]),
    "mlb_set_state_dev": (_I, [_P, _P, _P, _P]),
    "mlb_prolong_dev": (_I, [_P, _I, _I, _P, _P, _P]),
    "mlb_restrict_dev": (_I, [_P, _I, _I, _P, _P, _P]),
    "mlb_sweep_dev": (_I, [_P, _I, _I, _I, _P]),
    "mlb_vcycle_dev": (_I, [_P, _I, _I, _P, _P, _P]),
    "mlb_coarse_modes_dev": (_I, [_P, _I, _P, _P]),
    "mlb_adjoints_dev": (_I, [_P, _I, _P, _P]),
    "mlb_adjoint_rhs_dev": (_I, [_P, _I, _P, _P]),
    "mlb_set_tiles": (_I, [_P, _I, _I, _I]),
    "mlb_autotune": (_I, [_P, _I, C.POINTER(MlbTuneInfo), _P]),
    "mlb_set_omegas": (_I, [_P, _I, _P]),
    "mlb_get_omegas": (_I, [_P, _I, _P]),
    "mlb_solve_block_dev": (_I, [_P, _I, _P, _P, _D, _I, C.POINTER(MlbSolveInfo), _P]),
    "mlb_mac_dev": (_I, [_P, _I, _P, _I, _P, _P, _P, _P]),
    "mlb_sed_tv_dev": (_I, [_P, _I, _P, _D, _P, _P, _P, _P]),
    "mlb_dilate_dev": (_I, [_P, _I, _P, _D, _D, _P, _P, _P]),
    "mlb_dilate_noalloc_dev": (_I, [_P, _I, _P, _D, _D, _P, _P, _P]),
    "mlb_filter_project_dev": (_I, [_P, _P, _D, _D, _D, _P, _P, _P]),
    "mlb_filter_chain_dev": (_I, [_P, _I, _P, _D, _D, _D, _P, _P, _P, _P]),
    "mlb_set_penal": (_I, [_P, _D]),
    # optimisation layer (include/mlb_opt.h)
    "mlb_continuation": (_I, [_I, _D, _D, _I, _D, _D, _I, _D, C.POINTER(_D), C.POINTER(_D)]),
    "mlb_p1_functions_dev": (_I, [C.c_int64, _I, _P, _D, _P, _P, _P, C.c_int64, _D, _D, _D, _D, _P, _P, _P, _P]),
    "mlb_p2_functions_dev": (_I, [C.c_int64, _I, _P, _D, _P, _P, _P, C.c_int64, _D, _D, _D, _P, _P, _P, _P]),
    "mlb_mma_create": (_I, [C.c_int64, _I, C.POINTER(MlbMmaOpts), _I, C.POINTER(_P)]),
    "mlb_mma_destroy": (None, [_P]),
    "mlb_mma_last_error": (C.c_char_p, [_P]),
    "mlb_mma_update_dev": (_I, [_P, _P, _D, _P, _P, _P, C.c_int64, C.POINTER(MlbMmaInfo), _P]),
    # warm-start network kernels (include/mlb_nn.h)
    "mlb_nn_conv3d": (_I, [_I, _I, _I, _I, _I, _I, _I, _I, _P, _P, _P, _P, _I, _P]),
    "mlb_nn_conv3d_wgrad": (_I, [_I, _I, _I, _I, _I, _I, _I, _P, _P, _P, _P, _P]),
    "mlb_nn_conv3d_mfma": (_I, [_I, _I, _I, _I, _I, _I, _P, _P, _P, _P, _I, _P]),
    "mlb_nn_relu_mask": (_I, [C.c_int64, _P, _P, _P]),
    "mlb_nn_pool2": (_I, [C.c_int64, _I, _I, _I, C.c_float, _P, _P, _P]),
    "mlb_nn_axpy": (_I, [C.c_int64, C.c_float, _P, _P, _P]),
    "mlb_nn_unpool2": (_I, [C.c_int64, _I, _I, _I, C.c_float, _P, _P, _P]),
    "mlb_nn_concat": (_I, [_I, _I, _I, C.c_int64, _P, _P, _P, _P]),
    "mlb_nn_split": (_I, [_I, _I, _I, C.c_int64, _P, _P, _P, _P]),
    "mlb_nn_cell2node": (_I, [C.c_int64, _I, _I, _I, _P, _P, _P]),
    "mlb_nn_nodes_to_dofs": (_I, [_I, C.c_int64, _P, _P, _P]),
    "mlb_nn_node2cell_grad": (_I, [C.c_int64, _I, _I, _I, _P, _P, _P]),
    "mlb_nn_mse_work": (C.c_int64, [C.c_int64]),
    "mlb_nn_mse": (_I, [C.c_int64, _P, _P, _P, C.c_float, _P, _P, _P, _P]),
    "mlb_nn_adam": (_I, [C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, _I, _P, _P, _P, _P, _P, _P]),
    "mlb_nn_to_bf16": (_I, [C.c_int64, _P, _P, _P]),
    # batched independent 2D instances (include/mlb_batch.h)
    "mlb_batch_create": (_I, [C.POINTER(MlbBatchDesc), C.POINTER(_P)]),
    "mlb_batch_destroy": (None, [_P]),
    "mlb_batch_last_error": (C.c_char_p, [_P]),
    "mlb_batch_set_opts": (_I, [_P, C.POINTER(MlbBatchOpts)]),
    "mlb_batch_get_opts": (_I, [_P, C.POINTER(MlbBatchOpts)]),
    "mlb_batch_layout": (_I, [_P, _P, _P, _P]),
    "mlb_batch_set_problem_dev": (_I, [_P, _P, _P, _P, _P]),
    "mlb_batch_solve_dev": (_I, [_P, _D, _I, _P, _P, _P, C.POINTER(MlbBatchInfo), _P]),
    "mlb_batch_compliance_sens_dev": (_I, [_P, _P, _P]),
    "mlb_batch_residuals": (_I, [_P, _P, _P, _P]),
}

_lib = None


def load(path=LIB_PATH):
    """Loads libmlb.so and declares every signature; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run __graft_entry__.build()")
    # torch supplies device memory and streams, so the process must use ONE
    # HIP runtime: load torch (and its libamdhip64) before libmlb so that the
    # library's libamdhip64.so.7 dependency resolves to the same copy.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return sorted(_SIGS)


class MlbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
