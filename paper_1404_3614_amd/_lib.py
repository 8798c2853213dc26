"""ctypes declarations of libhom (include/hom.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhom.so")

HOM_OK = 0
HOM_NOT_CONVERGED = 1
HOM_E_INVALID = -1
HOM_E_UNSUPPORTED_SIZE = -2
HOM_E_NOT_SPD = -3
HOM_E_DEVICE = -4
HOM_E_WORKSPACE = -5
HOM_FP64 = 0
HOM_MIXED = 1


class Desc(C.Structure):
    _fields_ = [("d", C.c_int32), ("N", C.c_int32 * 3), ("Y", C.c_double * 3),
                ("precision", C.c_int32), ("ncoef", C.c_int32), ("M", C.c_int32 * 3)]


class Info(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32),
                ("rel_res_recur", C.c_double), ("rel_res_true", C.c_double), ("energy", C.c_double)]


class UNetDesc(C.Structure):
    _fields_ = [("d", C.c_int32), ("levels", C.c_int32), ("base", C.c_int32), ("cin", C.c_int32),
                ("cout", C.c_int32), ("size", C.c_int32 * 3), ("batch", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("row_pairs", C.c_int32), ("row_threads", C.c_int32), ("apply_points", C.c_int32),
                ("apply_half_exchange", C.c_int32), ("apply_all_packs", C.c_int32), ("candidates", C.c_int32),
                ("row_ms", C.c_double),
                ("apply_ms", C.c_double)]


class Result(C.Structure):
    _fields_ = [("A_up", C.c_double * 9), ("B_up", C.c_double * 9), ("A_low", C.c_double * 9),
                ("A_mean", C.c_double * 9), ("D", C.c_double * 9)]


EXPORTS = {
    "hom_status_str": (C.c_char_p, [C.c_int32]),
    "hom_group_create": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    "hom_group_solve_pair": (C.c_int32, [C.c_void_p, C.c_double, C.c_int32, C.POINTER(C.c_void_p),
                                         C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p]),
    "hom_group_solve_bounds": (C.c_int32, [C.c_void_p, C.c_double, C.c_int32, C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p, C.POINTER(Result)]),
    "hom_group_destroy": (None, [C.c_void_p]),
    "hom_group_set_launch": (C.c_int32, [C.c_void_p, C.c_int32]),
    "hom_batch_field_to_grid": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p,
                                            C.c_size_t]),
    "hom_batch_grid_to_field": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t,
                                            C.POINTER(C.c_void_p)]),
    "hom_batch_net_input": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32]),
    "hom_tune_cache_load": (C.c_int32, [C.c_char_p, C.c_char_p, C.POINTER(C.c_int32)]),
    "hom_tune_cache_save": (C.c_int32, [C.c_char_p, C.c_char_p]),
    "hom_tune_cache_clear": (C.c_int32, []),
    "hom_field_len": (C.c_int32, [C.POINTER(Desc), C.c_int32, C.POINTER(C.c_size_t)]),
    "hom_workspace_bytes": (C.c_int32, [C.POINTER(Desc), C.c_int32, C.POINTER(C.c_size_t)]),
    "hom_setup": (C.c_int32, [C.POINTER(Desc), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                              C.c_void_p, C.POINTER(C.c_void_p)]),
    "hom_update_coefficients": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "hom_solve_primal": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_void_p),
                                     C.c_double, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(Info)]),
    "hom_solve_dual": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_void_p),
                                   C.c_double, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(Info)]),
    "hom_bounds": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(Result)]),
    "hom_apply": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "hom_probe_copy": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32, C.c_void_p,
                                   C.POINTER(C.c_double)]),
    "hom_dual_start": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "hom_coef_scratch_bytes": (C.c_int32, [C.POINTER(Desc), C.c_int32, C.c_void_p, C.POINTER(C.c_size_t)]),
    "hom_coef_inclusions": (C.c_int32, [C.POINTER(Desc), C.POINTER(C.c_double), C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                        C.POINTER(C.c_double), C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                        C.c_void_p]),
    "hom_coef_inclusions_static": (C.c_int32, [C.POINTER(Desc), C.POINTER(C.c_double), C.c_int32,
                                               C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                               C.POINTER(C.c_double), C.c_int32, C.c_void_p, C.c_void_p]),
    "hom_coef_pixels": (C.c_int32, [C.POINTER(Desc), C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32,
                                    C.POINTER(C.c_double), C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                    C.c_void_p]),
    "hom_phase_eig_range": (C.c_int32, [C.c_int32, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "hom_profile_passes": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "hom_destroy": (None, [C.c_void_p]),
    "hom_field_to_grid": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_void_p), C.c_void_p]),
    "hom_grid_to_field": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_void_p)]),
    "hom_net_input": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "hom_net_weights": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "hom_unet_sizes": (C.c_int32, [C.c_void_p, C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "hom_unet_create": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "hom_unet_forward": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "hom_unet_forward_samples": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p]),
    "hom_unet_loss_samples": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_int32,
                                          C.POINTER(C.c_double)]),
    "hom_unet_loss": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "hom_unet_loss_weighted": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double)]),
    "hom_unet_backward": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "hom_unet_adam": (C.c_int32, [C.c_void_p, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32]),
    "hom_unet_destroy": (None, [C.c_void_p]),
    "hom_batch_workspace_bytes": (C.c_int32, [C.c_int32, C.POINTER(C.c_size_t)]),
    "hom_batch_create": (C.c_int32, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p, C.c_size_t,
                                     C.POINTER(C.c_void_p)]),
    "hom_batch_solve": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_double),
                                    C.POINTER(C.c_void_p), C.c_double, C.c_int32, C.POINTER(C.c_void_p),
                                    C.POINTER(Info)]),
    "hom_batch_bounds": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                     C.POINTER(Result)]),
    "hom_batch_profile_passes": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                             C.POINTER(C.c_double)]),
    "hom_batch_set_timing": (C.c_int32, [C.c_void_p, C.c_int32]),
    "hom_batch_get_timing": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "hom_set_tuning": (C.c_int32, [C.c_int32]),
    "hom_problem_set_stop": (C.c_int32, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double]),
    "hom_sample_inclusions": (C.c_int32, [C.POINTER(Desc), C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                          C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "hom_sample_pixels": (C.c_int32, [C.POINTER(Desc), C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32,
                                      C.POINTER(C.c_double), C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                      C.c_void_p]),
    "hom_gani_workspace_bytes": (C.c_int32, [C.POINTER(Desc), C.c_void_p, C.POINTER(C.c_size_t)]),
    "hom_smooth_pixels": (C.c_int32, [C.POINTER(C.c_int32), C.c_void_p, C.c_void_p, C.c_int32,
                                      C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p]),
    "hom_set_gani": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t]),
    "hom_clear_gani": (C.c_int32, [C.c_void_p]),
    "hom_gani_matrices": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                      C.POINTER(C.c_double)]),
    "hom_batch_set_stop": (C.c_int32, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double]),
    "hom_batch_solve_pair": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_void_p),
                                         C.POINTER(C.c_void_p), C.c_double, C.c_int32, C.POINTER(C.c_void_p),
                                         C.POINTER(C.c_void_p), C.POINTER(Info), C.POINTER(Info)]),
    "hom_batch_solve_bounds": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.c_double,
                                           C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                           C.POINTER(Info), C.POINTER(Info), C.POINTER(Result)]),
    "hom_batch_update_coefficients": (C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]),
    "hom_problem_tuning": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Tuning)]),
    "hom_batch_tuning": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Tuning)]),
    "hom_problem_set_tiles": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Tuning)]),
    "hom_batch_set_tiles": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(Tuning)]),
    "hom_batch_destroy": (None, [C.c_void_p]),
}

_lib = None


def load():
    """Load libhom.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libhom.so not built at {LIB_PATH}: run python -m paper_1404_3614_amd.build")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in EXPORTS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class HomError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        name = load().hom_status_str(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {name} ({status})")


def check(status, where, allow_not_converged=False):
    if status == HOM_OK or (allow_not_converged and status == HOM_NOT_CONVERGED):
        return status
    raise HomError(status, where)
