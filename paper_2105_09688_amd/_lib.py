"""ctypes declarations of libssm's C ABI (include/ssm.h).  Argument
marshalling only: every step of the scheme runs in the library's kernels."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssm.so")
MAX_D = 4

SSM_OK, SSM_ERR_INVALID, SSM_ERR_NEWTON, SSM_ERR_NONFINITE = 0, -1, -2, -3
SSM_ERR_HIP, SSM_ERR_OOM, SSM_ERR_STATE = -4, -5, -6
SSM_FP64, SSM_FP32, SSM_FP32_KAHAN = 0, 1, 2

# every function the header declares (checked by the CPU test suite)
EXPORTS = (
    "ssm_init", "ssm_step", "ssm_run", "ssm_sync", "ssm_moments", "ssm_get_state",
    "ssm_set_state", "ssm_state_layout", "ssm_bind_state", "ssm_state_refresh", "ssm_rmse", "ssm_sqdiff", "ssm_info", "ssm_profile", "ssm_destroy", "ssm_last_error",
    "ssm_pair_sum", "ssm_pair_workspace_bytes", "ssm_implicit_solve", "ssm_brownian",
    "ssm_philox_blocks", "ssm_mlp_num_params", "ssm_surrogate_load", "ssm_surrogate_enable",
    "ssm_surrogate_recheck",
    "ssm_surrogate_samples", "ssm_surrogate_predict", "ssm_mlp_forward", "ssm_mlp_forward_noalloc", "ssm_mlp_loss_grad", "ssm_mlp_train", "ssm_surrogate_train",
)


class Config(C.Structure):
    _fields_ = [
        ("d", C.c_int32), ("n_sys", C.c_int32),
        ("N", C.POINTER(C.c_int64)), ("ens", C.POINTER(C.c_int32)), ("h", C.POINTER(C.c_double)),
        ("T", C.c_double), ("h_fine", C.c_double), ("seed", C.c_uint64), ("precision", C.c_int32),
        ("v_rho", C.c_double), ("v_a", C.c_double), ("v_kappa", C.c_double), ("v_lam", C.c_double),
        ("b_c0", C.c_double), ("b_lam", C.c_double), ("b_g", C.c_double), ("b_ell", C.c_double),
        ("s0", C.c_double * MAX_D), ("s1", C.c_double * MAX_D), ("s2", C.c_double * MAX_D),
        ("x0_mean", C.c_double * MAX_D), ("x0_std", C.c_double * MAX_D),
        ("newton_max_iter", C.c_int32), ("allow_unstable_h", C.c_int32),
        ("stream", C.c_void_p),
        ("targets_per_lane", C.c_int32), ("sources_per_item", C.c_int32), ("pair_scheme", C.c_int32),
        ("graphs", C.c_int32),
        ("v_componentwise", C.c_int32), ("kahan_span", C.c_int32),
        ("v_ak", C.c_double * MAX_D), ("b_const", C.c_double * MAX_D), ("b_mat", C.c_double * (MAX_D * MAX_D)),
        ("b_mean", C.c_double * MAX_D), ("jside_band_groups", C.c_int32), ("persistent", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("tick", C.c_int64), ("ticks_total", C.c_int64), ("newton_max_seen", C.c_int32),
        ("newton_failures", C.c_int32), ("nonfinite", C.c_int32), ("n_pair_items", C.c_int32),
        ("targets_per_lane", C.c_int32), ("sources_per_item", C.c_int32), ("symmetric", C.c_int32),
        ("jside_band_groups", C.c_int32), ("device_bytes", C.c_int64),
        ("pair_launches", C.c_int64), ("pair_ms", C.c_double),
        ("update_launches", C.c_int64), ("update_ms", C.c_double),
        ("surr_checks", C.c_int64), ("surr_ticks", C.c_int64), ("surr_fallback_ticks", C.c_int64),
        ("surr_last_err", C.c_double), ("surr_max_err", C.c_double),
        ("surr_last_raw_err", C.c_double), ("surr_gain", C.c_double * MAX_D),
        ("persistent", C.c_int32), ("persistent_tiles", C.c_int32),
        ("persistent_launches", C.c_int64), ("persistent_ticks", C.c_int64),
        ("surr_rechecks", C.c_int64),
    ]


class TrainCfg(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
        ("beta2", C.c_float), ("eps", C.c_float), ("seed", C.c_uint64),
    ]


class SurrTrainCfg(C.Structure):
    _fields_ = [
        ("n_ens", C.c_int32), ("ens0", C.c_int32), ("N", C.c_int64), ("n_samples", C.c_int64),
        ("snapshots", C.c_int32), ("pad", C.c_int32), ("seed", C.c_uint64), ("train", TrainCfg),
    ]


_lib = None


def load():
    """Load libssm.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libssm.so is not built ({LIB_PATH}); run __graft_entry__.build() "
                          "or python paper_2105_09688_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, dp, i32, i64, u64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64, C.c_uint64
    st = C.c_int
    sig = {
        "ssm_init": (st, [C.POINTER(Config), C.POINTER(vp)]),
        "ssm_step": (st, [vp, i64]),
        "ssm_run": (st, [vp]),
        "ssm_sync": (st, [vp]),
        "ssm_moments": (st, [vp, i32, dp, dp]),
        "ssm_get_state": (st, [vp, i32, i32, dp, C.POINTER(C.c_int64)]),
        "ssm_set_state": (st, [vp, i32, dp, C.c_int64]),
        "ssm_state_layout": (st, [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
        "ssm_bind_state": (st, [vp, vp, C.c_size_t]),
        "ssm_state_refresh": (st, [vp, i32]),
        "ssm_rmse": (st, [vp, vp, dp, dp]),
        "ssm_sqdiff": (st, [vp, i32, vp, i32, dp]),
        "ssm_info": (st, [vp, C.POINTER(Info)]),
        "ssm_profile": (st, [vp, i32]),
        "ssm_destroy": (None, [vp]),
        "ssm_last_error": (C.c_char_p, []),
        "ssm_pair_sum": (st, [i32, i64, i32, vp, C.c_double, vp, vp, C.c_size_t, vp]),
        "ssm_pair_workspace_bytes": (C.c_size_t, [i32, i64, i32]),
        "ssm_implicit_solve": (st, [i32, i64, vp, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_double, dp, C.c_double, i32, vp, vp, vp]),
        "ssm_brownian": (st, [i32, i64, u64, i32, i64, i32, C.c_double, vp, vp]),
        "ssm_philox_blocks": (st, [u64, u64, u64, u64, u64, u64, i64, vp, vp]),
        "ssm_mlp_num_params": (i64, [i32]),
        "ssm_surrogate_load": (st, [vp, vp, i64]),
        "ssm_surrogate_enable": (st, [vp, i32, C.c_double, i32]),
        "ssm_surrogate_recheck": (st, [vp, i32]),
        "ssm_surrogate_samples": (st, [vp, i32, i64, u64, vp, vp]),
        "ssm_surrogate_predict": (st, [vp, i32, dp, vp]),
        "ssm_mlp_forward": (st, [i32, vp, vp, i64, vp, vp]),
        "ssm_mlp_forward_noalloc": (st, [i32, vp, vp, i64, vp, vp]),
        "ssm_mlp_loss_grad": (st, [i32, vp, vp, vp, i64, vp, dp, vp]),
        "ssm_mlp_train": (st, [i32, vp, vp, i64, C.POINTER(TrainCfg), vp, vp, vp]),
        "ssm_surrogate_train": (st, [vp, C.POINTER(SurrTrainCfg), vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class SSMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"libssm status {status}: {msg}")
        self.status = status


def check(status: int) -> None:
    if status != SSM_OK:
        raise SSMError(status, load().ssm_last_error().decode(errors="replace"))
