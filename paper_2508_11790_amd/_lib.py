"""ctypes loader of libwbmvdr.so and the C ABI signatures (include/wbmvdr.h).

There is no fallback: if the library is missing or cannot be loaded, every call raises.
"""

from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwbmvdr.so")

WBM_HALF_BIN = 1
FORM_PLAIN, FORM_FUSED, FORM_GRAPH, FORM_MIXED, FORM_MIXED_BF16 = 0, 1, 2, 3, 4
FORM_FUSED_F32, FORM_GRAPH_F32 = 5, 6
PREC_EXT, PREC_F32, PREC_MIXED, PREC_MIXED_BF16 = 0, 1, 2, 3
INFO_ROUTED = 1 << 30
INFO_WIDTH = 1 << 29
PAIR_MFMA, PAIR_RESIDENT, PAIR_WAVE, PAIR_BLOCK = 1, 2, 64, 256
STATUS = {0: "ok", 1: "invalid argument", 2: "shape mismatch", 3: "out of memory",
          4: "HIP runtime error", 5: "unsupported"}


class WbmConfig(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("m_fft", C.c_int32), ("k_sub", C.c_int32),
                ("l_train", C.c_int32), ("l_test", C.c_int32), ("max_targets", C.c_int32),
                ("w_max", C.c_int32), ("flags", C.c_int32), ("beta", C.c_double),
                ("d_over_lambda", C.c_double)]


class WbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


EXPORTS = ("wbm_plan_create", "wbm_plan_destroy", "wbm_plan_workspace_bytes",
           "wbm_plan_set_tuning", "wbm_plan_get_tuning", "wbm_beamform",
           "wbm_channelize", "wbm_beamspace", "wbm_steer", "wbm_full_mvdr", "wbm_stage_times",
           "wbm_profiles", "wbm_beamform_pairs", "wbm_beamform_learned", "wbm_sinr",
           "wbm_mlp_create", "wbm_mlp_destroy", "wbm_mlp_forward", "wbm_mlp_grad", "wbm_mlp_adam",
           "wbm_mlp_grad_static", "wbm_sweep_labels", "wbm_lift", "wbm_apply_lifted", "wbm_synthesize",
           "wbm_beam_pattern", "wbm_range_doppler", "wbm_beamform_upa", "wbm_beamspace_upa",
           "wbm_steer_upa", "wbm_lift_upa", "wbm_beam_pattern_upa", "wbm_status_str", "wbm_last_error", "wbm_version")
MLP_PARAMS = 25090
MLP_STATIC_MAX_BATCH = 4096
PROFILE_BINS = 64

_lib = None


def load() -> C.CDLL:
    """Load the library once; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2508_11790_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    lib.wbm_plan_create.argtypes = [C.POINTER(WbmConfig), C.POINTER(P)]
    lib.wbm_plan_destroy.argtypes = [P]
    lib.wbm_plan_workspace_bytes.argtypes = [P]
    lib.wbm_plan_workspace_bytes.restype = I64
    lib.wbm_plan_set_tuning.argtypes = [P, I32, I32, I32, I32, I32]
    lib.wbm_plan_get_tuning.argtypes = [P, I32, P, P, P, P]
    lib.wbm_beamform.argtypes = [P, P, P, P, I32, D, I32, P, P, P, P, P]
    lib.wbm_channelize.argtypes = [P, P, P, P]
    lib.wbm_beamspace.argtypes = [P, P, P, P]
    lib.wbm_steer.argtypes = [P, P, P, I32, P, P, P]
    lib.wbm_full_mvdr.argtypes = [P, P, P, I32, D, I32, I32, P, P, P, P]
    lib.wbm_stage_times.argtypes = [P, P, P, P, I32, D, I32, I32, P, P]
    lib.wbm_profiles.argtypes = [P, P, P, I32, D, P, P]
    lib.wbm_beamform_pairs.argtypes = [P, P, P, P, I32, P, P, P, P, P, P, P]
    lib.wbm_beamform_learned.argtypes = [P, P, P, I32, P, D, I32, D, P, P, P, P, P, P, P, P]
    lib.wbm_sinr.argtypes = [P, P, P, I32, P, P, P, P, P, I32, D, P, P]
    lib.wbm_mlp_create.argtypes = [I32, C.POINTER(P)]
    lib.wbm_mlp_destroy.argtypes = [P]
    lib.wbm_mlp_forward.argtypes = [P, P, P, I32, P, P]
    lib.wbm_mlp_grad.argtypes = [P, P, P, P, I32, P, P, P]
    lib.wbm_mlp_adam.argtypes = [P, P, P, P, P, I32, D, P]
    lib.wbm_mlp_grad_static.argtypes = [P, P, P, I32, P, P, P]
    lib.wbm_sweep_labels.argtypes = [P, P, I32, P, I32, P, I32, D, P, P]
    lib.wbm_lift.argtypes = [P, P, P, I32, P, P]
    lib.wbm_apply_lifted.argtypes = [P, P, P, I32, P, P]
    lib.wbm_synthesize.argtypes = [P, P, I32, P, P]
    lib.wbm_beam_pattern.argtypes = [P, P, I32, P, I32, P, P]
    lib.wbm_range_doppler.argtypes = [P, P, I32, C.c_int64, P, I32, I32, I32, I32, I32, D, P, P,
                                      P, P]
    lib.wbm_beamform_upa.argtypes = [P, P, I32, I32, P, P, P, P, I32, D, I32, P, P, P, P, P]
    lib.wbm_beamspace_upa.argtypes = [P, P, I32, I32, P, P]
    lib.wbm_steer_upa.argtypes = [P, I32, I32, P, P, P, P, I32, P, P, P]
    lib.wbm_lift_upa.argtypes = [P, P, P, I32, I32, P, I32, P, P]
    lib.wbm_beam_pattern_upa.argtypes = [P, P, I32, I32, P, I32, P, P]
    lib.wbm_status_str.argtypes = [I32]
    lib.wbm_status_str.restype = C.c_char_p
    lib.wbm_last_error.argtypes = []
    lib.wbm_last_error.restype = C.c_char_p
    lib.wbm_version.restype = C.c_char_p
    for name in ("wbm_plan_create", "wbm_plan_destroy", "wbm_beamform", "wbm_channelize",
                 "wbm_beamspace", "wbm_steer", "wbm_full_mvdr", "wbm_stage_times", "wbm_profiles",
                 "wbm_beamform_pairs", "wbm_beamform_learned", "wbm_sinr", "wbm_mlp_create",
                 "wbm_mlp_destroy", "wbm_mlp_forward", "wbm_mlp_grad", "wbm_mlp_adam",
                 "wbm_mlp_grad_static", "wbm_sweep_labels", "wbm_lift", "wbm_apply_lifted", "wbm_synthesize",
                 "wbm_beam_pattern", "wbm_range_doppler", "wbm_beamform_upa",
                 "wbm_beamspace_upa", "wbm_steer_upa", "wbm_lift_upa",
                 "wbm_beam_pattern_upa"):
        getattr(lib, name).restype = I32
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != 0:
        msg = load().wbm_last_error().decode(errors="replace")
        raise WbmError(status, msg)
