"""ctypes declarations of the C ABI in include/tn.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtn.so")

TN_OK = 0
STATUS = {
    -1: "TN_E_ARG", -2: "TN_E_RANGE", -3: "TN_E_ORDER", -4: "TN_E_NOMEM",
    -5: "TN_E_HIP", -6: "TN_E_UNSUPPORTED",
}
DIRECTED = 1
TIES_SEQUENTIAL = 2
FORWARD = 4
HLL = 8  # tn_plan_create: a plan for the HyperLogLog stream only
KERNELS = {1: "identity", 2: "rowor", 3: "out_sizes", 4: "in_sizes", 5: "batch",
           6: "hash", 7: "recombine", 8: "mlp_forward", 9: "mlp_backward", 10: "mlp_adam",
           11: "aux"}


class TNError(RuntimeError):
    """A negative tn_status; ``code`` is the status, the message is tn_last_error()."""

    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class PlanStats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_uint32),
        ("m", ctypes.c_int64),
        ("levels", ctypes.c_int64),
        ("pairs", ctypes.c_int64),
        ("gathers", ctypes.c_int64),
        ("gather_sources", ctypes.c_int64),
        ("compound_items", ctypes.c_int64),
        ("max_level_items", ctypes.c_int64),
        ("max_level_gathers", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64),
        ("host_seconds", ctypes.c_double),
        ("directed_pairs", ctypes.c_int64),
        ("ops", ctypes.c_int64),
        ("op_levels", ctypes.c_int64),
        ("scratch_rows", ctypes.c_int64),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StreamStats(ctypes.Structure):
    _fields_ = [
        ("chunks", ctypes.c_int64),
        ("chunks_run", ctypes.c_int64),
        ("events_run", ctypes.c_int64),
        ("levels_run", ctypes.c_int64),
        ("saturated", ctypes.c_int32),
        ("slice_words", ctypes.c_int32),
        ("seconds", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes)
_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_u32, _i32, _i64, _u64, _f32 = (ctypes.c_uint32, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_uint64, ctypes.c_float)
SIGNATURES = {
    "tn_last_error": (ctypes.c_char_p, []),
    "tn_create": (_i32, [ctypes.c_int, _P, _PP]),
    "tn_set_stream": (_i32, [_P, _P]),
    "tn_sync": (_i32, [_P]),
    "tn_profile_enable": (_i32, [_P, ctypes.c_int]),
    "tn_profile_take": (_i32, [_P, _P, _P, _i32]),
    "tn_destroy": (None, [_P]),
    "tn_plan_create": (_i32, [_P, _u32, _i64, _P, _P, _P, _u32, _PP]),
    "tn_plan_get_stats": (_i32, [_P, ctypes.POINTER(PlanStats)]),
    "tn_plan_destroy": (None, [_P]),
    "tn_schedule_build": (_i32, [_u32, _i64, _P, _P, _P, _u32, _PP]),
    "tn_schedule_arrays": (_i32, [_P, ctypes.POINTER(PlanStats), _PP, _PP, _PP, _PP, _PP, _PP]),
    "tn_schedule_destroy": (None, [_P]),
    "tn_schedule_fwd_arrays": (_i32, [_P, _u32, _P, _PP, _PP]),
    "tn_schedule_op_arrays": (_i32, [_P, _PP, _PP]),
    "tn_plan_execute": (_i32, [_P, _P, _P, _i64, _u32]),
    "tn_plan_execute_sizes": (_i32, [_P, _P, _P, _i64, _u32, _P, _P]),
    "tn_set_saturation": (_i32, [_P, ctypes.c_int]),
    "tn_hll_execute": (_i32, [_P, _P, _u32, _P, _P, _P]),
    "tn_hll_build": (_i32, [_P, _u32, _i64, _P, _P, _P, _u32, _u32, _P, _P, _P]),
    "tn_online_create": (_i32, [_P, _u32, _u32, _P, _i64, _PP]),
    "tn_online_insert": (_i32, [_P, _P, _i64, _P, _P, _P, _i64, ctypes.POINTER(StreamStats)]),
    "tn_online_destroy": (None, [_P]),
    "tn_plan_last_traffic": (_i32, [_P, _P]),
    "tn_build_component_matrix": (_i32, [_P, _u32, _i64, _P, _P, _P, _u32, _P, _i64]),
    "tn_build_component_matrix_streamed": (_i32, [_P, _u32, _i64, _P, _P, _P, _u32, _P, _i64,
                                                  _i64, ctypes.POINTER(StreamStats)]),
    "tn_component_sizes": (_i32, [_P, _u32, _P, _i64, _P, _P]),
    "tn_batch_create": (_i32, [_P, _i32, _P, _P, _P, _P, _P, _u32, _PP]),
    "tn_batch_execute": (_i32, [_P, _P, _P, _P]),
    "tn_batch_get_stats": (_i32, [_P, _P, _P, _P]),
    "tn_batch_get_shape": (_i32, [_P, _P]),
    "tn_batch_destroy": (None, [_P]),
    "tn_build_component_matrix_batched": (_i32, [_P, _i32, _P, _P, _P, _P, _P, _u32, _P, _P]),
    "tn_hash_build_proxies": (_i32, [_P, _u32, _i64, _P, _P, _P, _u32, _u32, _u32, _P, _i32,
                                     _P, _P, _P, _i64, _i64, ctypes.POINTER(StreamStats)]),
    "tn_hash_compress": (_i32, [_P, _u32, _i64, _P, _P, _P, _u32, _u32, _u32, _P, _i32, _P, _P,
                                _PP]),
    "tn_recombine": (_i32, [_P, _u32, _u32, _u32, _P, _i64, _P, _P, _P, _P]),
    "tn_mlp_param_count": (_i32, []),
    "tn_recommended_ld": (_i64, [_u32]),
    "tn_mlp_init": (_i32, [_P, _u64, _P]),
    "tn_mlp_features": (_i32, [_P, _u32, _u32, _P, _P]),
    "tn_mlp_forward": (_i32, [_P, _P, _P, _i64, _P]),
    "tn_mlp_predict": (_i32, [_P, _P, _P, _i64, _u32, _P, _P]),
    "tn_mlp_train_step": (_i32, [_P, _P, _P, _P, _i64, _P, _P, _P, _i64, _f32, _P, _P]),
    "tn_mlp_train_step_noalloc": (_i32, [_P, _P, _P, _P, _i64, _P, _P, _P, _i64, _f32, _P, _P]),
}


def load():
    # torch's HIP runtime must be the one in the process before libtn.so is
    # loaded: libtn.so then binds to it (same soname) and shares its devices,
    # streams and allocations instead of pulling in a second runtime.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is not built: the HIP library is required (run "
            "__graft_entry__.build() or python paper_2307_04890_amd/_build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = load()


def check(status: int) -> None:
    if status != TN_OK:
        msg = lib.tn_last_error()
        raise TNError(status, msg.decode() if msg else "")
