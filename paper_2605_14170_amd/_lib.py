"""ctypes declarations of libmbbp.so (the C ABI of include/mbbp.h).

Argument marshalling only.  Loading fails loudly if the HIP library has not
been built: there is no fallback implementation of any step.
"""

from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbbp.so")

MBBP_OK = 0
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOTINROWSPACE", -3: "ENOMEM", -4: "EDEVICE",
                -5: "EUNSUPPORTED", -6: "EABORTED"}
MBBP_FLAG_FIXED_T = 1
MBBP_FLAG_ONE_PER_WAVE = 2
NUM_COUNTERS = 8


class MbbpError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Sparse(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int32), ("cols", ctypes.c_int32),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p)]


class BasisList(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("basis_ptr", ctypes.c_void_p),
                ("rows", ctypes.c_void_p), ("extra", ctypes.POINTER(Sparse))]


class Bases(ctypes.Structure):
    _fields_ = [("hx", BasisList), ("hz", BasisList)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("lanes_per_instance", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("blocks", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("rule", ctypes.c_int32), ("alpha", ctypes.c_float), ("r_max", ctypes.c_float),
                ("select", ctypes.c_int32), ("max_batch", ctypes.c_int64), ("flags", ctypes.c_uint32)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libmbbp.so is not built ({LIB_PATH}); run __graft_entry__.build() "
                              "or python paper_2605_14170_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
        sig = {
            "mbbp_params_default": ([ctypes.POINTER(Params)], i32),
            "mbbp_create": ([ctypes.POINTER(Sparse), ctypes.POINTER(Sparse), ctypes.POINTER(Bases), i32, i32,
                             ctypes.POINTER(Params), ctypes.POINTER(P)], i32),
            "mbbp_destroy": ([P], None),
            "mbbp_decode": ([P, i64, P, P, P, P, i32, P, P, P, P, P, P, P], i32),
            "mbbp_decode_batched": ([P, i64, P, P, P, P, i32, P, P, P, P, P, P, P], i32),
            "mbbp_decode_detail": ([P, i32, i64, P, P, i32, P, P, P, P], i32),
            "mbbp_sample": ([P, u64, dbl, i64, i64, P, P, P, P, P], i32),
            "mbbp_failures": ([P, i64, P, P, P, P, P, P], i32),
            "mbbp_run": ([P, u64, dbl, i64, i64, P, P], i32),
            "mbbp_subtrees": ([ctypes.POINTER(Sparse), P, P, P, P], i32),
            "mbbp_build_bases": ([ctypes.POINTER(Sparse), i32, i32, i32, P, P, P, i32], i32),
            "mbbp_logicals": ([P, P, P, P], i32),
            "mbbp_edge_counts": ([P, i32, P], i32),
            "mbbp_last_error": ([], ctypes.c_char_p),
            "mbbp_set_timing": ([P, i32], i32),
            "mbbp_set_config": ([P, i32, ctypes.POINTER(LaunchConfig)], i32),
            "mbbp_get_config": ([P, i32, ctypes.POINTER(LaunchConfig)], i32),
            "mbbp_autotune": ([P, i32, u64, dbl, i64, ctypes.POINTER(LaunchConfig)], i32),
            "mbbp_set_graph": ([P, i32], i32),
            "mbbp_set_noise": ([P, i32], i32),
            "mbbp_bp_time": ([P, P, P, i32], i32),
            "mbbp_set_weights": ([P, P, P], i32),
            "mbbp_wbp_ckpt_floats": ([P, i32, i64, i32, P], i32),
            "mbbp_wbp_forward": ([P, i32, i64, P, P, i32, P, P, i32, P, P, P], i32),
            "mbbp_wbp_backward": ([P, i32, i64, P, P, i32, P, P, i32, P, P, P, P, P], i32),
            "mbbp_run_graph_config": ([P, i64, ctypes.POINTER(LaunchConfig)], i32),
            "mbbp_prior_llr": ([i32, dbl, ctypes.POINTER(ctypes.c_float)], i32),
            "mbbp_set_per_basis": ([P, i32], i32),
            "mbbp_run_static": ([P, u64, dbl, i64, i64, P, P], i32),
            "mbbp_set_serial_lanes": ([P, i32], i32),
            "mbbp_set_serial_kernel": ([P, i32], i32),
            "mbbp_set_stats": ([P, P], i32),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int, where: str) -> None:
    if status != MBBP_OK:
        msg = lib().mbbp_last_error()
        raise MbbpError(status, where, msg.decode() if msg else "")


EXPORTED = ["mbbp_params_default", "mbbp_create", "mbbp_destroy", "mbbp_decode", "mbbp_decode_batched",
            "mbbp_decode_detail", "mbbp_sample", "mbbp_failures", "mbbp_run", "mbbp_subtrees",
            "mbbp_build_bases", "mbbp_logicals", "mbbp_edge_counts", "mbbp_last_error", "mbbp_set_timing",
            "mbbp_bp_time", "mbbp_set_config", "mbbp_get_config", "mbbp_autotune", "mbbp_set_graph",
            "mbbp_set_weights", "mbbp_wbp_ckpt_floats", "mbbp_wbp_forward", "mbbp_wbp_backward",
            "mbbp_set_noise", "mbbp_run_graph_config", "mbbp_prior_llr", "mbbp_set_per_basis", "mbbp_run_static",
            "mbbp_set_serial_lanes", "mbbp_set_serial_kernel", "mbbp_set_stats"]
