"""ctypes declarations of the C ABI in include/xf.h (argument marshalling only).

torch is imported first so that the HIP runtime torch ships with is the one
the library binds to; device pointers and streams then interoperate.  There is
no fallback: if libxf.so is missing this module raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (binds the HIP runtime before libxf.so is loaded)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxf.so")

XF_OK, XF_EINVAL, XF_EUNSUPPORTED, XF_ENOMEM, XF_EDEVICE = range(5)
XF_EXACT, XF_RAW_ESTIMATE = 0, 1
XF_FP64, XF_MIXED = 0, 1

STATUS_NAMES = {0: "XF_OK", 1: "XF_EINVAL", 2: "XF_EUNSUPPORTED", 3: "XF_ENOMEM", 4: "XF_EDEVICE"}


class Bits128(ctypes.Structure):
    _fields_ = [("w", ctypes.c_uint64 * 2)]


class Work(ctypes.Structure):
    _fields_ = [("determinants", ctypes.c_int64), ("rank_sum", ctypes.c_int64), ("flops", ctypes.c_double),
                ("sample_ms", ctypes.c_double), ("eval_ms", ctypes.c_double), ("lemma", ctypes.c_int32),
                ("backward_lemma", ctypes.c_int32), ("general", ctypes.c_int32), ("backward_reused", ctypes.c_int32),
                ("fp32_bases", ctypes.c_int64), ("philox_blocks", ctypes.c_int64),
                ("tree_bitstrings", ctypes.c_int64)]


class Circuit(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_rot", ctypes.c_int32), ("rot", ctypes.c_void_p),
                ("k", ctypes.c_int32), ("pairs", ctypes.c_void_p), ("layer", ctypes.c_void_p),
                ("theta", ctypes.c_void_p)]


class Gate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("theta", ctypes.c_double), ("g", (ctypes.c_double * 2) * 16)]


XF_GATE_MATCHGATE, XF_GATE_CPHASE = 0, 1

EXPORTS = ["xf_plan_create", "xf_plan_set_params", "xf_plan_refreeze", "xf_plan_destroy",
           "xf_extent", "xf_trajectory_bound", "xf_probabilities", "xf_probabilities_noalloc", "xf_estimate",
           "xf_log_prob_backward",
           "xf_plan_last_term_count", "xf_plan_last_work", "xf_plan_set_evaluation", "xf_plan_set_workspace_limit", "xf_plan_set_mixed_condition",
           "xf_plan_set_tree_growth", "xf_plan_set_reuse_samples",
           "xf_expm_antihermitian", "xf_expm_adjoint", "xf_spin_rotations", "xf_spin_rotations_adjoint",
           "xf_antihermitian_reals_grad", "xf_circuit_from_gates", "xf_sample_gates", "xf_last_error"]

_lib = None


class XfError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(paper_2511_12416_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    S = ctypes.c_int
    L.xf_plan_create.argtypes = [ctypes.POINTER(Circuit), Bits128, S, ctypes.c_int, ctypes.POINTER(P)]
    L.xf_plan_set_params.argtypes = [P, P, P]
    L.xf_plan_refreeze.argtypes = [P]
    L.xf_plan_destroy.argtypes = [P]
    L.xf_extent.argtypes = [P, ctypes.POINTER(D)]
    L.xf_trajectory_bound.argtypes = [D, D, D, D, ctypes.POINTER(I64)]
    L.xf_probabilities.argtypes = [P, P, I64, S, I64, U64, P, P, P, P]
    L.xf_probabilities_noalloc.argtypes = [P, P, I64, S, I64, U64, P, P, P, P]
    L.xf_estimate.argtypes = [P, P, I64, D, D, U64, P, P, P, P]
    L.xf_log_prob_backward.argtypes = [P, P, I64, S, I64, U64, P, P, P, P]
    L.xf_plan_last_term_count.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    L.xf_plan_last_work.argtypes = [P, ctypes.POINTER(Work)]
    L.xf_plan_set_evaluation.argtypes = [P, S]
    L.xf_plan_set_workspace_limit.argtypes = [P, U64]
    L.xf_plan_set_mixed_condition.argtypes = [P, D]
    L.xf_plan_set_tree_growth.argtypes = [P, D]
    L.xf_plan_set_reuse_samples.argtypes = [P, I32]
    L.xf_expm_antihermitian.argtypes = [I32, P, P]
    L.xf_expm_adjoint.argtypes = [I32, P, P, P]
    L.xf_spin_rotations.argtypes = [I32, I32, P, P]
    L.xf_spin_rotations_adjoint.argtypes = [I32, I32, P, P, P]
    L.xf_antihermitian_reals_grad.argtypes = [I32, P, P]
    L.xf_sample_gates.argtypes = [I32, I32, P, Bits128, I64, S, I64, U64, S, ctypes.c_int, P, P]
    L.xf_circuit_from_gates.argtypes = [I32, I32, P, I32, I32, P, P, P, P, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    L.xf_last_error.argtypes = []
    L.xf_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "xf_last_error":
            getattr(L, name).restype = S
    _lib = L
    return L


def check(status: int) -> None:
    if status != XF_OK:
        msg = lib().xf_last_error().decode(errors="replace")
        raise XfError(status, msg)
