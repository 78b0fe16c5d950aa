"""ctypes declarations of liboim.so (include/oim.h).  Loading fails loudly when
the HIP library has not been built: there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboim.so")

OIM_OK, OIM_E_ARG, OIM_E_CSR, OIM_E_ASYM, OIM_E_NONFINITE = 0, 1, 2, 3, 4
OIM_E_UNSUPPORTED, OIM_E_NOMEM, OIM_E_HIP, OIM_E_STATE = 5, 6, 7, 8

OIM_LOOP_AUTO, OIM_LOOP_PERSISTENT, OIM_LOOP_STEPWISE = 0x0, 0x1, 0x2
OIM_PREC_FP32, OIM_PREC_BF16X3 = 0x0, 0x10
OIM_SCHED_PER_REPLICA = 0x100

_P = ctypes.c_void_p
_i32, _i64, _u32, _f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_float


# OIM_ABI_VERSION of the header these declarations follow
ABI_VERSION = 4


class RunCfg(ctypes.Structure):
    _fields_ = [("q", _i32), ("R", _i32), ("steps", _i32), ("dt", _f32),
                ("readout_every", _i32), ("flags", _u32)]


class Readout(ctypes.Structure):
    _fields_ = [("trace", _P), ("best_h", _P), ("best_step", _P), ("best_colour", _P)]


class AdjointCfg(ctypes.Structure):
    _fields_ = [("q", _i32), ("R", _i32), ("steps", _i32), ("dt", _f32),
                ("checkpoint_every", _i32), ("flags", _u32)]


OIM_TUNE_MAX = 64


class TuneReport(ctypes.Structure):
    _fields_ = [("n_tried", _i32), ("chosen_block", _i32), ("chosen_slices_per_wave", _i32),
                ("chosen_rows_per_lane", _i32), ("chosen_ms", _f32),
                ("block", _i32 * OIM_TUNE_MAX), ("slices_per_wave", _i32 * OIM_TUNE_MAX),
                ("rows_per_lane", _i32 * OIM_TUNE_MAX), ("ms", _f32 * OIM_TUNE_MAX)]


class ProblemInfo(ctypes.Structure):
    _fields_ = [("n", _i32), ("is_dense", _i32), ("nnz", _i64), ("integer_weights", _i32),
                ("n_instances", _i32), ("max_abs_row_sum", ctypes.c_double),
                ("sum_J_upper", ctypes.c_double), ("max_instance_n", _i32),
                ("uniform_weight", _f32), ("stepwise_row_length", _i32)]


# every symbol declared in include/oim.h, with its ctypes prototype
PROTOTYPES = {
    "oim_abi_version": (ctypes.c_int, []),
    "oim_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "oim_last_error": (ctypes.c_char_p, []),
    "oim_problem_from_csr": (ctypes.c_int, [_i32, _i64, _P, _P, _P, _u32, ctypes.POINTER(_P)]),
    "oim_problem_from_csr_blocks": (ctypes.c_int, [_i32, _i64, _P, _P, _P, _i32, _P, _u32,
                                                   ctypes.POINTER(_P)]),
    "oim_problem_from_dense": (ctypes.c_int, [_i32, _P, _u32, ctypes.POINTER(_P)]),
    "oim_problem_destroy": (None, [_P]),
    "oim_problem_info_get": (ctypes.c_int, [_P, ctypes.POINTER(ProblemInfo)]),
    "oim_run": (ctypes.c_int, [_P, ctypes.POINTER(RunCfg), _P, _P, _P, _P, _i64, _P, _P,
                               ctypes.POINTER(Readout), _P]),
    "oim_run_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(RunCfg), _P, _P, _P, _P, _i64, _P,
                                       _P, ctypes.POINTER(Readout), _P]),
    "oim_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "oim_phase_from_theta": (ctypes.c_int, [_i64, _P, _P, _P]),
    "oim_theta_from_phase": (ctypes.c_int, [_i64, _P, _P, _P]),
    "oim_round": (ctypes.c_int, [_i32, _i64, _P, _P, _P]),
    "oim_cut": (ctypes.c_int, [_P, _i32, _P, _P, _P, _P]),
    "oim_conflicts": (ctypes.c_int, [_P, _i32, _P, _P, _P]),
    "oim_energy": (ctypes.c_int, [_P, _i32, _i32, _P, _P, _P, _P, _P]),
    "oim_autotune": (ctypes.c_int, [_P, ctypes.POINTER(RunCfg), _P, _P, _P, _P, _P, _i32,
                                    ctypes.POINTER(TuneReport), _P]),
    "oim_set_tuning": (ctypes.c_int, [_P, _i32, _i32, _i32, _i32]),
    "oim_adjoint_checkpoint_words": (ctypes.c_int, [_P, ctypes.POINTER(AdjointCfg),
                                                    ctypes.POINTER(_i64)]),
    "oim_adjoint_forward": (ctypes.c_int, [_P, ctypes.POINTER(AdjointCfg), _P, _P, _P, _P, _i64,
                                           _P, _P, _P, _P, _P]),
    "oim_adjoint_backward": (ctypes.c_int, [_P, ctypes.POINTER(AdjointCfg), _P, _P, _P, _P,
                                            _i64, _P, _P, _P, _P, _P]),
}

_lib = None


class OimError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        self.detail = detail
        super().__init__(f"{status_name(status)}: {detail}")


def lib():
    """The loaded liboim.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.oim_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {L.oim_abi_version()}, this binding "
                              f"{ABI_VERSION}: rebuild the HIP library")
        _lib = L
    return _lib


def status_name(s: int) -> str:
    return lib().oim_status_str(int(s)).decode()


def check(status: int) -> None:
    if status != OIM_OK:
        raise OimError(status, lib().oim_last_error().decode())
