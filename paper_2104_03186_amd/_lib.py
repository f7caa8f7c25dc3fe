"""ctypes binding of the C ABI declared in include/lqt.h (marshalling only).

Loads ``liblqt.so`` from this package directory.  There is no fallback: when
the library is missing or cannot be loaded every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblqt.so")

# lqt_status
OK, EINVAL, ENOMEM, ENOTPD, ENONFINITE, EAGAIN, EBUSY, EHIP, ENOTSUP = range(9)
STATUS_NAMES = {OK: "LQT_OK", EINVAL: "LQT_EINVAL", ENOMEM: "LQT_ENOMEM", ENOTPD: "LQT_ENOTPD",
                ENONFINITE: "LQT_ENONFINITE", EAGAIN: "LQT_EAGAIN", EBUSY: "LQT_EBUSY", EHIP: "LQT_EHIP",
                ENOTSUP: "LQT_ENOTSUP"}
PREC_FP64, PREC_MIXED = 0, 1
TRAJ_MAPS, TRAJ_PREFIX = 0, 1
PS_F, PS_c, PS_L, PS_H, PS_X, PS_U = 1, 2, 4, 8, 16, 32

EXPORTED = ("lqt_plan", "lqt_solve", "lqt_tune", "lqt_submit", "lqt_poll", "lqt_serve_stats_read", "lqt_destroy",
            "lqt_profile_enable", "lqt_profile_select", "lqt_profile_read", "lqt_last_error", "lqt_nl_iterate",
            "lqt_fs_solve", "lqt_set_routing", "lqt_solve_noalloc", "lqt_set_graphs", "lqt_graphs_recorded")

_vp = ctypes.c_void_p


class Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("nu", ctypes.c_int32), ("ny", ctypes.c_int32), ("nyT", ctypes.c_int32),
                ("T", ctypes.c_int64), ("per_step", ctypes.c_uint32),
                ("F", _vp), ("c", _vp), ("L", _vp), ("H", _vp), ("X", _vp), ("U", _vp), ("r", _vp),
                ("HT", _vp), ("XT", _vp), ("rT", _vp), ("x0", _vp), ("M", _vp), ("s", _vp)]


class NLProblem(ctypes.Structure):
    _fields_ = [("model", ctypes.c_int32), ("ny", ctypes.c_int32), ("nyT", ctypes.c_int32), ("T", ctypes.c_int64),
                ("per_step", ctypes.c_uint32), ("dt", _vp), ("H", _vp), ("X", _vp), ("U", _vp), ("r", _vp),
                ("HT", _vp), ("XT", _vp), ("rT", _vp), ("x0", _vp)]


NL_UNICYCLE = 0


class FSProblem(ctypes.Structure):
    _fields_ = [("nstates", ctypes.c_int32), ("ncontrols", ctypes.c_int32), ("T", ctypes.c_int64),
                ("per_step", ctypes.c_uint32), ("next", _vp), ("cost", _vp), ("cost_T", _vp), ("x0", ctypes.c_int32)]


class FSOutputs(ctypes.Structure):
    _fields_ = [("V", _vp), ("u", _vp), ("x", _vp), ("ux", _vp), ("status", _vp)]


FS_NEXT, FS_COST = 1, 2


class Outputs(ctypes.Structure):
    _fields_ = [("S", _vp), ("v", _vp), ("K", _vp), ("d", _vp), ("x", _vp), ("u", _vp), ("status", _vp)]


class StageTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_nx", ctypes.c_int32), ("max_nu", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_size_t), ("max_steps", ctypes.c_int64),
                ("max_inflight", ctypes.c_int32), ("trajectory", ctypes.c_int32)]


class Routing(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int32), ("block", ctypes.c_int32), ("lane_chunk", ctypes.c_int32),
                ("wave_chunk", ctypes.c_int32), ("tree", ctypes.c_int32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("queued", ctypes.c_int32), ("running_batches", ctypes.c_int32),
                ("max_running_batches", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("pool_bytes", ctypes.c_size_t), ("pool_in_use", ctypes.c_size_t), ("pool_peak", ctypes.c_size_t)]


_lib = None


class LQTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load liblqt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library {LIB_PATH} is missing: build it with "
                          "`python -m paper_2104_03186_amd.build` (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    lib.lqt_plan.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(_vp)]
    lib.lqt_plan.restype = ctypes.c_int
    lib.lqt_solve.argtypes = [_vp, ctypes.POINTER(Problem), ctypes.POINTER(Outputs), ctypes.c_int32, _vp]
    lib.lqt_solve.restype = ctypes.c_int
    lib.lqt_solve_noalloc.argtypes = [_vp, ctypes.POINTER(Problem), ctypes.POINTER(Outputs), _vp]
    lib.lqt_solve_noalloc.restype = ctypes.c_int
    lib.lqt_tune.argtypes = [_vp, ctypes.POINTER(Problem), ctypes.POINTER(Outputs), ctypes.c_int32, _vp,
                             ctypes.POINTER(ctypes.c_int32)]
    lib.lqt_tune.restype = ctypes.c_int
    lib.lqt_submit.argtypes = [_vp, ctypes.POINTER(Problem), ctypes.POINTER(Outputs), ctypes.POINTER(ctypes.c_uint64)]
    lib.lqt_submit.restype = ctypes.c_int
    lib.lqt_poll.argtypes = [_vp, ctypes.c_uint64]
    lib.lqt_poll.restype = ctypes.c_int
    lib.lqt_serve_stats_read.argtypes = [_vp, ctypes.POINTER(ServeStats)]
    lib.lqt_serve_stats_read.restype = ctypes.c_int
    lib.lqt_destroy.argtypes = [_vp]
    lib.lqt_destroy.restype = ctypes.c_int
    lib.lqt_profile_enable.argtypes = [_vp, ctypes.c_int32]
    lib.lqt_profile_enable.restype = ctypes.c_int
    lib.lqt_profile_select.argtypes = [_vp, ctypes.c_char_p]
    lib.lqt_profile_select.restype = ctypes.c_int
    lib.lqt_profile_read.argtypes = [_vp, ctypes.POINTER(StageTime), ctypes.c_int32]
    lib.lqt_profile_read.restype = ctypes.c_int32
    lib.lqt_nl_iterate.argtypes = [_vp, ctypes.POINTER(NLProblem), ctypes.c_int32, _vp, _vp, _vp, _vp, _vp]
    lib.lqt_nl_iterate.restype = ctypes.c_int
    lib.lqt_fs_solve.argtypes = [_vp, ctypes.POINTER(FSProblem), ctypes.POINTER(FSOutputs), _vp]
    lib.lqt_fs_solve.restype = ctypes.c_int
    lib.lqt_graphs_recorded.argtypes = [_vp]
    lib.lqt_graphs_recorded.restype = ctypes.c_int32
    lib.lqt_set_graphs.argtypes = [_vp, ctypes.c_int32]
    lib.lqt_set_graphs.restype = ctypes.c_int
    lib.lqt_set_routing.argtypes = [_vp, ctypes.POINTER(Routing)]
    lib.lqt_set_routing.restype = ctypes.c_int
    lib.lqt_last_error.argtypes = [_vp]
    lib.lqt_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def last_error(plan) -> str:
    s = load().lqt_last_error(plan)
    return s.decode() if s else ""


def check(code: int, plan=None):
    if code != OK:
        raise LQTError(code, last_error(plan))
