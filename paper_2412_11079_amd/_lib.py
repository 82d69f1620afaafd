"""ctypes declarations of libuot.so (include/uot.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libuot.so")

UOT_OK, UOT_ERR_ARG, UOT_ERR_DTYPE, UOT_ERR_ALIGN, UOT_ERR_WORKSPACE, UOT_ERR_UNSUPPORTED, UOT_ERR_HIP = range(7)
UOT_F64, UOT_F32, UOT_BF16, UOT_FP8_E4M3 = range(4)
UOT_COST_SQEUCLID, UOT_COST_COSINE = 0, 1
UOT_ACC_F32, UOT_ACC_F64 = 0, 1
UOT_FLAG_NONFINITE, UOT_FLAG_ZERO_SUM, UOT_FLAG_NOT_CONVERGED, UOT_FLAG_BARRIER_TIMEOUT = 1, 2, 8, 16
UOT_NOALLOC_SCRATCH_BYTES = 64 << 20

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
_sz = ctypes.c_size_t


class Info(ctypes.Structure):
    _fields_ = [("iters", _i64), ("err", _dbl), ("absorptions", _i32), ("flags", ctypes.c_uint32)]


class Problem(ctypes.Structure):
    _fields_ = [("n", _i64), ("m", _i64), ("a", _vp), ("b", _vp), ("k_dtype", _i32), ("K", _vp),
                ("ldk", _i64), ("C", _vp), ("ldc", _i64), ("eps", _dbl), ("tau", _dbl), ("k_scale", _dbl)]


class Options(ctypes.Structure):
    _fields_ = [("max_iter", _i32), ("check_every", _i32), ("tol", _dbl), ("fused", _i32), ("accum", _i32),
                ("absorb_log_threshold", _dbl), ("checkpoint_every", _i32), ("tune", _i32),
                ("u0", _vp), ("v0", _vp), ("persistent", _i32), ("store_iterates", _i32)]


class Outputs(ctypes.Structure):
    _fields_ = [("u", _vp), ("v", _vp), ("r", _vp), ("c", _vp), ("loss", _vp), ("info", _vp), ("ckpt", _vp),
                ("f", _vp), ("g", _vp)]


class Profile(ctypes.Structure):
    _fields_ = [("fused_launches", _i32), ("fused_ms", ctypes.c_float),
                ("row_launches", _i32), ("row_ms", ctypes.c_float),
                ("col_launches", _i32), ("col_ms", ctypes.c_float),
                ("finalize_launches", _i32), ("finalize_ms", ctypes.c_float),
                ("loop_ms", ctypes.c_float)]


class BatchedMeta(ctypes.Structure):
    _fields_ = [("count", _i32), ("k_dtype", _i32), ("m_lds", _i64), ("items", _i32), ("nsplit", _i32),
                ("pool_bytes", _i64)]


class EpsSchedule(ctypes.Structure):
    _fields_ = [("eps0", _dbl), ("factor", _dbl), ("stage_iters", _i32), ("reserved", _i32)]


# Every symbol that include/uot.h declares, with its ctypes signature.
SIGNATURES = {
    "uot_status_string": ([_i32], ctypes.c_char_p),
    "uot_last_error": ([], ctypes.c_char_p),
    "uot_cost_workspace_size": ([_i64, _i64], _sz),
    "uot_cost_from_points": ([_vp, _vp, _i64, _i64, _i64, _i32, _i32, _vp, _i64, _vp, _sz, _vp], _i32),
    "uot_kernel_from_cost": ([_vp, _i64, _i64, _i64, _dbl, _vp, _vp, _i32, _vp, _i64, _vp], _i32),
    "uot_sinkhorn_workspace_size": ([ctypes.POINTER(Problem), ctypes.POINTER(Options)], _sz),
    "uot_sinkhorn": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(Outputs), _vp, _sz, _vp],
                     _i32),
    "uot_matrix_rescale_workspace_size": ([ctypes.POINTER(Problem), ctypes.POINTER(Options)], _sz),
    "uot_matrix_rescale": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(Outputs), _vp, _sz,
                            _vp], _i32),
    "uot_sinkhorn_points_workspace_size": ([ctypes.POINTER(Problem), _i64, _dbl, ctypes.POINTER(Options)], _sz),
    "uot_sinkhorn_points": ([ctypes.POINTER(Problem), _vp, _vp, _i64, _dbl, ctypes.POINTER(Options),
                             ctypes.POINTER(Outputs), _vp, _sz, _vp], _i32),
    "uot_sinkhorn_lse_workspace_size": ([ctypes.POINTER(Problem), ctypes.POINTER(Options),
                                         ctypes.POINTER(EpsSchedule)], _sz),
    "uot_sinkhorn_lse": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(EpsSchedule),
                          ctypes.POINTER(Outputs), _vp, _sz, _vp], _i32),
    "uot_sinkhorn_noalloc": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(Outputs), _vp],
                             _i32),
    "uot_sinkhorn_profiled": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(Outputs), _vp,
                               _sz, _vp, ctypes.POINTER(Profile)], _i32),
    "uot_kernel_to_f32": ([_vp, _i32, _i64, _dbl, _vp, _vp], _i32),
    "uot_sinkhorn_backward_workspace_size": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), _i64, _i32], _sz),
    "uot_sinkhorn_backward": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), _vp, _vp, _vp, _vp, _vp, _vp,
                               _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _sz, _vp], _i32),
    "uot_sinkhorn_implicit_backward_workspace_size": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), _i64],
                                                      _sz),
    "uot_sinkhorn_implicit_backward": ([ctypes.POINTER(Problem), ctypes.POINTER(Options), _vp, _vp, _vp, _vp, _vp,
                                        _vp, _i64, _vp, _vp, _i64, _vp, _vp, _vp, _sz, _vp], _i32),
    "uot_sinkhorn_batched_workspace_size": ([_i32], _sz),
    "uot_sinkhorn_batched": ([ctypes.POINTER(Problem), _i32, ctypes.POINTER(Options), ctypes.POINTER(Outputs), _vp,
                              _sz, _vp], _i32),
    "uot_batched_desc_bytes": ([_i32], _sz),
    "uot_batched_pack": ([ctypes.POINTER(Problem), _i32, ctypes.POINTER(Options), ctypes.POINTER(Outputs), _vp,
                          _sz], _i32),
    "uot_sinkhorn_batched_packed": ([_vp, ctypes.POINTER(BatchedMeta), ctypes.POINTER(Options), _vp, _sz, _vp,
                                     _vp], _i32),
    "uot_batched_tune": ([ctypes.POINTER(Problem), _i32, ctypes.POINTER(Options), ctypes.POINTER(Outputs), _vp,
                          _sz, _vp], _i32),
    "uot_device_wall_clock_khz": ([], _i64),
    "uot_plan": ([ctypes.POINTER(Problem), _vp, _vp, _vp, _vp, _vp, _i64, _i32, _vp], _i32),
    "uot_sinkhorn_multi_workspace_size": ([ctypes.POINTER(Problem), _i32, ctypes.POINTER(Options)], _sz),
    "uot_sinkhorn_multi": ([ctypes.POINTER(Problem), _i32, _vp, _vp, ctypes.POINTER(Options), _vp, _vp, _vp, _vp,
                            _vp, _sz, _vp], _i32),
}

_lib = None


class UOTError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"uot status {status}: {message}")
        self.status = status
        self.message = message


def lib():
    """Load the in-tree libuot.so; fails loudly when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2412_11079_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != UOT_OK:
        msg = lib().uot_last_error()
        raise UOTError(status, msg.decode() if msg else "")
