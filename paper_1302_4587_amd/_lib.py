"""ctypes binding of the C ABI in include/lm.h (argument marshalling only).

Every step of the matching runs in the HIP library liblm.so. There is no
Python or CPU fallback: if the library is missing, importing this module
fails with an error that says how to build it.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblm.so")

# status codes
LM_OK = 0
LM_PENDING = 1
LM_EINVAL = -1
LM_EGRAPH = -2
LM_EWEIGHT = -3
LM_ENOMEM = -4
LM_ETOOBIG = -5
LM_EAGAIN = -6
LM_ENOTFOUND = -7
LM_EDEVICE = -8

# flags
LM_IN_DEVICE = 0x1
LM_OUT_DEVICE = 0x2
LM_CHECK_GRAPH = 0x4
LM_PROFILE = 0x8
LM_GRAPH = 0x10
LM_WEIGHT_SUM = 0x20
LM_ASYNC = 0x40
LM_RENEW_KEYS = 0x80

# bytes of the per-GPU scratch array of lm_match_noalloc
LM_NOALLOC_SCRATCH_BYTES = 0x4000000

LM_K_INIT, LM_K_ARGMAX, LM_K_MUTUAL, LM_K_COMPACT, LM_K_PLAN, LM_K_TAIL = range(6)
KERNEL_KINDS = ("init", "argmax", "mutual", "compact", "plan", "tail")

LM_SERVE_BATCHED = 0
LM_SERVE_FIFO = 1

EXPORTED = (
    "lm_create", "lm_destroy", "lm_match", "lm_match_noalloc", "lm_match_batch", "lm_get_tuning", "lm_set_tuning",
    "lm_autotune_batch", "lm_server_create", "lm_server_submit", "lm_server_poll", "lm_server_wait",
    "lm_server_destroy", "lm_strerror", "lm_contract",
)


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class PhaseRec(ctypes.Structure):
    _fields_ = [("live_entries", ctypes.c_int64), ("live_rows", ctypes.c_int64),
                ("matched_edges", ctypes.c_int64), ("matched_entries", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("phases", ctypes.c_int32), ("log_len", ctypes.c_int32), ("matched_edges", ctypes.c_int64),
                ("device_ms", ctypes.c_double), ("bytes_alg", ctypes.c_double),
                ("log", ctypes.POINTER(PhaseRec)), ("log_cap", ctypes.c_int32),
                ("profile_kinds", ctypes.c_uint32), ("k_launches", ctypes.c_int32 * 6), ("k_ms", ctypes.c_double * 6),
                ("k_bytes", ctypes.c_double * 6), ("matched_weight", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("block_entries", ctypes.c_int32), ("grid_per_cu", ctypes.c_int32),
                ("phases_per_sync", ctypes.c_int32), ("tail_entries", ctypes.c_int32)]


class Coarse(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("vwgt", ctypes.c_void_p)]


class ContractStats(ctypes.Structure):
    _fields_ = [("device_ms", ctypes.c_double), ("bytes_alg", ctypes.c_double), ("long_rows", ctypes.c_int64),
                ("long_entries", ctypes.c_int64), ("table_rows", ctypes.c_int64)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_resident", ctypes.c_int32),
                ("queue_cap", ctypes.c_int32), ("phases_per_step", ctypes.c_int32), ("mode", ctypes.c_int32)]


class RequestStats(ctypes.Structure):
    _fields_ = [("phases", ctypes.c_int32), ("matched_edges", ctypes.c_int64),
                ("submit_to_admit_ms", ctypes.c_double), ("submit_to_done_ms", ctypes.c_double),
                ("admit_to_solved_ms", ctypes.c_double), ("solved_to_done_ms", ctypes.c_double)]


_lib = None


def load():
    """Loads liblm.so (in-tree build). Raises if it was never built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1302_4587_amd.build` "
                          "(hipcc for gfx950); there is no fallback path")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    lib.lm_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.POINTER(vp)]
    lib.lm_destroy.argtypes = [vp]
    lib.lm_destroy.restype = None
    lib.lm_match.argtypes = [vp, ctypes.POINTER(Csr), u64, vp, u32, vp, ctypes.POINTER(Stats)]
    lib.lm_match_noalloc.argtypes = [vp, ctypes.POINTER(Csr), u64, vp, u32, vp, ctypes.POINTER(Stats)]
    lib.lm_match_batch.argtypes = [vp, i32, vp, i64, vp, vp, vp, vp, u64, vp, u32, vp, ctypes.POINTER(Stats), vp]
    lib.lm_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.lm_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    lib.lm_autotune_batch.argtypes = [vp, i32, vp, i64, vp, vp, vp, u32, ctypes.c_char_p, ctypes.POINTER(Tuning)]
    lib.lm_server_create.argtypes = [vp, ctypes.POINTER(ServerOpts), ctypes.POINTER(vp)]
    lib.lm_server_submit.argtypes = [vp, ctypes.POINTER(Csr), u64, ctypes.POINTER(u64)]
    lib.lm_server_poll.argtypes = [vp, u64, vp, ctypes.POINTER(RequestStats)]
    lib.lm_server_wait.argtypes = [vp, u64, vp, ctypes.POINTER(RequestStats), i64]
    lib.lm_server_destroy.argtypes = [vp]
    lib.lm_contract.argtypes = [vp, ctypes.POINTER(Csr), vp, vp, vp, ctypes.POINTER(Coarse), u32, vp,
                                ctypes.POINTER(ContractStats)]
    lib.lm_strerror.argtypes = [i32]
    lib.lm_strerror.restype = ctypes.c_char_p
    for f in ("lm_create", "lm_match", "lm_match_noalloc", "lm_match_batch", "lm_get_tuning", "lm_set_tuning", "lm_autotune_batch",
              "lm_server_create", "lm_server_submit", "lm_server_poll", "lm_server_wait", "lm_server_destroy", "lm_contract"):
        getattr(lib, f).restype = i32
    _lib = lib
    return lib


class LMError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = load().lm_strerror(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")
        self.status = status


def check(status: int, what: str = "") -> int:
    if status < 0:
        raise LMError(status, what)
    return status


def strerror(status: int) -> str:
    return load().lm_strerror(status).decode()
