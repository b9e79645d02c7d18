"""ctypes binding of libgmminterp.so (argument marshalling only).

torch is imported before the library is loaded so that the HIP runtime that
torch ships is the one the library binds to (both use the same soname).
There is no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # noqa: F401  (loads the HIP runtime before libgmminterp.so)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libgmminterp.so")

INTERP_OK = 0
INTERP_EINVAL = -1
INTERP_ENOMEM = -2
INTERP_EAGAIN = -3
INTERP_EHIP = -4
INTERP_ENOTFOUND = -5

NOALLOC_SCRATCH_BYTES = 64 << 20   # INTERP_NOALLOC_SCRATCH_BYTES
KERNEL_NORMALIZED, KERNEL_DIAGONAL = 1, 2   # INTERP_KERNEL_* flags
STORAGE_F32, STORAGE_BF16, STORAGE_F16 = 0, 1, 2   # INTERP_STORAGE_*

QUEUED, RUNNING, DONE, FAILED = 0, 1, 2, 3

c_int32 = ctypes.c_int32
c_float = ctypes.c_float
c_size_t = ctypes.c_size_t
c_void_p = ctypes.c_void_p


class InterpProblem(ctypes.Structure):
    _fields_ = [("B", c_int32), ("N", c_int32), ("C", c_int32), ("H", c_int32), ("W", c_int32),
                ("radius", c_float), ("tile", c_int32), ("sigma_per_point", c_int32),
                ("kernel", c_int32), ("storage", c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("device", c_int32), ("max_slots", c_int32), ("max_queue", c_int32),
                ("reserved", c_int32), ("hbm_budget_bytes", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("prob", InterpProblem), ("pos", c_void_p), ("sigma", c_void_p),
                ("values", c_void_p), ("out", c_void_p), ("grad_out", c_void_p),
                ("grad_pos", c_void_p), ("grad_sigma", c_void_p), ("grad_values", c_void_p),
                ("ready", c_void_p)]


class Status(ctypes.Structure):
    _fields_ = [("state", c_int32), ("err", c_int32), ("t_submit_ns", ctypes.c_int64),
                ("t_admit_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


# every symbol include/gmminterp.h declares
EXPORTS = [
    "interp_workspace_bytes", "interp_saved_bytes", "interp_forward", "interp_forward_noalloc",
    "interp_backward",
    "interp_debug_bins", "interp_last_error", "interp_profile_enable", "interp_profile_read",
    "interp_server_create", "interp_submit", "interp_submit_many",
    "interp_poll", "interp_server_drain", "interp_server_destroy",
]

_lib = None
_lock = threading.Lock()


def _declare(L):
    P = ctypes.POINTER(InterpProblem)
    L.interp_workspace_bytes.argtypes = [P]
    L.interp_workspace_bytes.restype = c_size_t
    L.interp_saved_bytes.argtypes = [P]
    L.interp_saved_bytes.restype = c_size_t
    L.interp_forward.argtypes = [P, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                 c_void_p, c_size_t, c_void_p]
    L.interp_forward.restype = ctypes.c_int
    L.interp_forward_noalloc.argtypes = [P, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                         c_size_t, c_void_p]
    L.interp_forward_noalloc.restype = ctypes.c_int
    L.interp_backward.argtypes = [P, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t,
                                  c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]
    L.interp_backward.restype = ctypes.c_int
    L.interp_debug_bins.argtypes = [P, c_void_p, c_size_t, c_void_p, c_size_t, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_void_p]
    L.interp_debug_bins.restype = ctypes.c_int
    L.interp_last_error.argtypes = []
    L.interp_last_error.restype = ctypes.c_char_p
    L.interp_profile_enable.argtypes = [ctypes.c_int]
    L.interp_profile_enable.restype = ctypes.c_int
    L.interp_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_int64)]
    L.interp_profile_read.restype = ctypes.c_int
    if not hasattr(L, "interp_server_create"):
        return
    L.interp_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(c_void_p)]
    L.interp_server_create.restype = ctypes.c_int
    L.interp_submit.argtypes = [c_void_p, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.interp_submit.restype = ctypes.c_int
    L.interp_submit_many.argtypes = [c_void_p, ctypes.POINTER(Request), c_int32,
                                     ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(c_int32)]
    L.interp_submit_many.restype = ctypes.c_int
    L.interp_poll.argtypes = [c_void_p, ctypes.c_uint64, ctypes.POINTER(Status)]
    L.interp_poll.restype = ctypes.c_int
    L.interp_server_drain.argtypes = [c_void_p, ctypes.c_int64]
    L.interp_server_drain.restype = ctypes.c_int
    L.interp_server_destroy.argtypes = [c_void_p]
    L.interp_server_destroy.restype = ctypes.c_int


def lib():
    """The loaded library (loaded once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        with _lock:
            if _lib is None:
                if not os.path.exists(LIB_PATH):
                    raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                                       "`python -m paper_2012_13257_amd.build`")
                L = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
                _declare(L)
                _lib = L
    return _lib


def last_error() -> str:
    return lib().interp_last_error().decode(errors="replace")


class InterpError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with code {code}: {msg}")
        self.code = code


def profile_enable(on: bool) -> None:
    check("interp_profile_enable", lib().interp_profile_enable(1 if on else 0))


def profile_read(prefix: str = ""):
    """(total milliseconds, launches) of the recorded kernels whose name starts with prefix."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    check("interp_profile_read", lib().interp_profile_read(prefix.encode(), ctypes.byref(ms),
                                                            ctypes.byref(n)))
    return ms.value, n.value


def check(fn: str, rc: int) -> None:
    if rc != INTERP_OK:
        raise InterpError(fn, rc, last_error())
