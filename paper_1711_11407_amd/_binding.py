"""ctypes declarations of libfpssft.so (the C ABI in include/fpssft.h).

Argument marshalling only: every step of the transform runs in the HIP
kernels behind these calls. Loading fails loudly when the library has not
been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libfpssft.so")

MAX_D = 4
ABI_VERSION = 3
INFO_LEN = 8
FLAG_AXIS_SCHEDULE, FLAG_AMP_AVERAGE, FLAG_LITERAL_PEEL, FLAG_DETERMINISTIC = 0x1, 0x2, 0x4, 0x8
OK, INCOMPLETE, CAPACITY = 0, 1, 2
ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_NOMEM, ERR_NO_DEVICE = -1, -2, -3, -4, -5


class Desc(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("dims", C.c_int32 * MAX_D),
        ("max_iters", C.c_int32),
        ("max_k", C.c_int32),
        ("seed", C.c_uint64),
        ("zero_thresh", C.c_float),
        ("mag_rel_tol", C.c_float),
        ("grid_tol", C.c_float),
        ("flags", C.c_uint32),
        ("schedule", C.POINTER(C.c_int32)),
    ]


class Out(C.Structure):
    _fields_ = [
        ("freqs", C.c_void_p),
        ("amps", C.c_void_p),
        ("rec_iter", C.c_void_p),
        ("rec_bin", C.c_void_p),
        ("rec_sin", C.c_void_p),
        ("info", C.c_void_p),
    ]


class ShapeTuning(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("line_length", C.c_int32),
        ("block_threads", C.c_int32),
        ("lines_samples", C.c_int32),
    ]


class Tuning(C.Structure):
    _fields_ = [
        ("block_threads", C.c_int32),
        ("max_radix", C.c_int32),
        ("chunk_iters", C.c_int32),
        ("lines_wg", C.c_int32),
        ("lines_threads", C.c_int32),
        ("direct_launch", C.c_int32),
        ("lines_samples", C.c_int32),
        ("group_by_length", C.c_int32),
        ("nshapes", C.c_int32),
        ("shapes", C.POINTER(ShapeTuning)),
    ]


# (name, restype, argtypes) for every function the header declares.
SIGNATURES = [
    ("fpssft_strerror", C.c_char_p, [C.c_int32]),
    ("fpssft_abi_version", C.c_int32, []),
    ("fpssft_validate", C.c_int32, [C.POINTER(Desc), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    ("fpssft_schedule_generate", C.c_int32, [C.POINTER(Desc), C.c_int32, C.POINTER(C.c_int32)]),
    ("fpssft_plan_create", C.c_int32, [C.POINTER(Desc), C.c_int32, C.POINTER(Tuning), C.POINTER(C.c_void_p)]),
    ("fpssft_plan", C.c_int32, [C.POINTER(Desc), C.c_int32, C.POINTER(C.c_void_p)]),
    ("fpssft_plan_destroy", C.c_int32, [C.c_void_p]),
    ("fpssft_plan_get_schedule", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]),
    ("fpssft_plan_cube_info", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    ("fpssft_plan_spectra_elems", C.c_int64, [C.c_void_p]),
    ("fpssft_execute", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(Out), C.c_void_p]),
    ("fpssft_execute_noalloc", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(Out), C.c_void_p]),
    ("fpssft_execute_batched", C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.POINTER(Out), C.c_void_p]),
    ("fpssft_lines_fft", C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_int32,
                                     C.c_void_p, C.c_void_p]),
    ("fpssft_lines_fft_all", C.c_int32, [C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p, C.c_void_p]),
    ("fpssft_amp_backward", C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(Out), C.c_void_p, C.c_void_p,
                                        C.c_void_p]),
    ("fpssft_amp_backward_batched", C.c_int32, [C.c_void_p, C.POINTER(Out), C.POINTER(C.c_void_p),
                                                C.POINTER(C.c_void_p), C.c_void_p]),
]

_lib = None


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()' "
                "or python paper_1711_11407_amd/build.py). There is no CPU fallback.")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.fpssft_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {L.fpssft_abi_version()}, the binding expects "
                              f"{ABI_VERSION}: rebuild it")
        _lib = L
    return _lib


class FpsSftError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = lib().fpssft_strerror(status).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")
        self.status = status


def check(status: int, what: str = "") -> int:
    if status < 0:
        raise FpsSftError(status, what)
    return status
