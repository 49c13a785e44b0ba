"""ctypes declarations of libpolymat.so (the C ABI of include/polymat.h).

Loading fails loudly when the library has not been built: there is no
fallback path of any kind.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpolymat.so")

PM_OK, PM_ERR_INVALID, PM_ERR_WORKSPACE, PM_ERR_DEVICE, PM_ERR_UNSUPPORTED, PM_ERR_NONFINITE = range(6)
PM_PREC_FP64, PM_PREC_FP32, PM_PREC_BF16X3 = range(3)
PM_OP_N, PM_OP_C = 0, 1
PM_MAX_NTRUNC = 63
NOALLOC_SCRATCH_BYTES = 160 << 20   # PM_NOALLOC_SCRATCH_BYTES
PHASES = ("rescale", "forward", "product", "inverse", "other", "retrunc", "pipeline")


class PmProblem(ctypes.Structure):
    _fields_ = [
        ("A", ctypes.c_void_p),
        ("B", ctypes.c_void_p),
        ("C", ctypes.c_void_p),
        ("n", ctypes.c_int),
        ("ntrunc", ctypes.c_int),
        ("op_a", ctypes.c_int),
        ("op_b", ctypes.c_int),
        ("scale", ctypes.c_double),
    ]


class NsptParams(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("L", ctypes.c_int),
        ("k", ctypes.c_int),
        ("ntrunc", ctypes.c_int),
        ("eps", ctypes.c_double),
    ]


# symbol -> (restype, argtypes); the exported set that include/polymat.h declares
_VP, _SZ, _I, _D = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
_U64 = ctypes.c_ulonglong
SIGNATURES = {
    "polymat_abi_version": (_I, []),
    "polymat_strerror": (ctypes.c_char_p, [_I]),
    "polymat_transform_length": (_I, [_I]),
    "polymat_mul": (_I, [_VP, _VP, _VP, _I, _I, _I, _D, _VP, _SZ, _VP]),
    "polymat_workspace_size": (_SZ, [_I, _I, _I, _I]),
    "polymat_batched_workspace_size": (_SZ, [ctypes.POINTER(PmProblem), _I, _I]),
    "polymat_mul_batched": (_I, [ctypes.POINTER(PmProblem), _I, _I, _VP, _SZ, _VP]),
    "polymat_forward_transform": (_I, [_VP, _VP, _I, _I, _D, _VP, _SZ, _VP]),
    "polymat_inverse_transform": (_I, [_VP, _VP, _I, _I, _D, _VP, _SZ, _VP]),
    "polymat_transform_workspace_size": (_SZ, []),
    "polymat_timing_enable": (_I, [_I]),
    "polymat_check_enable": (_I, [_I]),
    "polymat_mul_noalloc": (_I, [_VP, _VP, _VP, _I, _I, _I, _D, _VP]),
    "polymat_timing_read": (_I, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]),
    "nspt_workspace_size": (_SZ, [_I, ctypes.POINTER(NsptParams), _I]),
    "nspt_langevin_step": (_I, [_VP, _VP, _I, ctypes.POINTER(NsptParams), _I, _VP, _SZ, _VP]),
    "polymat_mul_naive": (_I, [_VP, _VP, _VP, _I, _I, _I, _I, _VP]),
    "nspt_action": (_I, [_VP, _I, ctypes.POINTER(NsptParams), _I, _VP, _VP, _SZ, _VP]),
    "nspt_wilson_loop": (_I, [_VP, _I, ctypes.POINTER(NsptParams), _I, _I, _I, _VP, _VP, _SZ, _VP]),
    "nspt_md_trajectory": (_I, [_VP, _VP, _VP, _I, ctypes.POINTER(NsptParams), _I, _I, _VP, _SZ, _VP]),
    "nspt_gauge_fix": (_I, [_VP, _I, ctypes.POINTER(NsptParams), _D, _I, _VP, _SZ, _VP]),
    "nspt_noise": (_I, [_VP, _I, _I, _U64, _U64, _VP]),
    "nspt_langevin_steps": (_I, [_VP, _I, ctypes.POINTER(NsptParams), _U64, _U64, _I, _I, _VP, _SZ, _VP]),
}

_lib = None


class PolymatError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {strerror(status)} (status {status})")
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2001_02835_amd.build` "
                "(or __graft_entry__.build()); the library has no fallback path")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def strerror(status: int) -> str:
    return lib().polymat_strerror(int(status)).decode()


def check(status: int, what: str) -> None:
    if status != PM_OK:
        raise PolymatError(status, what)
