"""ctypes binding of libbg.so (argument marshalling only).

The shared library is built in-tree by ``paper_2106_06507_amd.build``.  There
is no fallback: if the library is missing every entry point raises.
"""
import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbg.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "bg.h")

BG_OK = 0
BG_EINVAL = -1
BG_ERANGE = -2
BG_ENODEV = -3
BG_EDEVICE = -4
BG_ENOMEM = -5
BG_EUNSUPPORTED = -6

MODE_COBG, MODE_CDBG, MODE_AUTO, MODE_LC, MODE_COMC = 0, 1, 2, 3, 4
PREC_FP64, PREC_FP32_MIXED = 0, 1
FLAG_VALIDATE, FLAG_FP32_UNCHECKED = 1, 2


class bg_request(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("mode", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("flags", ctypes.c_uint32),
        ("n_events", ctypes.c_int64),
        ("mom", ctypes.c_void_p),
        ("hel", ctypes.c_void_p),
        ("col", ctypes.c_void_p),
        ("me2", ctypes.c_void_p),
    ]


class bg_batch_config(ctypes.Structure):
    _fields_ = [
        ("blocks_per_cu", ctypes.c_int),
        ("cobg_tile_events", ctypes.c_int),
        ("cdbg_tile_events", ctypes.c_int),
        ("waves_per_simd", ctypes.c_int),
        ("split_kinds", ctypes.c_int),
    ]


BATCH_MAX_SEGS = 32

GEN_CUTS, GEN_HEL, GEN_COL = 1, 2, 4


class bg_gen_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int),
        ("flags", ctypes.c_int),
        ("sqrt_s", ctypes.c_double),
        ("pt_min", ctypes.c_double),
        ("dr_min", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("first_attempt", ctypes.c_uint64),
    ]

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64

_SIGNATURES = {
    "bg_context_create": (_I, [ctypes.POINTER(_P), _I, ctypes.c_uint32]),
    "bg_fp32_check_set": (_I, [_P, _I, _I, ctypes.c_float]),
    "bg_fp32_check_get": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_float)]),
    "bg_context_destroy": (None, [_P]),
    "bg_status_string": (ctypes.c_char_p, [_I]),
    "bg_num_orderings": (_I64, [_I]),
    "bg_color_matrix": (_I, [_I, _P, _I64]),
    "bg_currents": (_I, [_P, _I, _I64, _P, _P, _I, _P, _P]),
    "bg_color_contract": (_I, [_P, _I, _I64, _P, _P, _I, _P]),
    "bg_me2": (_I, [_P, ctypes.POINTER(bg_request), _P]),
    "bg_me2_noalloc": (_I, [_P, ctypes.POINTER(bg_request), _P]),
    "bg_me2_grad": (_I, [_P, ctypes.POINTER(bg_request), _P, _P, _P]),
    "bg_me2_batch": (_I, [_P, ctypes.POINTER(bg_request), _I, _P]),
    "bg_batch_config_get": (_I, [_P, _I, ctypes.POINTER(bg_batch_config)]),
    "bg_batch_config_set": (_I, [_P, _I, ctypes.POINTER(bg_batch_config)]),
    "bg_me2_batch_tune": (_I, [_P, ctypes.POINTER(bg_request), _I, ctypes.POINTER(bg_batch_config),
                               ctypes.POINTER(ctypes.c_double), _P]),
    "bg_generate": (_I, [_P, ctypes.POINTER(bg_gen_params), _I64, _I64, _P, _P, _P, _P, _P, _P]),
    "bg_me2_continuous": (_I, [_P, _I, _I, _I64, _P, _P, _P, _P, _P]),
    "bg_generate_continuous": (_I, [_P, _I, ctypes.c_uint64, ctypes.c_uint64, _I64, _P, _P, _P]),
    "bg_mfma_layout_probe": (_I, [_P, _P]),
}

_lib = None


class BGError(RuntimeError):
    def __init__(self, status, what):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


def header_symbols():
    """Function names declared in include/bg.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\*?\s+\*?(bg_[a-z_0-9]+)\s*\(", text, re.M)))


def lib():
    """Load libbg.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2106_06507_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def status_string(status):
    return lib().bg_status_string(status).decode()


def check(status, what):
    if status != BG_OK:
        raise BGError(status, what)
