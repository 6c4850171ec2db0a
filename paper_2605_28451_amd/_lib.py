"""ctypes loader for libbfpfft.so: argument marshalling only.

The library is built in-tree by ``build_lib.py``.  Loading fails loudly when
it is missing: there is no fallback implementation.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfpfft.so")

# bfp_status
OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP, ENODEV = 0, -1, -2, -3, -4, -5

# bfp_precision
PRECISIONS = {
    "fp32": 0,
    "fp16": 1,
    "fp16_fp32": 2,           # FP16 storage / FP32 compute
    "fp16_mul_fp32_acc": 3,   # FP16 multiply / FP32 accumulate
    "e4m3": 4,                # FP8 E4M3 storage
    "e5m2": 5,                # FP8 E5M2 storage
}
# bfp_format
FORMATS = {"fp32": 0, "fp16": 1, "e4m3": 2, "e5m2": 3}
STORAGE_OF = {0: "fp32", 1: "fp16", 2: "fp16", 3: "fp16", 4: "e4m3", 5: "e5m2"}
FILTER_OF = {0: "fp32", 1: "fp16", 2: "fp16", 3: "fp16", 4: "fp32", 5: "fp32"}

# bfp_flags
FLAG_NAIVE_POSTSCALE = 1
FLAG_CHECK_FINITE = 2
FLAG_TRANSPOSED_STORE = 4
FLAG_OUT_FP32 = 8
FLAG_CONJ_FILTER = 16
FLAG_AUTOFOCUS = 32

# every exported entry point: name -> (restype, argtypes)
_P = ctypes.c_void_p
_I = ctypes.c_int
_U = ctypes.c_uint
_LL = ctypes.c_longlong
SIGNATURES = {
    "bfp_storage_bytes": (_I, [_I]),
    "bfp_filter_format": (_I, [_I]),
    "bfp_format_bytes": (_I, [_I]),
    "bfp_status_string": (ctypes.c_char_p, [_I]),
    "bfp_last_error": (ctypes.c_char_p, []),
    "bfp_device_count": (_I, []),
    "fft_plan": (_I, [ctypes.POINTER(_P), _I, _I, _I, _U]),
    "fft_destroy": (_I, [_P]),
    "fft_plan_info": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I), ctypes.POINTER(_I),
                           ctypes.POINTER(_U)]),
    "fft_exec_fwd": (_I, [_P, _P, _P, _P]),
    "fft_exec_inv_bfp": (_I, [_P, _P, _P, _P, _P]),
    "fft_exec_inv_bfp_flags": (_I, [_P, _P, _P, _P, _U, _P]),
    "fft_plan_nonfinite": (_I, [_P, _P, ctypes.POINTER(ctypes.c_ulonglong)]),
    "fft_plan_set_tuning": (_I, [_P, _I, _I]),
    "fft_plan_get_tuning": (_I, [_P, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "fft_plan_set_tuning_ex": (_I, [_P, _P]),
    "fft_plan_get_tuning_ex": (_I, [_P, _P]),
    "fft_autotune": (_I, [_P, _I, _P, _P, _P, _I, ctypes.POINTER(ctypes.c_float), _P]),
    "fft_autotune_sets": (_I, [_P, _I, _P, _P, _I, _P, _I, ctypes.POINTER(ctypes.c_float), _P]),
    "fft_plan_uneven": (_I, [ctypes.POINTER(_P), _I, _P, _P, _I, _U]),
    "fft_uneven_offsets": (_I, [_P, ctypes.POINTER(_LL)]),
    "fft_uneven_total": (_I, [_P, ctypes.POINTER(_LL)]),
    "fft_exec_uneven": (_I, [_P, _P, _P, _P]),
    "bfp_make_filter": (_I, [_P, _I, _I, _I, _P]),
    "bfp_window": (_I, [_I, _I, _I, ctypes.c_double, _P]),
    "fft_exec_inv_bfp_adaptive": (_I, [_P, _P, _P, _P, _P, ctypes.c_uint, _P]),
    "sar_range_compress_adaptive": (_I, [_P, _P, _P, _P, _I, _P, ctypes.c_uint, _P]),
    "sar_range_compress_rcmc": (_I, [_P, _P, _P, _P, _P, _I, ctypes.c_uint, _P]),
    "bfp_convert": (_I, [_P, _I, _P, _I, _LL, _P]),
    "bfp_device_copy": (_I, [_P, _P, _LL, _P]),
    "sar_range_compress": (_I, [_P, _P, _P, _P, _I, _U, _P]),
    "sar_corner_turn": (_I, [_P, _P, _I, _I, _I, _P]),
    "sar_azimuth_compress": (_I, [_P, _P, _P, _P, _P, _I, _I, _U, _P]),
    "sar_image_entropy": (_I, [_P, _P, _LL, _P, _P]),
    "sar_image_entropy_noalloc": (_I, [_P, _LL, _P, _P]),
    "sar_azimuth_image_entropy": (_I, [_P, _P, _P, _P, _P, _I, _P, _P]),
    "sar_entropy_grad": (_I, [_P, _P, _P, _P, _LL, _P]),
    "sar_azimuth_phase_grad": (_I, [_P, _P, _P, _P, _P, _P, _P, _I, _P]),
    "sar_autofocus_adam": (_I, [_P, _P, _P, _P, _P, _I, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, _P]),
    "sar_autofocus_adam_schedule": (_I, [_P, _P, _P, _P, _P, _I, _P, _I, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_float, _P]),
}

_lib = None


class BfpError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def load():
    """Load the library (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2605_28451_amd.build_lib` "
                "(there is no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(status, where):
    if status != OK:
        msg = load().bfp_last_error().decode(errors="replace")
        raise BfpError(status, where, msg)
    return status
