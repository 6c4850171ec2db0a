"""Block-floating-point half-precision FFT and range-Doppler SAR for MI355X.

The compute path is the HIP library ``libbfpfft.so`` (C ABI in
``include/bfpfft.h``); this package only marshals arguments to it.
"""
from . import scenes  # noqa: F401
from ._lib import (FLAG_CHECK_FINITE, FLAG_CONJ_FILTER, FLAG_NAIVE_POSTSCALE,  # noqa: F401
                   FLAG_OUT_FP32, FORMATS, PRECISIONS, BfpError)
from .api import (FFTPlan, UnevenPlan, convert, corner_turn, device_count, empty, filter_format,  # noqa: F401
                  filter_tensor, make_filter, storage_format, to_device, to_host)
