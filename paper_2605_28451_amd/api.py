"""Thin torch binding over the C ABI (argument marshalling only).

Storage tensors carry a trailing axis of 2 (re, im): float32 for FP32,
float16 for the FP16 modes, uint8 for the FP8 modes.  torch supplies device
memory and the current stream; every step of the computation runs in the HIP
kernels of libbfpfft.so.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (FILTER_OF, FLAG_CHECK_FINITE, FLAG_CONJ_FILTER, FLAG_NAIVE_POSTSCALE,
                   FLAG_OUT_FP32, FLAG_TRANSPOSED_STORE, FORMATS, PRECISIONS, STORAGE_OF, check)

TORCH_DTYPE = {"fp32": torch.float32, "fp16": torch.float16, "e4m3": torch.uint8, "e5m2": torch.uint8}


def _prec(p):
    if isinstance(p, str):
        return PRECISIONS[p]
    return int(p)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def storage_format(precision) -> str:
    return STORAGE_OF[_prec(precision)]


def filter_format(precision) -> str:
    return FILTER_OF[_prec(precision)]


def empty(shape, fmt: str, device="cuda"):
    """Uninitialised storage tensor of complex shape `shape` in format `fmt`."""
    return torch.empty(tuple(shape) + (2,), dtype=TORCH_DTYPE[fmt], device=device)


def _check_storage(t, fmt, count, what):
    if t.dtype != TORCH_DTYPE[fmt]:
        raise TypeError(f"{what}: expected dtype {TORCH_DTYPE[fmt]} for {fmt}, got {t.dtype}")
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{what}: must be a contiguous device tensor")
    if t.numel() != 2 * count:
        raise ValueError(f"{what}: expected {count} complex elements, got {t.numel() // 2}")


def device_count() -> int:
    return int(_lib.load().bfp_device_count())


def make_filter(replica: np.ndarray, n: int, fmt: str) -> np.ndarray:
    """Matched filter conj(DFT_n(h)) / max|DFT_n(h)| (host FP64, rounded once),
    returned as a host storage array of shape (n, 2)."""
    h = np.ascontiguousarray(np.asarray(replica, dtype=np.complex128).reshape(-1))
    out = np.empty((n, 2), dtype={"fp32": np.float32, "fp16": np.float16,
                                  "e4m3": np.uint8, "e5m2": np.uint8}[fmt])
    check(_lib.load().bfp_make_filter(h.ctypes.data_as(ctypes.c_void_p), h.size, n,
                                      FORMATS[fmt], out.ctypes.data_as(ctypes.c_void_p)),
          "bfp_make_filter")
    return out


WINDOWS = {"rect": 0, "hamming": 1, "taylor": 2}


def window(kind: str, length: int, nbar: int = 5, sll_db: float = 40.0) -> np.ndarray:
    """Amplitude taper (host FP64) for weighted matched filters: 'rect',
    'hamming' or 'taylor' (nbar terms, nearest sidelobes near -sll_db dB).
    Multiply a replica by it over the replica's support before make_filter."""
    out = np.empty(int(length), dtype=np.float64)
    check(_lib.load().bfp_window(WINDOWS[kind], int(length), int(nbar), float(sll_db),
                                 out.ctypes.data_as(ctypes.c_void_p)), "bfp_window")
    return out


def filter_tensor(replica, n: int, precision, device="cuda"):
    """The filter in the plan's filter format, on the device."""
    return torch.from_numpy(make_filter(replica, n, filter_format(precision))).to(device)


def convert(x, in_fmt: str, out_fmt: str, out=None, stream=None):
    count = x.numel() // 2
    _check_storage(x, in_fmt, count, "convert input")
    if out is None:
        out = torch.empty(x.shape, dtype=TORCH_DTYPE[out_fmt], device=x.device)
    _check_storage(out, out_fmt, count, "convert output")
    check(_lib.load().bfp_convert(_ptr(x), FORMATS[in_fmt], _ptr(out), FORMATS[out_fmt], count,
                                  _stream(stream)), "bfp_convert")
    return out


def device_copy(src, dst, stream=None):
    """Streaming copy of a whole tensor (bytes a multiple of 16)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    check(_lib.load().bfp_device_copy(_ptr(src), _ptr(dst), nbytes, _stream(stream)),
          "bfp_device_copy")
    return dst


def corner_turn(x, fmt: str, out=None, stream=None):
    """out[c][r] = x[r][c] for a (rows, cols, 2) storage tensor."""
    rows, cols = x.shape[0], x.shape[1]
    _check_storage(x, fmt, rows * cols, "corner_turn input")
    if out is None:
        out = empty((cols, rows), fmt, x.device)
    _check_storage(out, fmt, rows * cols, "corner_turn output")
    check(_lib.load().sar_corner_turn(_ptr(x), _ptr(out), rows, cols, FORMATS[fmt],
                                      _stream(stream)), "sar_corner_turn")
    return out


class Tuning(ctypes.Structure):
    """bfp_tuning: the knobs of fft_plan_set_tuning_ex."""
    _fields_ = [("engine", ctypes.c_int), ("blocks_per_cu", ctypes.c_int),
                ("rows_per_thread", ctypes.c_int), ("radix_plan", ctypes.c_int)]


class FFTPlan:
    """Batched length-n transforms in one precision mode (see include/bfpfft.h)."""

    def __init__(self, n: int, batch: int, precision="fp16", flags: int = 0):
        lib = _lib.load()
        self.n = int(n)
        self.batch = int(batch)
        self.prec = _prec(precision)
        self.flags = int(flags)
        self._h = None
        h = ctypes.c_void_p()
        check(lib.fft_plan(ctypes.byref(h), self.n, self.batch, self.prec, self.flags), "fft_plan")
        self._h = h
        self.fmt = STORAGE_OF[self.prec]
        self.filter_fmt = FILTER_OF[self.prec]

    # ------------------------------------------------------------ helpers
    def _out(self, out, rows, fp32=False):
        fmt = "fp32" if fp32 else self.fmt
        if out is None:
            out = empty((rows, self.n), fmt)
        _check_storage(out, fmt, rows * self.n, "output")
        return out

    def _rows_of(self, x, rows):
        if rows is None:
            rows = self.batch
        _check_storage(x, self.fmt, rows * self.n, "input")
        return rows

    # -------------------------------------------------------------- calls
    def forward(self, x, out=None, stream=None):
        self._rows_of(x, None)
        out = self._out(out, self.batch, bool(self.flags & FLAG_OUT_FP32))
        check(_lib.load().fft_exec_fwd(self._h, _ptr(x), _ptr(out), _stream(stream)), "fft_exec_fwd")
        return out

    def inverse_bfp(self, z, filt=None, out=None, naive=False, conj_filter=False, stream=None):
        self._rows_of(z, None)
        out = self._out(out, self.batch, bool(self.flags & FLAG_OUT_FP32))
        if filt is not None:
            _check_storage(filt, self.filter_fmt, self.n, "filter")
        fl = (FLAG_NAIVE_POSTSCALE if naive else 0) | (FLAG_CONJ_FILTER if conj_filter else 0)
        check(_lib.load().fft_exec_inv_bfp_flags(self._h, _ptr(z), _ptr(out), _ptr(filt), fl,
                                                 _stream(stream)), "fft_exec_inv_bfp")
        return out

    def inverse_bfp_adaptive(self, z, filt=None, out=None, row_exp=None, stream=None):
        """BFP inverse with a per-row adaptive shift: returns (out, row_exp);
        the true rows are out[r] * 2**row_exp[r] (int32 row_exp on the device)."""
        self._rows_of(z, None)
        out = self._out(out, self.batch, False)
        if filt is not None:
            _check_storage(filt, self.filter_fmt, self.n, "filter")
        if row_exp is None:
            row_exp = torch.empty(self.batch, dtype=torch.int32, device=out.device)
        assert row_exp.dtype == torch.int32 and row_exp.numel() >= self.batch and row_exp.is_contiguous()
        check(_lib.load().fft_exec_inv_bfp_adaptive(self._h, _ptr(z), _ptr(out), _ptr(filt),
                                                    _ptr(row_exp), 0, _stream(stream)),
              "fft_exec_inv_bfp_adaptive")
        return out, row_exp

    def range_compress_adaptive(self, echo, filt, out=None, rows=None, row_exp=None, stream=None):
        """Fused compression with a per-row adaptive shift: (out, row_exp)."""
        rows = self._rows_of(echo, rows)
        out = self._out(out, rows, False)
        _check_storage(filt, self.filter_fmt, self.n, "filter")
        if row_exp is None:
            row_exp = torch.empty(rows, dtype=torch.int32, device=out.device)
        assert row_exp.dtype == torch.int32 and row_exp.numel() >= rows and row_exp.is_contiguous()
        check(_lib.load().sar_range_compress_adaptive(self._h, _ptr(echo), _ptr(out), _ptr(filt),
                                                      rows, _ptr(row_exp), 0, _stream(stream)),
              "sar_range_compress_adaptive")
        return out, row_exp

    def range_compress_rcmc(self, x, filt, shift, out=None, rows=None, stream=None):
        """Range compression with migration correction of Doppler-domain rows:
        row r compressed by filt and moved shift[r] bins toward smaller range
        (shift: device float32, one per row)."""
        rows = self._rows_of(x, rows)
        out = self._out(out, rows, False)
        _check_storage(filt, self.filter_fmt, self.n, "filter")
        assert shift.dtype == torch.float32 and shift.numel() >= rows and shift.is_contiguous()
        check(_lib.load().sar_range_compress_rcmc(self._h, _ptr(x), _ptr(out), _ptr(filt),
                                                  _ptr(shift), rows, 0, _stream(stream)),
              "sar_range_compress_rcmc")
        return out

    def range_compress(self, echo, filt, out=None, rows=None, naive=False, out_fp32=False,
                       transposed=False, stream=None):
        """transposed=True stores the result corner-turned, shape (n, rows):
        the layout azimuth_compress reads (the corner turn fused into the store)."""
        rows = self._rows_of(echo, rows)
        if transposed:
            if out is None:
                out = empty((self.n, rows), self.fmt)
            _check_storage(out, self.fmt, rows * self.n, "output")
        else:
            out = self._out(out, rows, out_fp32 or bool(self.flags & FLAG_OUT_FP32))
        _check_storage(filt, self.filter_fmt, self.n, "filter")
        fl = ((FLAG_NAIVE_POSTSCALE if naive else 0) | (FLAG_OUT_FP32 if out_fp32 else 0) |
              (FLAG_TRANSPOSED_STORE if transposed else 0))
        check(_lib.load().sar_range_compress(self._h, _ptr(echo), _ptr(out), _ptr(filt), rows, fl,
                                             _stream(stream)), "sar_range_compress")
        return out

    def azimuth_compress(self, rc_t, filt, out=None, rows=None, phase=None, adjoint=False,
                         naive=False, out_fp32=False, stream=None):
        rows = self._rows_of(rc_t, rows)
        out = self._out(out, rows, out_fp32 or bool(self.flags & FLAG_OUT_FP32))
        _check_storage(filt, self.filter_fmt, self.n, "filter")
        if phase is not None:
            if phase.dtype != torch.float32 or phase.numel() != self.n or not phase.is_cuda:
                raise ValueError("phase must be a float32 device tensor of n values")
        fl = (FLAG_NAIVE_POSTSCALE if naive else 0) | (FLAG_OUT_FP32 if out_fp32 else 0)
        check(_lib.load().sar_azimuth_compress(self._h, _ptr(rc_t), _ptr(out), _ptr(filt),
                                               _ptr(phase), rows, int(bool(adjoint)), fl,
                                               _stream(stream)), "sar_azimuth_compress")
        return out


    # ------------------------------------------------------------ tuning
    def set_tuning(self, engine: int = 1, blocks_per_cu: int = -1):
        check(_lib.load().fft_plan_set_tuning(self._h, int(engine), int(blocks_per_cu)),
              "fft_plan_set_tuning")

    def get_tuning(self):
        e, b = ctypes.c_int(), ctypes.c_int()
        check(_lib.load().fft_plan_get_tuning(self._h, ctypes.byref(e), ctypes.byref(b)),
              "fft_plan_get_tuning")
        return int(e.value), int(b.value)

    def set_tuning_ex(self, engine: int = 1, blocks_per_cu: int = -1, rows_per_thread: int = 1,
                      radix_plan: int = 0):
        t = Tuning(int(engine), int(blocks_per_cu), int(rows_per_thread), int(radix_plan))
        check(_lib.load().fft_plan_set_tuning_ex(self._h, ctypes.byref(t)), "fft_plan_set_tuning_ex")

    def get_tuning_ex(self):
        """(engine, blocks_per_cu, rows_per_thread, radix_plan)"""
        t = Tuning()
        check(_lib.load().fft_plan_get_tuning_ex(self._h, ctypes.byref(t)), "fft_plan_get_tuning_ex")
        return int(t.engine), int(t.blocks_per_cu), int(t.rows_per_thread), int(t.radix_plan)

    def autotune_on(self, op: int, x, out, filt=None, reps: int = 20, stream=None) -> float:
        """Time every tuning candidate on (x, out), keep the fastest; returns ms/call.
        x and out may also be equal-length lists of tensors: the calls then
        rotate over the pairs (sets larger than the last-level cache time
        every candidate from HBM)."""
        ms = ctypes.c_float()
        if isinstance(x, (list, tuple)):
            if len(x) != len(out) or not x:
                raise ValueError("x and out: lists of the same nonzero length")
            ins = (ctypes.c_void_p * len(x))(*[t.data_ptr() for t in x])
            outs = (ctypes.c_void_p * len(out))(*[t.data_ptr() for t in out])
            check(_lib.load().fft_autotune_sets(self._h, int(op), ins, outs, len(x), _ptr(filt), int(reps),
                                                ctypes.byref(ms), _stream(stream)), "fft_autotune_sets")
        else:
            check(_lib.load().fft_autotune(self._h, int(op), _ptr(x), _ptr(out), _ptr(filt), int(reps),
                                           ctypes.byref(ms), _stream(stream)), "fft_autotune")
        return float(ms.value)

    def nonfinite(self, stream=None) -> int:
        c = ctypes.c_ulonglong()
        check(_lib.load().fft_plan_nonfinite(self._h, _stream(stream), ctypes.byref(c)),
              "fft_plan_nonfinite")
        return int(c.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class UnevenPlan:
    """One persistent launch over transforms of mixed length and direction.

    log2n[i] in [8, 14]; inverse[i] = 1 selects the BFP inverse (no filter).
    Transforms are packed back to back in the given order."""

    def __init__(self, log2n, inverse, precision="fp16", flags: int = 0):
        lib = _lib.load()
        l2 = np.ascontiguousarray(np.asarray(log2n, dtype=np.int32))
        inv = np.ascontiguousarray(np.asarray(inverse, dtype=np.uint8))
        if l2.shape != inv.shape:
            raise ValueError("log2n and inverse must have the same length")
        self.count = int(l2.size)
        self.prec = _prec(precision)
        self._h = None
        h = ctypes.c_void_p()
        check(lib.fft_plan_uneven(ctypes.byref(h), self.count, l2.ctypes.data_as(ctypes.c_void_p),
                                  inv.ctypes.data_as(ctypes.c_void_p), self.prec, int(flags)),
              "fft_plan_uneven")
        self._h = h
        self.fmt = STORAGE_OF[self.prec]
        tot = ctypes.c_longlong()
        check(lib.fft_uneven_total(self._h, ctypes.byref(tot)), "fft_uneven_total")
        self.total = int(tot.value)
        self.offsets = np.empty(self.count, dtype=np.int64)
        if self.count:
            check(lib.fft_uneven_offsets(self._h, self.offsets.ctypes.data_as(
                ctypes.POINTER(ctypes.c_longlong))), "fft_uneven_offsets")

    # ------------------------------------------------------------ tuning
    def set_tuning(self, engine: int = 1, blocks_per_cu: int = 0):
        check(_lib.load().fft_plan_set_tuning(self._h, int(engine), int(blocks_per_cu)),
              "fft_plan_set_tuning")

    def get_tuning(self):
        e, b = ctypes.c_int(), ctypes.c_int()
        check(_lib.load().fft_plan_get_tuning(self._h, ctypes.byref(e), ctypes.byref(b)),
              "fft_plan_get_tuning")
        return int(e.value), int(b.value)

    def set_tuning_ex(self, engine: int = 0, blocks_per_cu: int = 0, rows_per_thread: int = 1,
                      radix_plan: int = 0):
        t = Tuning(int(engine), int(blocks_per_cu), int(rows_per_thread), int(radix_plan))
        check(_lib.load().fft_plan_set_tuning_ex(self._h, ctypes.byref(t)), "fft_plan_set_tuning_ex")

    def autotune_on(self, op: int, x, out, filt=None, reps: int = 20, stream=None) -> float:
        """Time every tuning candidate on (x, out), keep the fastest; returns ms/call.
        x and out may also be equal-length lists of tensors: the calls then
        rotate over the pairs (sets larger than the last-level cache time
        every candidate from HBM)."""
        ms = ctypes.c_float()
        if isinstance(x, (list, tuple)):
            if len(x) != len(out) or not x:
                raise ValueError("x and out: lists of the same nonzero length")
            ins = (ctypes.c_void_p * len(x))(*[t.data_ptr() for t in x])
            outs = (ctypes.c_void_p * len(out))(*[t.data_ptr() for t in out])
            check(_lib.load().fft_autotune_sets(self._h, int(op), ins, outs, len(x), _ptr(filt), int(reps),
                                                ctypes.byref(ms), _stream(stream)), "fft_autotune_sets")
        else:
            check(_lib.load().fft_autotune(self._h, int(op), _ptr(x), _ptr(out), _ptr(filt), int(reps),
                                           ctypes.byref(ms), _stream(stream)), "fft_autotune")
        return float(ms.value)

    def execute(self, x, out=None, stream=None):
        _check_storage(x, self.fmt, self.total, "input")
        if out is None:
            out = empty((self.total,), self.fmt, x.device)
        _check_storage(out, self.fmt, self.total, "output")
        check(_lib.load().fft_exec_uneven(self._h, _ptr(x), _ptr(out), _stream(stream)),
              "fft_exec_uneven")
        return out

    def nonfinite(self, stream=None) -> int:
        c = ctypes.c_ulonglong()
        check(_lib.load().fft_plan_nonfinite(self._h, _stream(stream), ctypes.byref(c)),
              "fft_plan_nonfinite")
        return int(c.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().fft_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------- host helpers --
def to_device(x: np.ndarray, fmt: str, device="cuda"):
    """Encode complex values to `fmt` (round to nearest-even) and upload."""
    from .scenes import encode
    return torch.from_numpy(np.ascontiguousarray(encode(x, fmt))).to(device)


def to_host(t, fmt: str) -> np.ndarray:
    """Download a storage tensor and decode it exactly to complex128."""
    from .scenes import decode
    return decode(t.detach().cpu().numpy(), fmt)
