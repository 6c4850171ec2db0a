"""FP64 CPU oracle for the block-floating-point FFT and range-Doppler SAR path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``; never by the product package.  It shares
no code with the GPU path.  Inputs are numpy ``complex128`` arrays (callers
pass the storage-rounded values, which are exact in FP64).

Every function evaluates the plain mathematical definition (paper Sec. III-B
and Eq. (1)); see ``oracle.c`` for the algorithms.  The block-floating-point
shift is a mathematical no-op, so the oracle computes the exact linear maps.

Parity status of each function is recorded in ``tests/test_oracle.py``; the
FP16/FP8 emulator in ``emulator.py`` reproduces Tables I and V of the paper.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L = ctypes.c_long
        lib.oracle_fft_rows.argtypes = [dp, dp, L, L, ctypes.c_int]
        lib.oracle_dft_direct.argtypes = [dp, dp, L, ctypes.c_int]
        lib.oracle_root.argtypes = [ctypes.c_longlong, ctypes.c_longlong, dp, dp]
        lib.oracle_matched_filter.argtypes = [dp, L, L, dp]
        lib.oracle_compress_rows.argtypes = [dp, dp, dp, L, L, ctypes.c_int]
        lib.oracle_transpose.argtypes = [dp, dp, L, L]
        lib.oracle_apply_phase.argtypes = [dp, dp, dp, L, L]
        lib.oracle_sar_image.argtypes = [dp, L, L, dp, dp, dp, dp, dp]
        lib.oracle_entropy.argtypes = [dp, L, dp]
        lib.oracle_entropy.restype = ctypes.c_double
        lib.oracle_autofocus.argtypes = [dp, L, L, dp, dp, dp, dp]
        lib.oracle_autofocus.restype = ctypes.c_double
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def fft(x, inverse: bool = False):
    """Row-wise forward DFT (unscaled) or normalised inverse over the last axis."""
    x = _c128(x)
    n = x.shape[-1]
    out = np.empty_like(x)
    rows = x.size // n if n else 0
    if _load().oracle_fft_rows(_ptr(x), _ptr(out), rows, n, int(inverse)) != 0:
        raise ValueError("length must be a power of two")
    return out


def dft_direct(x, inverse: bool = False):
    """Brute-force O(N^2) DFT of a 1-D vector of any length."""
    x = _c128(x).reshape(-1)
    out = np.empty_like(x)
    if _load().oracle_dft_direct(_ptr(x), _ptr(out), x.size, int(inverse)) != 0:
        raise ValueError("empty input")
    return out


def root(k: int, n: int) -> complex:
    """exp(-2 pi i k / n) as evaluated by the oracle (exact argument reduction)."""
    re = ctypes.c_double()
    im = ctypes.c_double()
    _load().oracle_root(k, n, ctypes.byref(re), ctypes.byref(im))
    return complex(re.value, im.value)


def matched_filter(h, n: int):
    """H = conj(DFT_n(h)) / max|DFT_n(h)| for a replica h zero-padded to n."""
    h = _c128(h).reshape(-1)
    H = np.empty(n, dtype=np.complex128)
    if _load().oracle_matched_filter(_ptr(h), h.size, n, _ptr(H)) != 0:
        raise ValueError("bad filter length")
    return H


def compress(x, H, conj_filter: bool = False):
    """Row-wise y = IDFT(DFT(x) . H) (conj(H) when conj_filter)."""
    x = _c128(x)
    n = x.shape[-1]
    H = _c128(H).reshape(-1)
    assert H.size == n
    out = np.empty_like(x)
    if _load().oracle_compress_rows(_ptr(x), _ptr(out), _ptr(H), x.size // n, n,
                                    int(conj_filter)) != 0:
        raise ValueError("length must be a power of two")
    return out


def transpose(x):
    x = _c128(x)
    r, c = x.shape
    out = np.empty((c, r), dtype=np.complex128)
    _load().oracle_transpose(_ptr(x), _ptr(out), r, c)
    return out


def sar_image(echo, Hr, Ha, phi=None, return_rc=False):
    """Range-Doppler image [range][azimuth] of an echo [pulse][range]."""
    echo = _c128(echo)
    n_pulse, n_range = echo.shape
    Hr = _c128(Hr).reshape(-1)
    Ha = _c128(Ha).reshape(-1)
    assert Hr.size == n_range and Ha.size == n_pulse
    img = np.empty((n_range, n_pulse), dtype=np.complex128)
    rct = np.empty((n_range, n_pulse), dtype=np.complex128) if return_rc else None
    ph = None if phi is None else np.ascontiguousarray(phi, dtype=np.float64)
    if ph is not None:
        assert ph.size == n_pulse
    if _load().oracle_sar_image(_ptr(echo), n_pulse, n_range, _ptr(Hr), _ptr(Ha),
                                _ptr(ph), _ptr(img), _ptr(rct)) != 0:
        raise ValueError("sizes must be powers of two")
    return (img, rct) if return_rc else img


def apply_phase(rc_t, phi):
    rc_t = _c128(rc_t)
    nr, npul = rc_t.shape
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    out = np.empty_like(rc_t)
    _load().oracle_apply_phase(_ptr(rc_t), _ptr(out), _ptr(ph), nr, npul)
    return out


def entropy(img, want_grad: bool = False):
    img = _c128(img)
    g = np.empty_like(img) if want_grad else None
    E = _load().oracle_entropy(_ptr(img), img.size, _ptr(g))
    return (E, g) if want_grad else E


def autofocus(rc_t, Ha, phi, want_image: bool = False):
    """Entropy E of A_az(rc_t . e^{i phi}) and its analytic gradient dE/dphi."""
    rc_t = _c128(rc_t)
    nr, npul = rc_t.shape
    Ha = _c128(Ha).reshape(-1)
    ph = np.ascontiguousarray(phi, dtype=np.float64)
    g = np.empty(npul, dtype=np.float64)
    img = np.empty_like(rc_t) if want_image else None
    E = _load().oracle_autofocus(_ptr(rc_t), nr, npul, _ptr(Ha), _ptr(ph), _ptr(g), _ptr(img))
    return (E, g, img) if want_image else (E, g)


def adam_step(phi, g, m, v, k, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, 2015, Algorithm 1) in FP64, for step
    number k >= 1: the moment estimates, their bias corrections, and the
    update of phi.  Returns (phi, m, v) as new arrays."""
    phi = np.asarray(phi, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** k)
    v_hat = v / (1.0 - beta2 ** k)
    return phi - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def adaptive_exponent(z, n: int):
    """Per-row exponent of the adaptive block shift (the per-block exponents
    of Sec. VIII's future work, as this library defines them): for the
    inverse's input row z (after the filter product) with M = max(|Re z|,
    |Im z|), k is the smallest integer in [-15, 14] with
    sqrt(2) n M 2^-k < 2^15; returns k - log2(n) per row (true output =
    stored output * 2^exponent).  Plain loops, FP64."""
    z = np.atleast_2d(_c128(z))
    log2n = int(n).bit_length() - 1
    out = np.empty(z.shape[0], dtype=np.int64)
    for r in range(z.shape[0]):
        m = max(np.max(np.abs(z[r].real)), np.max(np.abs(z[r].imag)))
        b = np.sqrt(2.0) * n * m
        k = -15
        while k < 14 and b * 2.0 ** -k >= 2.0 ** 15:
            k += 1
        out[r] = k - log2n
    return out


def rcmc_compress(x, H, shift):
    """Range compression with range cell migration correction, row by row:
    y_r = IDFT(DFT(x_r) . H . exp(+2 pi i k s_r / n)), k the signed bin
    (k - n for k >= n/2).  The linear phase is the band-limited (periodic
    sinc) interpolation y_r[t] = (x_r compressed)[t + s_r]: it moves the row
    s_r bins toward smaller range."""
    x = _c128(x)
    n = x.shape[-1]
    shift = np.asarray(shift, dtype=np.float64).reshape(-1)
    assert shift.size == x.shape[0]
    k = np.arange(n, dtype=np.float64)
    k[n // 2:] -= n
    X = fft(x)
    ramp = np.exp(2j * np.pi * k[None, :] * shift[:, None] / n)
    return fft(X * _c128(H).reshape(1, -1) * ramp, inverse=True)


def rda_rcmc_image(echo, Hr, Ha, shift):
    """Range-Doppler image [range][azimuth] of an echo [pulse][range] with
    range cell migration correction: azimuth DFT (pulses -> Doppler), per
    Doppler bin the range compression with that bin's migration shift
    (rcmc_compress), then per range bin the azimuth compression in the
    Doppler domain, IDFT(. Ha)."""
    echo = _c128(echo)
    rd = transpose(fft(transpose(echo)))          # [Doppler][range]
    rc = rcmc_compress(rd, Hr, shift)             # migration removed
    return fft(transpose(rc) * _c128(Ha).reshape(1, -1), inverse=True)
