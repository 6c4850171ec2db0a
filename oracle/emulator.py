"""CPU emulation of the paper's low-precision FFT experiments (test infrastructure).

Two harnesses, both written from the text of the paper:

* ``fp16_radix2_fft`` -- Sec. III-A / Table I: a radix-2 Stockham FFT carried
  out entirely in IEEE half precision, every arithmetic result rounded to
  nearest-even FP16, with FP16 twiddles rounded once from FP64.  Two
  butterflies: the standard one (complex product by 4 multiplies and 2 adds,
  then a +/- t) and a dual-select FMA butterfly (6 fused multiply-adds) that
  factors the larger of |cos|, |sin| out of the twiddle, following the
  fused-multiply-add FFT formulation of Linzer & Feig (1993).
* ``storage_fft`` -- Sec. VII / Table V: FP64 arithmetic and twiddles, with
  the data rounded to a storage format (FP16, OCP FP8 E4M3 or E5M2,
  saturating) after the input and after every radix-2 stage.  Two of the
  precision-recovery ideas the paper names as future work (Sec. VII,
  Sec. VIII) are options of the same harness: stochastic rounding (round up
  with probability equal to the distance to the lower neighbour, in units of
  the spacing), and error feedback, in which each stored value keeps its
  rounding residual, itself stored in the same format, and the next stage
  reads the sum of the two (twice the bytes).

Rounding: FP16 sums and products are formed in FP32 and rounded to FP16.
FP32 carries 24 >= 2*11+2 significand bits, so this double rounding equals a
single correct rounding for +, -, x.  FMAs are formed in FP64 before the one
rounding to FP16.
"""
import numpy as np

from . import fft as _oracle_fft
from . import root as _oracle_root


# ----------------------------------------------------------------- formats --
FORMATS = {
    # name: (mantissa bits, minimum normal exponent, max finite, saturating)
    "fp16": (10, -14, 65504.0, False),
    "e4m3": (3, -6, 448.0, True),
    "e5m2": (2, -14, 57344.0, True),
}


def round_to_format(x, fmt: str):
    """Round real values to nearest-even in ``fmt``.  FP8 formats saturate at
    their largest finite value (OCP convention with saturation); FP16 overflows
    to +/-inf as IEEE does."""
    mant, emin, vmax, sat = FORMATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    if fmt == "fp16":
        return x.astype(np.float16).astype(np.float64)
    ax = np.abs(x)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.maximum(e, emin)
    q = np.ldexp(1.0, (e - mant).astype(np.int64))
    r = np.rint(x / q) * q
    if sat:
        r = np.clip(r, -vmax, vmax)
    return r


def round_complex(z, fmt: str):
    return round_to_format(z.real, fmt) + 1j * round_to_format(z.imag, fmt)


def round_to_format_stochastic(x, fmt: str, u):
    """Stochastic rounding to ``fmt``: with lo <= x < hi the neighbouring
    values of the format, x rounds to hi when u < (x - lo) / (hi - lo), else
    to lo; u are uniform [0, 1) draws of x's shape.  Exact values stay."""
    mant, emin, vmax, sat = FORMATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    ax = np.abs(x)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    e = np.maximum(e, emin)
    q = np.ldexp(1.0, (e - mant).astype(np.int64))
    lo = np.floor(x / q) * q
    r = np.where(u < (x - lo) / q, lo + q, lo)
    if sat:
        r = np.clip(r, -vmax, vmax)
    return r


def _f16(a):
    """Round an FP32/FP64 array to FP16 and return it as FP32 (exact)."""
    return np.asarray(a, dtype=np.float32).astype(np.float16).astype(np.float32)


def _fma16(a, b, c):
    return _f16(np.asarray(a, np.float64) * np.asarray(b, np.float64) + np.asarray(c, np.float64))


def _twiddles(n):
    """W_n^j = exp(-2 pi i j / n), j < n/2, from the oracle's FP64 roots."""
    return np.array([_oracle_root(j, n) for j in range(n // 2)], dtype=np.complex128)


def fp16_radix2_fft(x, butterfly: str = "standard"):
    """Radix-2 Stockham FFT of each row of ``x`` in emulated FP16 arithmetic.

    ``x`` is complex; it is rounded to FP16 first.  Returns complex128 values
    that are exactly the FP16 results."""
    x = np.atleast_2d(np.asarray(x))
    rows, n = x.shape
    stages = int(np.log2(n))
    assert 1 << stages == n
    w64 = _twiddles(n)
    wr = _f16(w64.real)
    wi = _f16(w64.imag)
    if butterfly == "fma6":
        use_c = np.abs(w64.real) >= np.abs(w64.imag)
        # ratio and the factored magnitude, each rounded once from FP64
        with np.errstate(divide="ignore", invalid="ignore"):
            ratio = np.where(use_c, w64.imag / w64.real, w64.real / w64.imag)
        ratio = _f16(ratio)
        fac = _f16(np.where(use_c, w64.real, w64.imag))
    ar = _f16(x.real)
    ai = _f16(x.imag)
    half = n // 2
    l = 1  # size of the sub-transforms already done
    m = half  # number of butterflies per sub-block
    for _ in range(stages):
        # Stockham autosort: input viewed as (2, m, l)... output (m, 2, l)
        a_r = ar.reshape(rows, 2, m, l)
        a_i = ai.reshape(rows, 2, m, l)
        c0r, c1r = a_r[:, 0], a_r[:, 1]
        c0i, c1i = a_i[:, 0], a_i[:, 1]
        # twiddle index for position (j, k): k * m  (W_{2l}^k = W_n^{k m})
        tw_idx = (np.arange(l) * m)[None, :]
        if butterfly == "standard":
            twr = wr[tw_idx]
            twi = wi[tw_idx]
            p1 = _f16(c1r * twr)
            p2 = _f16(c1i * twi)
            p3 = _f16(c1r * twi)
            p4 = _f16(c1i * twr)
            tr = _f16(p1 - p2)
            ti = _f16(p3 + p4)
            yr0 = _f16(c0r + tr)
            yi0 = _f16(c0i + ti)
            yr1 = _f16(c0r - tr)
            yi1 = _f16(c0i - ti)
        elif butterfly == "fma6":
            uc = use_c[tw_idx]
            rt = ratio[tw_idx]
            fc = fac[tw_idx]
            # |c| >= |s|:  w b = c [(br - (s/c) bi) + i (bi + (s/c) br)]
            # |s| >  |c|:  w b = s [((c/s) br - bi) + i ((c/s) bi + br)]
            u = np.where(uc, _fma16(-rt, c1i, c1r), _fma16(rt, c1r, -c1i))
            v = np.where(uc, _fma16(rt, c1r, c1i), _fma16(rt, c1i, c1r))
            yr0 = _fma16(fc, u, c0r)
            yi0 = _fma16(fc, v, c0i)
            yr1 = _fma16(-fc, u, c0r)
            yi1 = _fma16(-fc, v, c0i)
        else:
            raise ValueError(butterfly)
        out_r = np.stack([yr0, yr1], axis=2)  # (rows, m, 2, l)
        out_i = np.stack([yi0, yi1], axis=2)
        ar = out_r.reshape(rows, n)
        ai = out_i.reshape(rows, n)
        l *= 2
        m //= 2
    return ar.astype(np.float64) + 1j * ai.astype(np.float64)


def storage_fft(x, fmt: str, rounding: str = "rne", feedback: bool = False, seed: int = 0):
    """Radix-2 Stockham FFT in FP64 arithmetic with FP64 twiddles, rounding the
    data to ``fmt`` after the input and after each of the log2(N) stages.

    rounding="stochastic": each rounding is stochastic (uniform draws from
    numpy's generator seeded with ``seed``).  feedback=True: each stored
    value is the pair (r, round(x - r)) with r = round(x), both in ``fmt``,
    and every stage reads their sum."""
    x = np.atleast_2d(np.asarray(x, dtype=np.complex128))
    rows, n = x.shape
    stages = int(np.log2(n))
    w = _twiddles(n)
    rng = np.random.default_rng(seed)

    def rnd(v):
        if rounding == "rne":
            return round_complex(v, fmt)
        if rounding == "stochastic":
            return (round_to_format_stochastic(v.real, fmt, rng.random(v.shape)) +
                    1j * round_to_format_stochastic(v.imag, fmt, rng.random(v.shape)))
        raise ValueError(rounding)

    def store(v):
        r = rnd(v)
        return r + rnd(v - r) if feedback else r

    a = store(x)
    l, m = 1, n // 2
    for _ in range(stages):
        v = a.reshape(rows, 2, m, l)
        c0, c1 = v[:, 0], v[:, 1]
        t = c1 * w[(np.arange(l) * m)][None, None, :]
        out = np.stack([c0 + t, c0 - t], axis=2)
        a = store(out.reshape(rows, n))
        l *= 2
        m //= 2
    return a


def sqnr_db(ref, out):
    ref = np.asarray(ref)
    err = np.asarray(out) - ref
    return 10.0 * np.log10(np.sum(np.abs(ref) ** 2) / np.sum(np.abs(err) ** 2))


def table1_sqnr(n: int, butterfly: str, trials: int = 200, seed: int = 0):
    """Table I harness: complex N(0,1) draws, SQNR of the FP16 FFT against the
    FP64 FFT of the unquantised draw, pooled over all trials."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((2, trials, n))
    x = g[0] + 1j * g[1]
    ref = _oracle_fft(x)
    return sqnr_db(ref, fp16_radix2_fft(x, butterfly))


def table5_sqnr(n: int, fmt: str, trials: int = 200, seed: int = 0, rounding: str = "rne",
                feedback: bool = False):
    """Table V harness (storage rounding, double compute), optionally with
    stochastic rounding or error feedback."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((2, trials, n))
    x = g[0] + 1j * g[1]
    ref = _oracle_fft(x)
    return sqnr_db(ref, storage_fft(x, fmt, rounding=rounding, feedback=feedback, seed=seed + 1))


def fp16_compress(x, H, bfp: bool = True, butterfly: str = "standard"):
    """Matched-filter chain y = (1/N) IFFT(FFT(x) . H) in emulated pure FP16,
    with the inverse realised as conj-FFT-conj (Sec. III-B).

    bfp=True folds the exact 1/N = 2^-log2N shift into the pre-inverse
    conjugate (Eq. (1)); bfp=False applies it after the inverse, as the
    conventional output scaling does."""
    x = np.atleast_2d(np.asarray(x))
    n = x.shape[-1]
    k = int(np.log2(n))
    X = fp16_radix2_fft(x, butterfly)
    Hr = _f16(np.real(H))
    Hi = _f16(np.imag(H))
    zr = _f16(_f16(X.real * Hr) - _f16(X.imag * Hi))
    zi = _f16(_f16(X.real * Hi) + _f16(X.imag * Hr))
    zi = -zi  # conj
    if bfp:
        zr = _f16(np.ldexp(zr, -k))
        zi = _f16(np.ldexp(zi, -k))
    with np.errstate(over="ignore", invalid="ignore"):
        Y = fp16_radix2_fft(zr + 1j * zi, butterfly)
        y = np.conj(Y)
        if not bfp:
            y = _f16(np.ldexp(y.real, -k)) + 1j * _f16(np.ldexp(y.imag, -k))
    return y
