"""Seeded synthetic inputs shared by the GPU path, its tests and the oracle.

This module holds no arithmetic of the transform or of matched filtering: it
draws random numbers, synthesises radar echoes (replicas placed at target
positions plus noise) and encodes values into the storage formats.  The
paper's scene (Sec. VI: X-band, B = 100 MHz, v = 100 m/s, R0 = 20 km, 20 dB
additive noise) is not fully specified, so the workloads are stated in
normalised units:

* range replica: linear-FM chirp h[n] = exp(+i pi b (n - L/2)^2 / L),
  n = 0..L-1, b = 0.8, L = 1024 (sweeps -b/2..+b/2 cycles/sample);
* azimuth phase history of a target centred on pulse c:
  exp(-i pi b_a (m - c)^2 / A) for |m - c| < A/2, b_a = 0.8, A = 512
  (parabolic history; the migration of this geometry stays below one range
  bin, so no range-cell-migration correction is needed);
* noise: circular complex white Gaussian, E|n|^2 = 10^(-SNR/10) relative to a
  unit-amplitude target.

Chirp phases are reduced exactly in integers before the one FP64 exp.
Storage encoders round to nearest-even (FP16, FP32) or to nearest-even with
saturation (OCP FP8 E4M3 / E5M2).
"""
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

# ------------------------------------------------------------ replicas ----

def lfm_chirp(length: int, b_num: int = 4, b_den: int = 5, sign: int = +1) -> np.ndarray:
    """exp(sign * i pi (b_num/b_den) (n - L/2)^2 / L), n = 0..L-1 (FP64)."""
    n = np.arange(length, dtype=np.int64) - length // 2
    den = 2 * length * b_den  # phase in cycles = b_num n^2 / den
    q = (b_num * n * n) % den
    return np.exp(sign * 2j * np.pi * q.astype(np.float64) / den)


def azimuth_replica_centred(n: int, aperture: int = 512, b_num: int = 4, b_den: int = 5) -> np.ndarray:
    """Length-n azimuth replica centred on index 0 (circularly wrapped):
    g[m mod n] = exp(-i pi b_a m^2 / A) for -A/2 <= m < A/2."""
    m = np.arange(-aperture // 2, aperture // 2, dtype=np.int64)
    den = 2 * aperture * b_den
    q = (b_num * m * m) % den
    g = np.zeros(n, dtype=np.complex128)
    g[m % n] = np.exp(-2j * np.pi * q.astype(np.float64) / den)
    return g


def range_replica_padded(n: int, length: int = 1024, b_num: int = 4, b_den: int = 5) -> np.ndarray:
    h = np.zeros(n, dtype=np.complex128)
    h[:length] = lfm_chirp(length, b_num, b_den, +1)
    return h


def weighted_range_replica(n: int, taper, length: int = 1024, b_num: int = 4,
                           b_den: int = 5) -> np.ndarray:
    """range_replica_padded with its `length` chirp samples multiplied by the
    given taper (weighted matched filter; the echo itself is unweighted)."""
    taper = np.asarray(taper, dtype=np.float64)
    assert taper.shape == (length,)
    h = range_replica_padded(n, length, b_num, b_den)
    h[:length] *= taper
    return h


def weighted_azimuth_replica(n: int, taper, aperture: int = 512, b_num: int = 4,
                             b_den: int = 5) -> np.ndarray:
    """azimuth_replica_centred with sample m (-A/2 <= m < A/2) multiplied by
    taper[m + A/2]."""
    taper = np.asarray(taper, dtype=np.float64)
    assert taper.shape == (aperture,)
    g = azimuth_replica_centred(n, aperture, b_num, b_den)
    m = np.arange(-aperture // 2, aperture // 2, dtype=np.int64)
    g[m % n] *= taper
    return g


def awgn(rng, shape, snr_db: float) -> np.ndarray:
    p = 10.0 ** (-snr_db / 10.0)
    g = rng.standard_normal((2,) + tuple(shape))
    return np.sqrt(p / 2.0) * (g[0] + 1j * g[1])


# ----------------------------------------------------------- workloads ----

def gaussian_rows(seed: int, rows: int, n: int) -> np.ndarray:
    """Complex N(0,1) per component: x = g[0] + i g[1], g ~ N(0,1)^(2,rows,n)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((2, rows, n))
    return g[0] + 1j * g[1]


@dataclass
class RangeScene:
    echo: np.ndarray        # [pulse][range] complex128
    replica: np.ndarray     # length-n zero-padded range replica
    delays: np.ndarray      # target range starts


def range_scene(seed: int = 2, n_pulses: int = 2048, n: int = 4096, length: int = 1024,
                n_targets: int = 5, snr_db: float = 20.0) -> RangeScene:
    """Point targets of unit amplitude at uniform random range delays
    d ~ U{0..n-L} (the same for every pulse; no circular wrap) plus AWGN drawn
    independently per pulse after the target draws."""
    rng = np.random.default_rng(seed)
    delays = rng.integers(0, n - length + 1, size=n_targets)
    h = lfm_chirp(length)
    line = np.zeros(n, dtype=np.complex128)
    for d in delays:
        line[d:d + length] += h
    echo = np.broadcast_to(line, (n_pulses, n)).copy()
    echo += awgn(rng, (n_pulses, n), snr_db)
    return RangeScene(echo=echo, replica=range_replica_padded(n, length), delays=delays)


@dataclass
class SarScene:
    echo: np.ndarray                 # [pulse][range] complex128
    range_replica: np.ndarray        # length n_range, zero-padded chirp
    azimuth_replica: np.ndarray      # length n_pulse, centred on 0
    targets: List[Tuple[int, int]]   # (range start, azimuth centre)
    phase_error: np.ndarray = field(default=None)  # per-pulse radians (or None)


def sar_scene(seed: int = 3, n: int = 4096, length: int = 1024, aperture: int = 512,
              ranges=(1024, 2048, 3072), azimuths=(1024, 2048, 3072), snr_db: float = 20.0,
              n_pulse: int = None, phase_error: np.ndarray = None) -> SarScene:
    """Raw echo [pulse][range] of a grid of unit point targets.

    A target (range start d, azimuth centre c) contributes
    h[k - d] * exp(-i pi b_a (m - c)^2 / A) at pulse m, range sample k.
    ``phase_error`` (per pulse, radians) multiplies pulse m by exp(i phi_m)."""
    n_pulse = n if n_pulse is None else n_pulse
    rng = np.random.default_rng(seed)
    h = lfm_chirp(length)
    echo = np.zeros((n_pulse, n), dtype=np.complex128)
    ha = lfm_chirp(aperture, sign=-1)  # exp(-i pi b (u - A/2)^2 / A), u = 0..A-1
    targets = []
    for d in ranges:
        for c in azimuths:
            m0 = c - aperture // 2
            rows = (np.arange(aperture) + m0) % n_pulse
            echo[np.ix_(rows, np.arange(d, d + length) % n)] += np.outer(ha, h)
            targets.append((int(d), int(c)))
    echo += awgn(rng, (n_pulse, n), snr_db)
    if phase_error is not None:
        echo *= np.exp(1j * np.asarray(phase_error, dtype=np.float64))[:, None]
    return SarScene(echo=echo, range_replica=range_replica_padded(n, length),
                    azimuth_replica=azimuth_replica_centred(n_pulse, aperture),
                    targets=targets, phase_error=phase_error)


def autofocus_phase_error(seed: int = 5, n_pulse: int = 4096, quad_rad: float = 4 * np.pi,
                          half_aperture: int = 256, sigma: float = 0.3) -> np.ndarray:
    """phi_m = quad_rad ((m - n/2) / half_aperture)^2 + N(0, sigma^2) per pulse."""
    rng = np.random.default_rng(seed)
    m = np.arange(n_pulse, dtype=np.float64)
    return quad_rad * ((m - n_pulse // 2) / half_aperture) ** 2 + sigma * rng.standard_normal(n_pulse)


@dataclass
class UnevenBatch:
    log2n: np.ndarray      # int32 per transform
    inverse: np.ndarray    # uint8 per transform (1 = BFP inverse)
    offsets: np.ndarray    # int64 element offset of each transform (packed in order)
    x: np.ndarray          # packed complex128 data


def uneven_batch(seed: int = 4, count: int = 20000, e_min: int = 8, e_max: int = 14) -> UnevenBatch:
    """count transforms, N = 2^e with e ~ U{e_min..e_max}, direction ~ Bernoulli(1/2),
    packed back to back in draw order, N(0,1) complex data."""
    rng = np.random.default_rng(seed)
    e = rng.integers(e_min, e_max + 1, size=count).astype(np.int32)
    inv = rng.integers(0, 2, size=count).astype(np.uint8)
    sizes = (1 << e.astype(np.int64))
    offsets = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    total = int(sizes.sum())
    g = rng.standard_normal((2, total))
    return UnevenBatch(log2n=e, inverse=inv, offsets=offsets, x=g[0] + 1j * g[1])


# ------------------------------------------------------------ storage ----
_FP8 = {
    # mantissa bits, exponent bias, max finite, has infinities
    "e4m3": (3, 7, 448.0),
    "e5m2": (2, 15, 57344.0),
}


def _fp8_encode_real(v: np.ndarray, fmt: str) -> np.ndarray:
    mant, bias, vmax = _FP8[fmt]
    emin = 1 - bias
    v = np.asarray(v, dtype=np.float64)
    sign = np.signbit(v)
    a = np.minimum(np.abs(v), vmax)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0))).astype(np.int64)
    e = np.maximum(e, emin)
    a = np.where(np.isnan(a), 0.0, a)
    q = np.rint(np.ldexp(a, (mant - e)))  # significand in units of the quantum
    # rounding may carry into the next binade
    carry = q >= (2 << mant)
    e = np.where(carry, e + 1, e)
    q = np.where(carry, q / 2, q)
    q = q.astype(np.int64)
    normal = q >= (1 << mant)
    ef = np.where(normal, e + bias, 0)
    mf = np.where(normal, q - (1 << mant), q)
    bits = (ef << mant) | mf
    bits = np.where(a == 0, 0, bits)
    bits = np.where(np.isnan(v), 0x7F, bits)  # NaN stays NaN (both formats)
    return (bits | (sign.astype(np.int64) << 7)).astype(np.uint8)


def _fp8_decode_real(b: np.ndarray, fmt: str) -> np.ndarray:
    mant, bias, _ = _FP8[fmt]
    b = np.asarray(b, dtype=np.int64)
    s = np.where(b & 0x80, -1.0, 1.0)
    ef = (b >> mant) & ((1 << (7 - mant)) - 1)
    mf = b & ((1 << mant) - 1)
    val = np.where(ef == 0, np.ldexp(mf.astype(np.float64), 1 - bias - mant),
                   np.ldexp((mf + (1 << mant)).astype(np.float64), (ef - bias - mant)))
    if fmt == "e4m3":  # S.1111.111 is NaN; no infinities
        val = np.where((ef == 15) & (mf == 7), np.nan, val)
    else:              # exponent 31: infinity (mantissa 0) or NaN
        val = np.where(ef == 31, np.where(mf == 0, np.inf, np.nan), val)
    return s * val


STORAGE_FORMATS = ("fp32", "fp16", "e4m3", "e5m2")


def encode(x: np.ndarray, fmt: str) -> np.ndarray:
    """Complex values -> interleaved (re, im) storage array of shape x.shape + (2,)."""
    x = np.asarray(x, dtype=np.complex128)
    pair = np.stack([x.real, x.imag], axis=-1)
    if fmt == "fp32":
        return pair.astype(np.float32)
    if fmt == "fp16":
        return pair.astype(np.float16)
    if fmt in _FP8:
        return _fp8_encode_real(pair, fmt)
    raise ValueError(fmt)


def decode(a: np.ndarray, fmt: str) -> np.ndarray:
    """Interleaved storage array (..., 2) -> complex128 (exact)."""
    if fmt in ("fp32", "fp16"):
        a = np.asarray(a).astype(np.float64)
    elif fmt in _FP8:
        a = _fp8_decode_real(a, fmt)
    else:
        raise ValueError(fmt)
    out = np.empty(a.shape[:-1], dtype=np.complex128)
    out.real = a[..., 0]
    out.imag = a[..., 1]
    return out


def quantize(x: np.ndarray, fmt: str) -> np.ndarray:
    """The storage-rounded values as complex128 (what both sides consume)."""
    return decode(encode(x, fmt), fmt)


# ------------------------------------------------- range cell migration ----
# Normalised range-Doppler geometry with true hyperbolic migration (the RCMC
# step of the paper's pipeline, Sec. VI; its scene states no geometry).  In
# range bins: slant range R(m) = sqrt(rho0^2 + kappa^2 m^2) at pulse offset m
# from closest approach; two-way phase -2 pi mu R(m) with mu = 2 dr / lambda
# (cycles of two-way path per range bin).  kappa^2 = rho_ref (b_a / A) / mu
# gives, at the reference range, the azimuth chirp of the unmigrated scene
# (b_a over A pulses); the migration at the aperture edge is then
# A b_a / (8 mu) range bins (6.4 for A = 512, b_a = 0.8, mu = 8).  A far
# reference range (rho_ref = 1e6 bins) keeps the azimuth FM rate and the
# migration within 0.1% over the swath, so one azimuth filter and one
# migration curve (range-invariant RCMC at the reference range) apply.

@dataclass
class MigrationScene:
    echo: np.ndarray                 # [pulse][range] complex128
    range_replica: np.ndarray        # length n_range, zero-padded chirp
    azimuth_replica: np.ndarray      # length n_pulse, centred on 0, hyperbolic phase at rho_ref
    rcmc_shift: np.ndarray           # per Doppler bin k: range shift (bins) that undoes the migration
    targets: List[Tuple[int, int]]   # (range start at closest approach, azimuth centre)
    migration_edge_bins: float       # migration at the aperture edge


def migration_scene(seed: int = 7, n: int = 4096, length: int = 1024, aperture: int = 512,
                    ranges=(1536, 2048, 2560), azimuths=(1024, 2048, 3072), mu: float = 8.0,
                    rho_ref: float = 1.0e6, b_num: int = 4, b_den: int = 5,
                    snr_db: float = 20.0) -> MigrationScene:
    """Raw echo [pulse][range] of unit point targets with hyperbolic range
    migration.  A target (range start d, azimuth centre c) sits at closest
    range rho0 = rho_ref + d - n/2; at pulse m (|m - c| < A/2) its echo is the
    range chirp delayed by R - rho0 bins beyond d (sampled from the analytic
    chirp at fractional delay) times exp(-2 pi i mu (R - rho0))."""
    rng = np.random.default_rng(seed)
    b = b_num / b_den
    kappa2 = rho_ref * (b / aperture) / mu
    echo = np.zeros((n, n), dtype=np.complex128)
    k = np.arange(n, dtype=np.float64)
    for d in ranges:
        rho0 = rho_ref + d - n // 2
        for c in azimuths:
            for m in range(c - aperture // 2, c + aperture // 2):
                dm = m - c
                R = np.sqrt(rho0 * rho0 + kappa2 * dm * dm)
                delay = d + (R - rho0)
                t = k - delay                       # chirp time in samples
                on = (t >= 0.0) & (t < length)
                tc = t[on] - length / 2.0
                echo[m % n, on] += np.exp(1j * np.pi * b * tc * tc / length) * \
                    np.exp(-2j * np.pi * mu * (R - rho0))
    echo += awgn(rng, (n, n), snr_db)
    # azimuth replica at the reference range, centred on pulse 0
    mm = np.arange(-aperture // 2, aperture // 2, dtype=np.float64)
    Rr = np.sqrt(rho_ref * rho_ref + kappa2 * mm * mm)
    g = np.zeros(n, dtype=np.complex128)
    g[np.arange(-aperture // 2, aperture // 2) % n] = np.exp(-2j * np.pi * mu * (Rr - rho_ref))
    # migration per Doppler bin: a target seen at Doppler f (cycles/pulse)
    # sits at range rho / D(f), D = sqrt(1 - (f / (mu kappa))^2)
    f = np.fft.fftfreq(n)
    D = np.sqrt(1.0 - (f / (mu * np.sqrt(kappa2))) ** 2)
    shift = rho_ref * (1.0 / D - 1.0)
    return MigrationScene(echo=echo, range_replica=range_replica_padded(n, length, b_num, b_den),
                          azimuth_replica=g, rcmc_shift=shift,
                          targets=[(d, c) for d in ranges for c in azimuths],
                          migration_edge_bins=float(aperture * b / (8.0 * mu)))
