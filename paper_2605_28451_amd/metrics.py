"""Image-quality metrics, applied identically to oracle and GPU outputs.

* ``sqnr_db`` -- 10 log10(sum|ref|^2 / sum|ref - a*out|^2), pooled over every
  element.  ``align=True`` uses the optimal real scale a* = Re<out,ref>/|out|^2,
  the amplitude alignment of Sec. IV-B (each transform carries a 1/N block
  exponent relative to an unscaled reference); ``align=False`` uses a = 1.
* ``point_target`` -- PSLR, ISLR, 3 dB impulse-response width (IRW) and SNR
  of one point target, measured in range and in azimuth.  The paper does not
  state its procedure (Sec. VI); the one used here is: take a 64x64 chip
  centred on the peak, upsample it x16 by FFT zero-padding (FP64), cut through
  the upsampled peak along each axis, delimit the mainlobe by the first local
  minimum on each side, then
    PSLR = max sidelobe power / peak power,
    ISLR = sidelobe energy / mainlobe energy within +/-20 samples of the peak,
    IRW  = -3 dB width with linear interpolation of both crossings (samples),
    SNR  = peak power / mean power of a target-free 256x256 patch.
  Image layout is [range][azimuth] (rows = range bins).
"""
import numpy as np

UPSAMPLE = 16
CHIP = 64
ISLR_HALF_WIDTH = 20


def sqnr_db(ref, out, align: bool = False) -> float:
    ref = np.asarray(ref, dtype=np.complex128)
    out = np.asarray(out, dtype=np.complex128)
    a = 1.0
    if align:
        den = np.vdot(out, out).real
        a = np.vdot(out, ref).real / den if den > 0 else 1.0
    err = ref - a * out
    num = np.sum(np.abs(ref) ** 2)
    den = np.sum(np.abs(err) ** 2)
    if den == 0:
        return float("inf")
    return float(10.0 * np.log10(num / den))


def _upsample2d(chip, f):
    """Band-limited x f interpolation by zero-padding the centred 2-D spectrum."""
    n0, n1 = chip.shape
    S = np.fft.fftshift(np.fft.fft2(chip))
    P = np.zeros((n0 * f, n1 * f), dtype=np.complex128)
    o0 = (n0 * f - n0) // 2
    o1 = (n1 * f - n1) // 2
    P[o0:o0 + n0, o1:o1 + n1] = S
    return np.fft.ifft2(np.fft.ifftshift(P)) * (f * f)


def _cut_metrics(p, ipk, f):
    """Metrics of one power cut p (linear) with its peak at index ipk."""
    n = p.size
    peak = p[ipk]
    # first minima on each side
    lo = ipk
    while lo > 0 and p[lo - 1] < p[lo]:
        lo -= 1
    hi = ipk
    while hi < n - 1 and p[hi + 1] < p[hi]:
        hi += 1
    side = np.concatenate([p[:lo], p[hi + 1:]])
    pslr = 10.0 * np.log10(side.max() / peak) if side.size else float("-inf")
    w = ISLR_HALF_WIDTH * f
    a, b = max(0, ipk - w), min(n, ipk + w + 1)
    main_e = p[lo:hi + 1].sum()
    side_e = p[a:lo].sum() + p[hi + 1:b].sum()
    islr = 10.0 * np.log10(side_e / main_e)
    # -3 dB crossings, linear interpolation in power
    half = peak / 2.0
    i = ipk
    while i > 0 and p[i - 1] >= half:
        i -= 1
    xl = i - 1 + (half - p[i - 1]) / (p[i] - p[i - 1]) if i > 0 else 0.0
    j = ipk
    while j < n - 1 and p[j + 1] >= half:
        j += 1
    xr = j + (p[j] - half) / (p[j] - p[j + 1]) if j < n - 1 else float(n - 1)
    irw = (xr - xl) / f
    return pslr, islr, irw


def point_target(img, r0: int, a0: int, search: int = 8, noise_patch=None):
    """Metrics of the target nearest (r0, a0) in an image [range][azimuth].

    noise_patch = (r_start, a_start) of a 256x256 target-free region for SNR
    (omitted: SNR is not computed).  Returns a dict."""
    img = np.asarray(img, dtype=np.complex128)
    nr, na = img.shape
    win = np.abs(img[r0 - search:r0 + search + 1, a0 - search:a0 + search + 1]) ** 2
    k = int(np.argmax(win))
    pr = r0 - search + k // win.shape[1]
    pa = a0 - search + k % win.shape[1]
    h = CHIP // 2
    rows = np.arange(pr - h, pr + h) % nr
    cols = np.arange(pa - h, pa + h) % na
    chip = img[np.ix_(rows, cols)]
    up = np.abs(_upsample2d(chip, UPSAMPLE)) ** 2
    ku = int(np.argmax(up))
    ur, ua = ku // up.shape[1], ku % up.shape[1]
    rng = _cut_metrics(up[:, ua], ur, UPSAMPLE)
    azi = _cut_metrics(up[ur, :], ua, UPSAMPLE)
    out = {
        "peak_rc": (int(pr), int(pa)),
        "peak_power": float(up[ur, ua]),
        "pslr_range": rng[0], "islr_range": rng[1], "irw_range": rng[2],
        "pslr_azimuth": azi[0], "islr_azimuth": azi[1], "irw_azimuth": azi[2],
    }
    if noise_patch is not None:
        nr0, na0 = noise_patch
        patch = img[nr0:nr0 + 256, na0:na0 + 256]
        out["snr"] = float(10.0 * np.log10(np.abs(img[pr, pa]) ** 2 / np.mean(np.abs(patch) ** 2)))
    return out


def cut_metrics_1d(x, f: int = UPSAMPLE):
    """PSLR/ISLR/IRW of a 1-D compressed pulse (peak searched over the whole
    vector), using the same procedure as ``point_target``."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.size
    k = int(np.argmax(np.abs(x)))
    h = CHIP // 2
    idx = np.arange(k - h, k + h) % n
    seg = x[idx]
    S = np.fft.fftshift(np.fft.fft(seg))
    P = np.zeros(CHIP * f, dtype=np.complex128)
    o = (CHIP * f - CHIP) // 2
    P[o:o + CHIP] = S
    up = np.abs(np.fft.ifft(np.fft.ifftshift(P)) * f) ** 2
    ku = int(np.argmax(up))
    return _cut_metrics(up, ku, f)
