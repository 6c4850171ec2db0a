"""Amplitude tapers for weighted apertures, FP64 (oracle side).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.  The paper's
limitations paragraph (Sec. VIII) names deeply weighted apertures, with
sidelobes near -40 dB, as the case where the FP16 noise floor comes near
and the FP32-accumulate mode is the remedy.  These are the textbook tapers,
written out from their definitions; they share no code with the library's
``bfp_window``.  Pins (tests/test_oracle.py): scipy.signal.windows, and the
sidelobe levels of their transforms (Hamming about -42.7 dB; Taylor at the
design level).
"""
import numpy as np


def hamming(length: int) -> np.ndarray:
    """w[n] = 0.54 - 0.46 cos(2 pi n / (L - 1)), n = 0..L-1 (symmetric)."""
    if length == 1:
        return np.ones(1)
    n = np.arange(length, dtype=np.float64)
    return 0.54 - 0.46 * np.cos(2.0 * np.pi * n / (length - 1))


def taylor(length: int, nbar: int = 5, sll_db: float = 40.0) -> np.ndarray:
    """Taylor taper: the nbar - 1 sidelobes nearest the mainlobe near
    -sll_db dB, the rest falling like a uniform aperture's.

    The line-source pattern of a uniform aperture has zeros at u = +-1, +-2,
    ...; Taylor moves the first nbar - 1 of them to u_i = s sqrt(A^2 +
    (i - 1/2)^2), where cosh(pi A) = 10^(sll/20) sets the sidelobe level and
    s = nbar / sqrt(A^2 + (nbar - 1/2)^2) joins the moved zeros to the
    unmoved ones at u = nbar.  The aperture weight is the Fourier series of
    that pattern P (with P(0) = 1) sampled at the integers m < nbar:
        w(x) = 1 + 2 sum_m F_m cos(2 pi m x),  x in [-1/2, 1/2],  F_m = P(m),
    where P(u) = sinc(u) prod_i (1 - u^2 / u_i^2) / (1 - u^2 / i^2); at
    u = m the uniform factor sinc(u) / (1 - u^2 / m^2) tends to
    (-1)^(m+1) / 2, and the rest is a product over the moved zeros divided
    by one over the other removed zeros.  Scaled to 1 at x = 0."""
    A = np.arccosh(10.0 ** (sll_db / 20.0)) / np.pi
    s2 = nbar ** 2 / (A ** 2 + (nbar - 0.5) ** 2)
    moved = s2 * (A ** 2 + (np.arange(1, nbar) - 0.5) ** 2)   # squares of the moved zeros
    F = np.zeros(nbar)
    for m in range(1, nbar):
        ratio_moved = np.prod(1.0 - m ** 2 / moved)
        others = [i for i in range(1, nbar) if i != m]
        ratio_removed = np.prod([1.0 - m ** 2 / i ** 2 for i in others]) if others else 1.0
        F[m] = (-1) ** (m + 1) * ratio_moved / (2.0 * ratio_removed)
    x = (np.arange(length, dtype=np.float64) - (length - 1) / 2.0) / length
    w = np.ones(length)
    for m in range(1, nbar):
        w += 2.0 * F[m] * np.cos(2.0 * np.pi * m * x)
    return w / (1.0 + 2.0 * F[1:].sum())
