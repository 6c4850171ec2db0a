"""Pins of the quality metrics (SQNR, PSLR, ISLR, IRW, SNR) against closed forms.

The metric code is applied identically to oracle and GPU images, so the
"within 0.1 dB" comparisons are method-consistent; these tests pin the
method itself to textbook values for an unweighted aperture (sinc response:
PSLR -13.26 dB, 3 dB width 0.886 / b) and to the matched-filter SNR gain.
"""
import numpy as np
import pytest

import oracle
from paper_2605_28451_amd import metrics
from paper_2605_28451_amd import scenes


def test_sqnr_definitions():
    rng = np.random.default_rng(0)
    ref = rng.standard_normal(1000) + 1j * rng.standard_normal(1000)
    assert metrics.sqnr_db(ref, 3 * ref) == pytest.approx(-10 * np.log10(4), abs=1e-12)
    assert metrics.sqnr_db(ref, 3 * ref, align=True) > 250
    noise = 1e-3 * (rng.standard_normal(1000) + 1j * rng.standard_normal(1000))
    expect = 10 * np.log10(np.sum(np.abs(ref) ** 2) / np.sum(np.abs(noise) ** 2))
    assert metrics.sqnr_db(ref, ref + noise) == pytest.approx(expect, abs=1e-9)
    # alignment only rescales: for an unbiased error it changes little
    assert metrics.sqnr_db(ref, 0.5 * (ref + noise), align=True) == pytest.approx(expect, abs=0.01)


def _sinc_islr(b, half_width=20):
    # closed-form definition evaluated by quadrature on a fine grid
    u = np.linspace(-half_width, half_width, 2_000_001)
    p = np.sinc(b * u) ** 2
    main = np.abs(u) <= 1.0 / b
    du = u[1] - u[0]
    return 10 * np.log10(p[~main].sum() * du / (p[main].sum() * du))


@pytest.mark.parametrize("frac", [0.0, 0.3, 0.5])
def test_ideal_sinc_response(frac):
    b = 0.8
    n = np.arange(4096)
    x = np.sinc(b * (n - 2048 - frac)).astype(complex)
    pslr, islr, irw = metrics.cut_metrics_1d(x)
    assert pslr == pytest.approx(-13.26, abs=0.05)
    assert irw == pytest.approx(0.8859 / b, abs=0.01)
    assert islr == pytest.approx(_sinc_islr(b), abs=0.1)


def test_lfm_compression_is_sinc_like():
    # unweighted LFM (b = 0.8, L = 1024, TBP 819): compressed pulse has the
    # sinc's PSLR and width to within 0.1 dB / 0.02 samples
    n, L = 4096, 1024
    h = scenes.range_replica_padded(n, L)
    H = oracle.matched_filter(h, n)
    x = np.zeros((1, n), complex)
    x[0, 1500:1500 + L] = h[:L]
    y = oracle.compress(x, H)[0]
    pslr, islr, irw = metrics.cut_metrics_1d(y)
    assert pslr == pytest.approx(-13.26, abs=0.1)
    assert irw == pytest.approx(0.8859 / 0.8, abs=0.02)
    assert islr == pytest.approx(_sinc_islr(0.8), abs=0.3)


@pytest.mark.slow
def test_point_target_and_processed_snr():
    # one target, 2048 x 2048 frame; processed SNR = 20 dB + 10 log10(L A)
    sc = scenes.sar_scene(seed=3, n=2048, ranges=(512,), azimuths=(1024,))
    Hr = oracle.matched_filter(sc.range_replica, 2048)
    Ha = oracle.matched_filter(sc.azimuth_replica, 2048)
    img = oracle.sar_image(sc.echo, Hr, Ha)
    m = metrics.point_target(img, 512, 1024, noise_patch=(1400, 100))
    assert m["peak_rc"] == (512, 1024)
    for ax in ("range", "azimuth"):
        assert m["pslr_" + ax] == pytest.approx(-13.26, abs=0.15)
        assert m["irw_" + ax] == pytest.approx(0.8859 / 0.8, abs=0.03)
    expect_snr = 20 + 10 * np.log10(1024) + 10 * np.log10(512)
    assert m["snr"] == pytest.approx(expect_snr, abs=0.3)
