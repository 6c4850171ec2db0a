"""Parity of the fused SAR kernels with the FP64 oracle (GPU tier)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_28451_amd import metrics
from paper_2605_28451_amd.metrics import sqnr_db
from paper_2605_28451_amd import _lib, api, scenes
from tests.gpu_util import announce, download, need_gpu, upload

pytestmark = pytest.mark.gpu

# unaligned compression SQNR bars (dB), about 3 dB under the lowest value
# measured over N = 256..16384 (FP32 134.4, pure FP16 56.8, FP16 storage
# 65.6, FP16 multiply 63.5; E4M3 38.8 and E5M2 29.8 on the range scene)
RC_SQNR_MIN = {"fp32": 131.0, "fp16": 53.8, "fp16_fp32": 62.5, "fp16_mul_fp32_acc": 60.5,
               "e4m3": 35.5, "e5m2": 26.5}


@pytest.mark.parametrize("mode", ["fp32", "fp16", "fp16_fp32", "fp16_mul_fp32_acc", "e4m3", "e5m2"])
def test_range_compression_matches_oracle(mode):
    # range-compression scene (5 LFM targets, 20 dB noise), 256 of its pulses
    need_gpu()
    announce(f"range compression 256x4096 mode={mode}")
    sc = scenes.range_scene(seed=2, n_pulses=256)
    fmt = api.storage_format(mode)
    ffmt = api.filter_format(mode)
    echo = scenes.quantize(sc.echo, fmt)
    H = scenes.quantize(oracle.matched_filter(sc.replica, 4096), ffmt)
    ref = oracle.compress(echo, H)
    plan = api.FFTPlan(4096, 256, mode, flags=api.FLAG_CHECK_FINITE)
    Hd = api.filter_tensor(sc.replica, 4096, mode)
    rc = download(plan.range_compress(upload(echo, fmt), Hd), fmt)
    assert plan.nonfinite() == 0
    s = sqnr_db(ref, rc)
    print(f"[measure] range_compression.{mode} {s:.3f}")
    assert s >= RC_SQNR_MIN[mode]
    # peaks at the target delays
    for d in sc.delays:
        assert np.argmax(np.abs(rc[0, max(d - 3, 0):d + 4])) + max(d - 3, 0) == d


def test_headline_compression_full_size_every_row():
    # the benchmark's workload and launch: 2048 pulses x 4096, pure FP16, the
    # plan's default grid (the pipelined persistent kernel); every row
    # against the oracle, unaligned (the BFP inverse must equal the
    # normalised inverse)
    need_gpu()
    rows, n = 2048, 4096
    announce(f"headline compression {rows}x{n} fp16, default grid, every row")
    sc = scenes.range_scene(seed=2, n_pulses=rows, n=n)
    echo = scenes.quantize(sc.echo, "fp16")
    plan = api.FFTPlan(n, rows, "fp16", flags=api.FLAG_CHECK_FINITE)
    Hd = api.filter_tensor(sc.replica, n, "fp16")
    got = download(plan.range_compress(upload(echo, "fp16"), Hd), "fp16")
    assert plan.nonfinite() == 0
    H = scenes.quantize(oracle.matched_filter(sc.replica, n), "fp16")
    ref = oracle.compress(echo, H)
    per_row = 10.0 * np.log10(np.sum(np.abs(ref) ** 2, 1) / np.sum(np.abs(ref - got) ** 2, 1))
    s = sqnr_db(ref, got)
    print(f"[measure] headline_rows_min {per_row.min():.3f}")
    print(f"[measure] headline_pooled {s:.3f}")
    # measured: worst row 56.5 dB, pooled 57.4 dB
    assert per_row.min() >= 53.5, (int(np.argmin(per_row)), per_row.min())
    assert s >= 55.0


@pytest.mark.parametrize("mode", ["fp32", "fp16", "fp16_fp32", "fp16_mul_fp32_acc"])
@pytest.mark.parametrize("n", [256, 512, 1024, 2048, 4096, 8192, 16384])
def test_compression_and_filtered_inverse_all_sizes(mode, n):
    # fused compression and the filtered BFP inverse at every length, with a
    # ragged batch (not a multiple of the transforms per workgroup); the
    # large lengths read the filter per row in pure FP16, the others hold it
    # in registers
    need_gpu()
    rows = 3 if n <= 1024 else 2
    announce(f"compression + filtered inverse n={n} rows={rows} mode={mode}")
    fmt = api.storage_format(mode)
    ffmt = api.filter_format(mode)
    sc = scenes.range_scene(seed=2, n_pulses=rows, n=n, length=n // 4)
    echo = scenes.quantize(sc.echo, fmt)
    H = scenes.quantize(oracle.matched_filter(sc.replica, n), ffmt)
    plan = api.FFTPlan(n, rows, mode, flags=api.FLAG_CHECK_FINITE)
    Hd = api.filter_tensor(sc.replica, n, mode)
    bar = RC_SQNR_MIN[mode]
    rc = download(plan.range_compress(upload(echo, fmt), Hd), fmt)
    s = sqnr_db(oracle.compress(echo, H), rc)
    print(f"[measure] compression_all_sizes.{mode}.n{n} {s:.3f}")
    assert s >= bar, (n, mode, s)
    # every target is a peak of its neighbourhood (equal amplitudes: no global order)
    for d in sc.delays:
        lo = max(int(d) - 2, 0)
        assert lo + int(np.argmax(np.abs(rc[0, lo:int(d) + 3]))) == d, (n, mode, d)
    # BFP inverse of a spectrum-domain input times the filter: IDFT(z . H)
    g = np.random.default_rng(n + 9).standard_normal((2, rows, n))
    z = scenes.quantize((g[0] + 1j * g[1]) * np.sqrt(n), fmt)
    y = download(plan.inverse_bfp(upload(z, fmt), Hd), fmt)
    si = sqnr_db(oracle.fft(z * H, inverse=True), y)
    print(f"[measure] filtered_inverse_all_sizes.{mode}.n{n} {si:.3f}")
    assert si >= bar, (n, mode, si)
    assert plan.nonfinite() == 0


@pytest.mark.parametrize("mode", ["fp16", "fp16_fp32"])
def test_range_compression_naive_overflows(mode):
    need_gpu()
    sc = scenes.range_scene(seed=2, n_pulses=16)
    fmt = api.storage_format(mode)
    plan = api.FFTPlan(4096, 16, mode, flags=api.FLAG_CHECK_FINITE)
    Hd = api.filter_tensor(sc.replica, 4096, mode)
    rc = download(plan.range_compress(upload(sc.echo, fmt), Hd, naive=True), fmt)
    assert not np.all(np.isfinite(rc))
    assert plan.nonfinite() > 0


def test_filter_matches_oracle_rounding():
    # host FP64 filter (library) vs oracle filter rounded by numpy
    need_gpu()
    sc = scenes.range_scene(seed=2, n_pulses=1)
    H = oracle.matched_filter(sc.replica, 4096)
    for fmt in ("fp16", "fp32"):
        got = scenes.decode(api.make_filter(sc.replica, 4096, fmt), fmt)
        want = scenes.quantize(H, fmt)
        assert np.mean(got == want) > 0.999
        assert np.max(np.abs(got - want)) <= 2 ** -10


@pytest.mark.parametrize("fmt", ["fp16", "fp32", "e4m3"])
def test_corner_turn_exact(fmt):
    need_gpu()
    rng = np.random.default_rng(0)
    # vector form (both dims multiples of the chunk, full and ragged tiles),
    # element form (odd shapes), and a misaligned view (element form)
    for rows, cols in [(4096, 4096), (100, 260), (130, 66), (64, 1), (3, 5)]:
        announce(f"corner turn {rows}x{cols} {fmt}")
        x = scenes.quantize(0.1 * (rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols))), fmt)
        y = download(api.corner_turn(upload(x, fmt), fmt), fmt)
        assert np.array_equal(y, x.T)
    rows, cols = 128, 256
    x = scenes.quantize(rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols)), fmt)
    flat = upload(np.concatenate([np.zeros(1, complex), x.ravel()]), fmt)
    view = flat[1:].view(rows, cols, *flat.shape[1:])
    y = download(api.corner_turn(view, fmt), fmt)
    assert np.array_equal(y, x.T)


@pytest.mark.parametrize("mode,n,rows", [("fp16", 4096, 300), ("fp16", 1024, 77), ("fp16", 4096, 4096),
                                         ("fp32", 4096, 65), ("fp16_mul_fp32_acc", 4096, 40),
                                         ("fp16_fp32", 512, 129), ("e4m3", 2048, 33)])
def test_transposed_store_equals_corner_turn(mode, n, rows):
    # the corner turn fused into the compression's store: bitwise the same
    # as compressing row-major and transposing, for one-workgroup-per-row and
    # persistent grids (the latter with the XCD-aware row order)
    need_gpu()
    announce(f"transposed store mode={mode} n={n} rows={rows}")
    fmt = api.storage_format(mode)
    sc = scenes.range_scene(seed=2, n_pulses=rows, n=n, length=n // 4)
    x = upload(scenes.quantize(sc.echo, fmt), fmt)
    H = api.filter_tensor(sc.replica, n, mode)
    plan = api.FFTPlan(n, rows, mode)
    ref = api.corner_turn(plan.range_compress(x, H), fmt)
    engine, _ = plan.get_tuning()
    for bpc in (0, 1, 3):
        plan.set_tuning(engine, bpc)
        got = plan.range_compress(x, H, transposed=True)
        assert got.shape[:2] == (n, rows)
        assert torch.equal(got, ref), f"blocks_per_cu={bpc}"


def test_transposed_store_rejects_other_variants():
    need_gpu()
    plan = api.FFTPlan(1024, 8, "fp16")
    H = api.filter_tensor(scenes.range_replica_padded(1024, 256), 1024, "fp16")
    x = torch.zeros((8, 1024, 2), dtype=torch.float16, device="cuda")
    for kw in ({"naive": True}, {"out_fp32": True}):
        with pytest.raises(_lib.BfpError):
            plan.range_compress(x, H, transposed=True, **kw)


@pytest.mark.parametrize("src,dst", [("fp32", "fp16"), ("fp32", "e4m3"), ("fp32", "e5m2"),
                                     ("fp16", "e4m3"), ("fp16", "e5m2"), ("e4m3", "fp32"),
                                     ("e5m2", "fp16")])
def test_convert_matches_host_encoder(src, dst):
    need_gpu()
    rng = np.random.default_rng(1)
    v = rng.standard_normal(5000) * 10.0 ** rng.uniform(-6, 5, 5000)
    v[:6] = [np.nan, -np.nan, 1e9, -1e9, np.inf, -np.inf]  # NaN stays NaN; inf saturates in FP8
    x = np.empty(2500, complex)
    with np.errstate(over="ignore", invalid="ignore"):
        x.real = scenes.decode(scenes.encode(v[:2500].astype(complex), src), src).real
        x.imag = scenes.decode(scenes.encode(v[2500:].astype(complex), src), src).real
    with np.errstate(over="ignore", invalid="ignore"):
        want = scenes.encode(x, dst)
    got = api.convert(upload(x, src), src, dst).cpu().numpy()
    # bitwise for every non-NaN value; NaN stays NaN (payload bits may differ)
    dg, dw = scenes.decode(got, dst), scenes.decode(want, dst)
    for part in ("real", "imag"):
        a, b = getattr(dg, part), getattr(dw, part)
        assert np.array_equal(np.isnan(a), np.isnan(b))
    comp_nan = np.stack([np.isnan(dw.real), np.isnan(dw.imag)], -1)
    assert np.array_equal(np.where(comp_nan, 0, got), np.where(comp_nan, 0, want))
    assert comp_nan.any()


def _gpu_frame(sc, mode, phase=None):
    """range compress -> corner turn -> azimuth compress on the GPU."""
    fmt = api.storage_format(mode)
    npul, nr = sc.echo.shape
    rplan = api.FFTPlan(nr, npul, mode, flags=api.FLAG_CHECK_FINITE)
    aplan = api.FFTPlan(npul, nr, mode, flags=api.FLAG_CHECK_FINITE)
    Hr = api.filter_tensor(sc.range_replica, nr, mode)
    Ha = api.filter_tensor(sc.azimuth_replica, npul, mode)
    rc = rplan.range_compress(upload(scenes.quantize(sc.echo, fmt), fmt), Hr)
    rct = api.corner_turn(rc, fmt)
    ph = None if phase is None else torch.tensor(phase, dtype=torch.float32, device="cuda")
    img = aplan.azimuth_compress(rct, Ha, phase=ph)
    out = download(img, fmt)
    assert rplan.nonfinite() == 0 and aplan.nonfinite() == 0
    return out


def _oracle_frame(sc, mode, phase=None):
    fmt = api.storage_format(mode)
    ffmt = api.filter_format(mode)
    Hr = scenes.quantize(oracle.matched_filter(sc.range_replica, sc.echo.shape[1]), ffmt)
    Ha = scenes.quantize(oracle.matched_filter(sc.azimuth_replica, sc.echo.shape[0]), ffmt)
    return oracle.sar_image(scenes.quantize(sc.echo, fmt), Hr, Ha, phi=phase)


# frame SQNR bars (dB), about 3 dB under the measured values (pure FP16 55.4,
# FP16 storage 64.0, FP16 multiply 62.5, FP32 132.7, E4M3 29.3, E5M2 23.8);
# pure FP16 also meets the 40 dB end-to-end bar
FRAME_SQNR_MIN = {"fp16": 52.5, "fp16_fp32": 61.0, "fp16_mul_fp32_acc": 59.5, "fp32": 129.5,
                  "e4m3": 26.5, "e5m2": 21.0}
# (PSLR/ISLR dB, SNR dB, IRW samples) bars of the frame metrics against the
# oracle: the paper's 0.1 dB / 0.02-bin parity for the FP16 and FP32 modes
# (worst measured over the 9 targets: 0.007 dB, 0.0003 samples).  The FP8
# storage modes are the paper's FP8 study (Sec. VII) carried to the image:
# worst measured E4M3 PSLR 0.17 / ISLR 0.10 / SNR 0.23 dB / IRW 0.005, E5M2
# 0.52 / 0.46 / 0.42 dB / 0.021; their bars are 0.5 / 1.0 dB (PSLR, ISLR,
# SNR) and 0.02 / 0.05 samples
FRAME_METRIC_BARS = {"fp16": (0.1, 0.1, 0.02), "fp16_fp32": (0.1, 0.1, 0.02),
                     "fp16_mul_fp32_acc": (0.1, 0.1, 0.02), "fp32": (0.1, 0.1, 0.02),
                     "e4m3": (0.5, 0.5, 0.02), "e5m2": (1.0, 1.0, 0.05)}


@pytest.mark.parametrize("mode", ["fp16", "fp16_fp32", "fp16_mul_fp32_acc", "fp32", "e4m3", "e5m2"])
def test_sar_frame_4096_matches_oracle_metrics(mode):
    # full range-Doppler frame, 4096 x 4096, 3 x 3 point targets
    need_gpu()
    announce(f"SAR frame 4096x4096 mode={mode}")
    sc = scenes.sar_scene(seed=3)
    img = _gpu_frame(sc, mode)
    ref = _oracle_frame(sc, mode)
    s = metrics.sqnr_db(ref, img)
    print(f"[measure] frame_sqnr.{mode} {s:.3f}")
    assert np.all(np.isfinite(img))
    assert s >= FRAME_SQNR_MIN[mode]
    # FP8 storage rounds the echo, the range-compressed data and the image
    # to 3 (E4M3) or 2 (E5M2) mantissa bits; the oracle sees only the rounded
    # echo, so the image metrics move further than in the FP16 modes: their
    # bars are readings of the FP8 floor (PSLR/ISLR, SNR, IRW per mode)
    bar_db, bar_snr, bar_irw = FRAME_METRIC_BARS[mode]
    worst = {}
    for (r0, a0) in sc.targets:
        mg = metrics.point_target(img, r0, a0, noise_patch=(r0 + 300, a0 + 300))
        mo = metrics.point_target(ref, r0, a0, noise_patch=(r0 + 300, a0 + 300))
        assert mg["peak_rc"] == mo["peak_rc"] == (r0, a0)
        for k in ("pslr_range", "pslr_azimuth", "islr_range", "islr_azimuth", "snr",
                  "irw_range", "irw_azimuth"):
            worst[k] = max(worst.get(k, 0.0), abs(mg[k] - mo[k]))
        for k in ("pslr_range", "pslr_azimuth", "islr_range", "islr_azimuth"):
            assert abs(mg[k] - mo[k]) <= bar_db, (r0, a0, k, mg[k], mo[k])
        assert abs(mg["snr"] - mo["snr"]) <= bar_snr, (r0, a0, mg["snr"], mo["snr"])
        for k in ("irw_range", "irw_azimuth"):
            assert abs(mg[k] - mo[k]) <= bar_irw, (r0, a0, k, mg[k], mo[k])
    for k, v in worst.items():
        print(f"[measure] frame_worst_delta.{mode}.{k} {v:.4f}")


def _weighted_frames(sc, mode, taper):
    """GPU frame with filters tapered by the library's bfp_window, and the
    oracle frame with the oracle's own tapers (same scene, same storage)."""
    from oracle import windows as W
    npul, nr = sc.echo.shape
    fmt, ffmt = api.storage_format(mode), api.filter_format(mode)
    if taper == "taylor":
        wl, wa = api.window("taylor", 1024, 5, 40.0), api.window("taylor", 512, 5, 40.0)
        ol, oa = W.taylor(1024, 5, 40.0), W.taylor(512, 5, 40.0)
    else:
        wl, wa = api.window("hamming", 1024), api.window("hamming", 512)
        ol, oa = W.hamming(1024), W.hamming(512)
    rplan = api.FFTPlan(nr, npul, mode, flags=api.FLAG_CHECK_FINITE)
    aplan = api.FFTPlan(npul, nr, mode, flags=api.FLAG_CHECK_FINITE)
    Hr = api.filter_tensor(scenes.weighted_range_replica(nr, wl), nr, mode)
    Ha = api.filter_tensor(scenes.weighted_azimuth_replica(npul, wa), npul, mode)
    rc = rplan.range_compress(upload(scenes.quantize(sc.echo, fmt), fmt), Hr)
    img = download(aplan.azimuth_compress(api.corner_turn(rc, fmt), Ha), fmt)
    assert rplan.nonfinite() == 0 and aplan.nonfinite() == 0
    Hro = scenes.quantize(oracle.matched_filter(scenes.weighted_range_replica(nr, ol), nr), ffmt)
    Hao = scenes.quantize(oracle.matched_filter(scenes.weighted_azimuth_replica(npul, oa), npul), ffmt)
    ref = oracle.sar_image(scenes.quantize(sc.echo, fmt), Hro, Hao)
    return img, ref


# Weighted apertures (Sec. VIII, limitations): with -40 dB Taylor sidelobes
# the modes that accumulate in FP32 keep PSLR/ISLR/SNR within 0.1 dB of the
# FP64 oracle; pure FP16 moves the Taylor PSLR by up to about 0.15 dB
# (measured 0.14 dB), the approach to the FP16 floor the paper anticipates,
# so its PSLR bar here is 0.25 dB (ISLR, SNR and IRW still at 0.1 dB /
# 0.02 samples).
@pytest.mark.parametrize("mode,taper", [("fp32", "taylor"), ("fp16_fp32", "taylor"),
                                        ("fp16_mul_fp32_acc", "taylor"), ("fp16", "taylor"),
                                        ("fp16_mul_fp32_acc", "hamming"), ("fp16", "hamming")])
def test_weighted_frame_4096_matches_oracle_metrics(mode, taper):
    need_gpu()
    announce(f"weighted SAR frame 4096x4096 mode={mode} taper={taper}")
    sc = scenes.sar_scene(seed=3)
    img, ref = _weighted_frames(sc, mode, taper)
    assert np.all(np.isfinite(img))
    pslr_bar = 0.25 if mode == "fp16" else 0.1
    worst = 0.0
    for (r0, a0) in sc.targets:
        mg = metrics.point_target(img, r0, a0, noise_patch=(r0 + 300, a0 + 300))
        mo = metrics.point_target(ref, r0, a0, noise_patch=(r0 + 300, a0 + 300))
        assert mg["peak_rc"] == mo["peak_rc"] == (r0, a0)
        # the taper is in effect: sidelobes near its design level
        assert mo["pslr_range"] < (-39.0 if taper == "taylor" else -42.0)
        for k in ("pslr_range", "pslr_azimuth"):
            worst = max(worst, abs(mg[k] - mo[k]))
            assert abs(mg[k] - mo[k]) <= pslr_bar, (r0, a0, k, mg[k], mo[k])
        for k in ("islr_range", "islr_azimuth", "snr"):
            assert abs(mg[k] - mo[k]) <= 0.1, (r0, a0, k, mg[k], mo[k])
        for k in ("irw_range", "irw_azimuth"):
            assert abs(mg[k] - mo[k]) <= 0.02, (r0, a0, k, mg[k], mo[k])
    print(f"mode={mode} taper={taper} worst PSLR shift {worst:.3f} dB")


def test_azimuth_phase_correction_matches_oracle():
    need_gpu()
    sc = scenes.sar_scene(seed=3, n=1024, length=256, aperture=128, ranges=(300,), azimuths=(512,))
    rng = np.random.default_rng(3)
    phi = rng.uniform(-3, 3, 1024).astype(np.float32).astype(np.float64)
    img = _gpu_frame(sc, "fp16_fp32", phase=phi)
    ref = _oracle_frame(sc, "fp16_fp32", phase=phi)
    s = metrics.sqnr_db(ref, img)
    print(f"[measure] phase_corrected_frame.fp16_fp32 {s:.3f}")
    assert s >= 60.5  # measured 63.7


# ------------------------------------------ range cell migration (RCMC) ----
# measured at N = 4096 / 1024: FP32 130.7 / 131.2, FP16 storage 66.0, FP16
# multiply 64.1 / 64.2, pure FP16 57.2 / 58.1, E4M3 31.5
RCMC_SQNR_MIN = {"fp32": 127.5, "fp16_fp32": 63.0, "fp16_mul_fp32_acc": 61.0, "fp16": 54.0,
                 "e4m3": 28.5, "e5m2": 22.0}


@pytest.mark.parametrize("mode", ["fp32", "fp16_fp32", "fp16_mul_fp32_acc", "fp16", "e4m3"])
@pytest.mark.parametrize("n,rows", [(4096, 48), (1024, 96)])
def test_rcmc_compress_matches_oracle(mode, n, rows):
    # Doppler rows of range data, each compressed and moved by its own
    # fractional shift (negative, zero and beyond the migration range)
    need_gpu()
    announce(f"rcmc compress mode={mode} n={n}")
    fmt = api.storage_format(mode)
    rng = np.random.default_rng(12)
    scale = 0.125 if mode in ("e4m3", "e5m2") else 1.0
    x = scenes.quantize(scale * scenes.gaussian_rows(13, rows, n), fmt)
    shift = np.concatenate([[0.0, 3.0, -5.5], rng.uniform(-12.0, 12.0, rows - 3)]).astype(np.float32)
    h = scenes.range_replica_padded(n, n // 4)
    Hq = scenes.quantize(oracle.matched_filter(h, n), api.filter_format(mode))
    plan = api.FFTPlan(n, rows, mode, flags=api.FLAG_CHECK_FINITE)
    y = plan.range_compress_rcmc(upload(x, fmt), api.filter_tensor(h, n, mode),
                                 torch.tensor(shift, device="cuda"))
    got = download(y, fmt)
    ref = oracle.rcmc_compress(x, Hq, shift.astype(np.float64))
    s = metrics.sqnr_db(ref, got)
    print(f"[measure] rcmc_compress.{mode}.n{n} {s:.3f}")
    assert plan.nonfinite() == 0
    assert s >= RCMC_SQNR_MIN[mode]


def _gpu_rcmc_frame(sc, mode):
    """azimuth FFT -> corner turn -> migration-corrected range compression
    per Doppler bin -> corner turn -> azimuth BFP inverse with H_a."""
    fmt = api.storage_format(mode)
    npul, nr = sc.echo.shape
    aplan = api.FFTPlan(npul, nr, mode, flags=api.FLAG_CHECK_FINITE)
    rplan = api.FFTPlan(nr, npul, mode, flags=api.FLAG_CHECK_FINITE)
    echo = upload(scenes.quantize(sc.echo, fmt), fmt)
    spec = aplan.forward(api.corner_turn(echo, fmt))              # [range][Doppler]
    rd = api.corner_turn(spec, fmt)                               # [Doppler][range]
    shift = torch.tensor(sc.rcmc_shift.astype(np.float32), device="cuda")
    rc = rplan.range_compress_rcmc(rd, api.filter_tensor(sc.range_replica, nr, mode), shift)
    img = aplan.inverse_bfp(api.corner_turn(rc, fmt), api.filter_tensor(sc.azimuth_replica, npul, mode))
    out = download(img, fmt)
    assert rplan.nonfinite() == 0 and aplan.nonfinite() == 0
    return out


@pytest.mark.parametrize("mode", ["fp32", "fp16_fp32", "fp16"])
def test_rcmc_frame_4096_matches_oracle_metrics(mode):
    need_gpu()
    announce(f"RCMC frame 4096x4096 mode={mode}")
    sc = scenes.migration_scene()
    img = _gpu_rcmc_frame(sc, mode)
    fmt, ffmt = api.storage_format(mode), api.filter_format(mode)
    Hr = scenes.quantize(oracle.matched_filter(sc.range_replica, 4096), ffmt)
    Ha = scenes.quantize(oracle.matched_filter(sc.azimuth_replica, 4096), ffmt)
    ref = oracle.rda_rcmc_image(scenes.quantize(sc.echo, fmt), Hr, Ha,
                                sc.rcmc_shift.astype(np.float32).astype(np.float64))
    s = metrics.sqnr_db(ref, img)
    print(f"[measure] rcmc_frame_sqnr.{mode} {s:.3f}")
    assert np.all(np.isfinite(img))
    assert s >= FRAME_SQNR_MIN[mode]
    for (r0, a0) in sc.targets:
        mg = metrics.point_target(img, r0, a0, noise_patch=(r0 + 300, a0 + 300))
        mo = metrics.point_target(ref, r0, a0, noise_patch=(r0 + 300, a0 + 300))
        assert mg["peak_rc"] == mo["peak_rc"] == (r0, a0)
        for k in ("pslr_range", "pslr_azimuth", "islr_range", "islr_azimuth", "snr"):
            assert abs(mg[k] - mo[k]) <= 0.1, (r0, a0, k, mg[k], mo[k])
        for k in ("irw_range", "irw_azimuth"):
            assert abs(mg[k] - mo[k]) <= 0.02, (r0, a0, k, mg[k], mo[k])
