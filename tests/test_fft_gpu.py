"""Parity of the HIP FFT path with the FP64 oracle (GPU tier).

All calls go through the C ABI (ctypes) of libbfpfft.so.  The oracle runs on
the storage-rounded inputs, so SQNR measures the transform alone (the
primary reading; the paper's own harness compares against the unquantised
draw, which only adds the input rounding).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_28451_amd.metrics import sqnr_db
from paper_2605_28451_amd import api, scenes
from tests.gpu_util import (FP16_MODES, FWD_SQNR_MIN, MODES, ROUNDTRIP_SQNR_MIN, announce, download,
                            need_gpu, rand_rows, upload)

pytestmark = pytest.mark.gpu

SIZES = [256, 512, 1024, 2048, 4096, 8192, 16384]


def _scale(mode):
    return 0.125 if mode in ("e4m3", "e5m2") else 1.0


@pytest.mark.parametrize("mode", MODES)
def test_forward_n4096_sqnr(mode):
    need_gpu()
    announce(f"forward n=4096 rows=64 mode={mode}")
    fmt = api.storage_format(mode)
    x = scenes.quantize(rand_rows(64, 4096, 1, _scale(mode)), fmt)
    plan = api.FFTPlan(4096, 64, mode)
    X = download(plan.forward(upload(x, fmt)), fmt)
    ref = oracle.fft(x)
    s = sqnr_db(ref, X)
    print(f"[measure] forward_n4096.{mode} {s:.3f}")
    assert np.all(np.isfinite(X))
    assert s >= FWD_SQNR_MIN[mode]


@pytest.mark.parametrize("mode", ["fp32", "fp16", "fp16_fp32", "fp16_mul_fp32_acc"])
@pytest.mark.parametrize("n", SIZES)
def test_forward_and_inverse_all_sizes(mode, n):
    need_gpu()
    # ragged batch: not a multiple of the transforms per workgroup
    rows = 3 if n <= 1024 else 2
    announce(f"fwd+inv n={n} rows={rows} mode={mode}")
    fmt = api.storage_format(mode)
    x = scenes.quantize(rand_rows(rows, n, n + 7), fmt)
    plan = api.FFTPlan(n, rows, mode)
    X = download(plan.forward(upload(x, fmt)), fmt)
    s = sqnr_db(oracle.fft(x), X)
    print(f"[measure] forward_all_sizes.{mode}.n{n} {s:.3f}")
    # one more radix pass above 4096 points
    bar = FWD_SQNR_MIN[mode] - (1.5 if n > 4096 else 0.0)
    assert s >= bar, (n, mode, s)
    # BFP inverse of a fresh spectrum-domain input (normalised IDFT)
    z = scenes.quantize(rand_rows(rows, n, n + 8) * np.sqrt(n), fmt)
    y = download(plan.inverse_bfp(upload(z, fmt)), fmt)
    si = sqnr_db(oracle.fft(z, inverse=True), y)
    print(f"[measure] inverse_all_sizes.{mode}.n{n} {si:.3f}")
    assert si >= bar, (n, mode, si)


@pytest.mark.parametrize("mode", MODES)
def test_round_trip_config1(mode):
    # 64 x 4096 N(0,1): forward, then 1/N prescale and inverse
    need_gpu()
    announce(f"round trip n=4096 rows=64 mode={mode}")
    fmt = api.storage_format(mode)
    x = scenes.quantize(rand_rows(64, 4096, 1, _scale(mode)), fmt)
    plan = api.FFTPlan(4096, 64, mode)
    X = plan.forward(upload(x, fmt))
    y = download(plan.inverse_bfp(X), fmt)
    s = sqnr_db(x, y)
    print(f"[measure] round_trip.{mode} {s:.3f}")
    assert s >= ROUNDTRIP_SQNR_MIN[mode]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("n", [256, 4096, 16384])
def test_dc_and_alternating_bit_exact(mode, n):
    # every butterfly-decomposed mode maps DC and (-1)^n exactly
    need_gpu()
    announce(f"dc/alternating n={n} mode={mode}")
    fmt = api.storage_format(mode)
    a = 1.0 / 64 if mode in ("e4m3", "e5m2") else 1.0
    x = np.stack([np.full(n, a, complex), a * (-1.0) ** np.arange(n)])
    plan = api.FFTPlan(n, 2, mode)
    X = download(plan.forward(upload(x, fmt)), fmt)
    e = np.zeros((2, n), complex)
    e[0, 0] = a * n
    e[1, n // 2] = a * n
    assert np.array_equal(X, e)


@pytest.mark.parametrize("mode", FP16_MODES)
def test_prescale_bit_exact_including_subnormals(mode):
    # inverse of c delta[0]: every output equals fp16(c 2^-log2N) bitwise, so
    # the fold of Eq. (1) is exact for normal results and RNE into subnormals
    need_gpu()
    n = 4096
    c = np.array([1.0, 0.5, 3.0e-3, 1.0e-3, 7.0e-4, 2.5e-4, -6.1e-5, 1e-2 + 1e-3j, 40000.0, 3e-7])
    c16 = scenes.quantize(c, "fp16")
    z = np.zeros((c.size, n), complex)
    z[:, 0] = c16
    plan = api.FFTPlan(n, c.size, mode)
    y = download(plan.inverse_bfp(upload(z, "fp16")), "fp16")
    expect_re = (c16.real * 2.0 ** -12).astype(np.float16).astype(np.float64)
    expect_im = (c16.imag * 2.0 ** -12).astype(np.float16).astype(np.float64)
    assert np.array_equal(y.real, np.repeat(expect_re[:, None], n, 1))
    assert np.array_equal(y.imag, np.repeat(expect_im[:, None], n, 1))


def _zadoff_chu(n):
    m = np.arange(n)
    x = np.exp(-1j * np.pi * ((m * m) % (2 * n)) / n)
    X = oracle.fft(x[None])[0]
    return x, np.conj(X) / np.sqrt(n)


@pytest.mark.parametrize("mode", FP16_MODES)
def test_naive_overflows_bfp_does_not(mode):
    # Sec. III-B: without the fold the inverse overflows FP16; with it the
    # output is sqrt(N) delta
    need_gpu()
    n = 4096
    x, H = _zadoff_chu(n)
    X = oracle.fft(x[None])[0]
    fmt = api.storage_format(mode)
    plan = api.FFTPlan(n, 1, mode, flags=api.FLAG_CHECK_FINITE)
    Xd = upload(scenes.quantize(X[None], fmt), fmt)
    Hd = upload(H, api.filter_format(mode))
    y = download(plan.inverse_bfp(Xd, Hd), fmt)[0]
    assert plan.nonfinite() == 0
    assert np.all(np.isfinite(y))
    assert abs(abs(y[0]) - np.sqrt(n)) < 0.1
    assert np.max(np.abs(y[1:])) < 0.1
    yn = download(plan.inverse_bfp(Xd, Hd, naive=True), fmt)[0]
    assert not np.all(np.isfinite(yn))
    assert plan.nonfinite() > 0


def test_fp32_naive_is_finite():
    need_gpu()
    n = 4096
    x, H = _zadoff_chu(n)
    X = oracle.fft(x[None])[0]
    plan = api.FFTPlan(n, 1, "fp32")
    y = download(plan.inverse_bfp(upload(X[None], "fp32"), upload(H, "fp32"), naive=True), "fp32")
    assert np.all(np.isfinite(y))
    assert abs(abs(y[0, 0]) - 64.0) < 1e-3


@pytest.mark.parametrize("mode", ["fp16", "fp32"])
def test_in_place_equals_out_of_place(mode):
    need_gpu()
    fmt = api.storage_format(mode)
    x = scenes.quantize(rand_rows(5, 2048, 3), fmt)
    plan = api.FFTPlan(2048, 5, mode)
    a = upload(x, fmt)
    b = plan.forward(a)
    a2 = upload(x, fmt)
    plan.forward(a2, out=a2)
    torch.cuda.synchronize()
    assert torch.equal(a2, b)
    plan.inverse_bfp(a2, out=a2)
    c = plan.inverse_bfp(b)
    torch.cuda.synchronize()
    assert torch.equal(a2, c)


def test_deterministic_and_empty_batch():
    need_gpu()
    x = scenes.quantize(rand_rows(8, 4096, 5), "fp16")
    plan = api.FFTPlan(4096, 8, "fp16")
    d = upload(x, "fp16")
    assert torch.equal(plan.forward(d), plan.forward(d))
    empty = api.FFTPlan(4096, 0, "fp16")
    e = api.empty((0, 4096), "fp16")
    empty.forward(e)  # no-op, no error
    torch.cuda.synchronize()


def test_invalid_arguments_rejected():
    need_gpu()
    with pytest.raises(api._lib.BfpError):
        api.FFTPlan(1000, 1, "fp16")
    with pytest.raises(api._lib.BfpError):
        api.FFTPlan(4, 1, "fp16")
    with pytest.raises(api._lib.BfpError):
        api.FFTPlan(32768, 1, "fp16")
    with pytest.raises(api._lib.BfpError):
        api.FFTPlan(4096, 1, 9)
