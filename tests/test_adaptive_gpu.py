"""Adaptive block shift (per-row exponents, the future work of Sec. VIII)
on the GPU against the FP64 oracle.

The stored rows times 2^row_exp must equal the exact result (SQNR bars as
for the fixed schedule) at every input scale, including scales at which the
fixed shift 2^-log2N pushes the inverse into the FP16 subnormals; each row's
exponent equals the oracle's rule on the exact inverse input, up to one step
where the GPU's rounded maximum sits at a power of two."""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_28451_amd import _lib, api, scenes
from paper_2605_28451_amd.metrics import sqnr_db
from tests.gpu_util import FP16_MODES, announce, download, need_gpu, rand_rows, upload

pytestmark = pytest.mark.gpu

# the fixed schedule's inverse bars (pure FP16: the paper's 55 dB less the
# filter product's rounding)
ADAPT_SQNR_MIN = {"fp16": 54.0, "fp16_fp32": 60.0, "fp16_mul_fp32_acc": 58.0}


def _chirp_filter(n, mode):
    h = scenes.range_replica_padded(n, n // 4)
    H = oracle.matched_filter(h, n)
    return scenes.quantize(H, api.filter_format(mode)), api.filter_tensor(h, n, mode)


@pytest.mark.parametrize("mode", FP16_MODES)
@pytest.mark.parametrize("n,rows", [(4096, 64), (1024, 64)])
@pytest.mark.parametrize("log2_scale", [-10, 0, 5])
def test_adaptive_inverse_matches_oracle(mode, n, rows, log2_scale):
    need_gpu()
    announce(f"adaptive inverse mode={mode} n={n} scale=2^{log2_scale}")
    fmt = api.storage_format(mode)
    z = scenes.quantize(rand_rows(rows, n, 11, 2.0 ** log2_scale), fmt)
    Hq, Ht = _chirp_filter(n, mode)
    plan = api.FFTPlan(n, rows, mode)
    zd = upload(z, fmt)
    y, e = plan.inverse_bfp_adaptive(zd, Ht)
    ex = e.cpu().numpy().astype(np.int64)
    got = download(y, fmt) * np.ldexp(1.0, ex)[:, None]
    ref = oracle.fft(z * Hq[None], inverse=True)
    s = sqnr_db(ref, got)
    want = oracle.adaptive_exponent(z * Hq[None], n)
    fixed = sqnr_db(ref, download(plan.inverse_bfp(zd, Ht), fmt))
    print(f"mode={mode} n={n} scale=2^{log2_scale}: adaptive {s:.2f} dB, fixed {fixed:.2f} dB, "
          f"exponents {ex.min()}..{ex.max()}")
    assert np.all(np.isfinite(got))
    assert np.max(np.abs(ex - want)) <= 1
    assert s >= ADAPT_SQNR_MIN[mode]
    if log2_scale == -10 and mode == "fp16":
        assert s >= fixed + 10.0  # the fixed shift has reached the subnormals


@pytest.mark.parametrize("mode", FP16_MODES)
@pytest.mark.parametrize("log2_scale", [-12, -16, 0])
def test_adaptive_compression_matches_oracle(mode, log2_scale):
    # weak echoes: at 2^-12 (peak echo 1e-3) the fixed schedule's pure FP16
    # compression falls to about 42 dB and at 2^-16 (inputs already
    # subnormal) to about 19 dB; the adaptive shift keeps about 57 dB
    need_gpu()
    announce(f"adaptive compression mode={mode} scale=2^{log2_scale}")
    fmt = api.storage_format(mode)
    sc = scenes.range_scene(seed=2, n_pulses=128)
    echo = scenes.quantize(sc.echo * 2.0 ** log2_scale, fmt)
    plan = api.FFTPlan(4096, 128, mode)
    Ht = api.filter_tensor(sc.replica, 4096, mode)
    Hq = scenes.quantize(oracle.matched_filter(sc.replica, 4096), api.filter_format(mode))
    ed = upload(echo, fmt)
    y, e = plan.range_compress_adaptive(ed, Ht)
    ex = e.cpu().numpy().astype(np.int64)
    got = download(y, fmt) * np.ldexp(1.0, ex)[:, None]
    ref = oracle.compress(echo, Hq)
    s = sqnr_db(ref, got)
    fixed = sqnr_db(ref, download(plan.range_compress(ed, Ht), fmt))
    want = oracle.adaptive_exponent(oracle.fft(echo) * Hq[None], 4096)
    print(f"mode={mode} scale=2^{log2_scale}: adaptive {s:.2f} dB, fixed {fixed:.2f} dB, "
          f"exponents {ex.min()}..{ex.max()}")
    assert np.max(np.abs(ex - want)) <= 1
    assert s >= ADAPT_SQNR_MIN[mode] - 3.0  # two transforms and the filter product
    if log2_scale == -12 and mode == "fp16":
        assert s >= fixed + 10.0


def test_adaptive_pipelined_kernel_bitwise_equal():
    # the persistent pipelined grid and one workgroup per row give the same
    # rows and exponents
    need_gpu()
    sc = scenes.range_scene(seed=2, n_pulses=257)
    ed = upload(scenes.quantize(sc.echo * 2.0 ** -6, "fp16"), "fp16")
    Ht = api.filter_tensor(sc.replica, 4096, "fp16")
    plan = api.FFTPlan(4096, 257, "fp16")
    res = []
    for bpc in (0, 1, 3):
        plan.set_tuning(1, bpc)
        y, e = plan.range_compress_adaptive(ed, Ht)
        torch.cuda.synchronize()
        res.append((y.clone(), e.clone()))
    for y, e in res[1:]:
        assert torch.equal(y, res[0][0]) and torch.equal(e, res[0][1])


def test_adaptive_rejections():
    need_gpu()
    p32 = api.FFTPlan(1024, 4, "fp32")
    z = upload(scenes.quantize(rand_rows(4, 1024, 3), "fp32"), "fp32")
    with pytest.raises(_lib.BfpError):
        p32.inverse_bfp_adaptive(z)
    p16 = api.FFTPlan(1024, 4, "fp16")
    z16 = upload(scenes.quantize(rand_rows(4, 1024, 3), "fp16"), "fp16")
    lib = _lib.load()
    out = torch.empty_like(z16)
    assert lib.fft_exec_inv_bfp_adaptive(p16._h, api._ptr(z16), api._ptr(out), None, None, 0,
                                         None) == _lib.EINVAL
    ex = torch.empty(4, dtype=torch.int32, device="cuda")
    assert lib.fft_exec_inv_bfp_adaptive(p16._h, api._ptr(z16), api._ptr(out), None, api._ptr(ex),
                                         api.FLAG_NAIVE_POSTSCALE, None) == _lib.EINVAL
