"""Uneven persistent batch: parity with the oracle and with per-size launches."""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_28451_amd.metrics import sqnr_db
from paper_2605_28451_amd import api, scenes
from tests.gpu_util import FWD_SQNR_MIN, announce, download, need_gpu, upload

pytestmark = pytest.mark.gpu


def _oracle_uneven(ub, xq):
    ref = np.empty_like(xq)
    for e in range(8, 15):
        for inv in (0, 1):
            idx = np.nonzero((ub.log2n == e) & (ub.inverse == inv))[0]
            if idx.size == 0:
                continue
            n = 1 << e
            rows = np.stack([xq[ub.offsets[i]:ub.offsets[i] + n] for i in idx])
            out = oracle.fft(rows, inverse=bool(inv))
            for k, i in enumerate(idx):
                ref[ub.offsets[i]:ub.offsets[i] + n] = out[k]
    return ref


@pytest.mark.parametrize("mode", ["fp16", "fp16_fp32", "fp32"])
def test_uneven_small_matches_oracle(mode):
    need_gpu()
    announce(f"uneven 300 transforms mode={mode}")
    ub = scenes.uneven_batch(seed=4, count=300)
    fmt = api.storage_format(mode)
    xq = scenes.quantize(ub.x, fmt)
    plan = api.UnevenPlan(ub.log2n, ub.inverse, mode, flags=api.FLAG_CHECK_FINITE)
    assert plan.total == xq.size and np.array_equal(plan.offsets, ub.offsets)
    y = download(plan.execute(upload(xq, fmt)), fmt)
    assert plan.nonfinite() == 0
    ref = _oracle_uneven(ub, xq)
    for e in range(8, 15):
        for inv in (0, 1):
            idx = np.nonzero((ub.log2n == e) & (ub.inverse == inv))[0]
            if idx.size == 0:
                continue
            sel = np.concatenate([np.arange(ub.offsets[i], ub.offsets[i] + (1 << e)) for i in idx])
            s = sqnr_db(ref[sel], y[sel])
            assert s >= FWD_SQNR_MIN[mode] - 4.0, (e, inv, s)


def test_uneven_full_config_equals_per_size_launches():
    # 20,000 transforms, N log-uniform in 256..16384, random directions:
    # the persistent launch is bitwise identical to per-size row launches
    need_gpu()
    announce("uneven 20000 transforms fp16")
    ub = scenes.uneven_batch(seed=4, count=20000)
    xq = scenes.quantize(ub.x, "fp16")
    xd = upload(xq, "fp16")
    plan = api.UnevenPlan(ub.log2n, ub.inverse, "fp16")
    y = plan.execute(xd)
    torch.cuda.synchronize()
    yh = y.cpu()
    xh = xd.cpu()
    for e in range(8, 15):
        n = 1 << e
        for inv in (0, 1):
            idx = np.nonzero((ub.log2n == e) & (ub.inverse == inv))[0]
            if idx.size == 0:
                continue
            rows = torch.stack([xh[ub.offsets[i]:ub.offsets[i] + n] for i in idx]).cuda().contiguous()
            p = api.FFTPlan(n, idx.size, "fp16")
            r = (p.inverse_bfp(rows) if inv else p.forward(rows)).cpu()
            got = torch.stack([yh[ub.offsets[i]:ub.offsets[i] + n] for i in idx])
            assert torch.equal(got, r), (e, inv)
    # sampled parity with the oracle at full size
    rng = np.random.default_rng(0)
    pick = rng.choice(20000, 200, replace=False)
    yq = scenes.decode(yh.numpy(), "fp16")
    for i in pick[:50]:
        n = 1 << int(ub.log2n[i])
        seg = xq[ub.offsets[i]:ub.offsets[i] + n]
        ref = oracle.fft(seg[None], inverse=bool(ub.inverse[i]))[0]
        assert sqnr_db(ref, yq[ub.offsets[i]:ub.offsets[i] + n]) >= 50.0


def test_uneven_empty_and_single():
    need_gpu()
    p0 = api.UnevenPlan(np.zeros(0, np.int32), np.zeros(0, np.uint8), "fp16")
    assert p0.total == 0
    x = scenes.quantize(scenes.gaussian_rows(9, 1, 16384)[0], "fp16")
    p1 = api.UnevenPlan([14], [0], "fp16")
    y = download(p1.execute(upload(x, "fp16")), "fp16")
    assert sqnr_db(oracle.fft(x[None])[0], y) >= 52.0
    with pytest.raises(api._lib.BfpError):
        api.UnevenPlan([7], [0], "fp16")
