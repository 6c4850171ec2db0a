"""HIP-graph capture of the SAR frame and of the uneven persistent launch.

Each graph is replayed several times with eager work and synchronisations in
between, and every replay is compared bitwise with the eager result.  None of
the captured calls records a memset (the uneven launch clears its work
counter with a kernel)."""
import numpy as np
import pytest
import torch

from paper_2605_28451_amd import api, scenes
from tests.gpu_util import announce, need_gpu, upload

pytestmark = pytest.mark.gpu


def _capture(fn):
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("mode", ["fp16", "fp16_mul_fp32_acc"])
def test_sar_frame_graph_replays_match_eager(mode):
    need_gpu()
    announce(f"graph SAR frame mode={mode}")
    fmt = api.storage_format(mode)
    n = 4096 if mode == "fp16_mul_fp32_acc" else 1024
    sc = scenes.sar_scene(seed=3, n=n, length=256, aperture=128, ranges=(300,), azimuths=(n // 2,))
    echo = upload(scenes.quantize(sc.echo, fmt), fmt)
    rp = api.FFTPlan(n, n, mode)
    ap = api.FFTPlan(n, n, mode)
    Hr = api.filter_tensor(sc.range_replica, n, mode)
    Ha = api.filter_tensor(sc.azimuth_replica, n, mode)
    rc, rct, img = (torch.empty_like(echo) for _ in range(3))

    def frame():
        rp.range_compress(echo, Hr, out=rc)
        api.corner_turn(rc, fmt, out=rct)
        ap.azimuth_compress(rct, Ha, out=img)

    frame()
    torch.cuda.synchronize()
    eager = img.clone()
    g = _capture(frame)
    for k in range(3):
        img.zero_()
        rc.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(img, eager), f"replay {k}"
        frame()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(img, eager)


def test_uneven_graph_replays_match_eager():
    need_gpu()
    announce("graph uneven 2000 transforms")
    ub = scenes.uneven_batch(seed=4, count=2000)
    x = upload(scenes.quantize(ub.x, "fp16"), "fp16")
    plan = api.UnevenPlan(ub.log2n, ub.inverse, "fp16")
    out = torch.empty_like(x)
    plan.execute(x, out=out)
    torch.cuda.synchronize()
    eager = out.clone()
    g = _capture(lambda: plan.execute(x, out=out))
    for k in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {k}"
        plan.execute(x, out=out)
        torch.cuda.synchronize()


def test_concurrent_frames_on_two_streams_match_eager():
    # independent frames dealt to two streams forked and joined inside one
    # graph (the benchmark's concurrent frames); the plans are shared, which
    # the compression calls without a phase vector allow
    need_gpu()
    announce("graph: two SAR frames on two streams")
    mode, fmt, n = "fp16", "fp16", 1024
    sc = scenes.sar_scene(seed=3, n=n, length=256, aperture=128, ranges=(300,), azimuths=(n // 2,))
    echo0 = upload(scenes.quantize(sc.echo, fmt), fmt)
    echoes = [echo0, torch.flip(echo0, dims=[0]).contiguous()]
    rp = api.FFTPlan(n, n, mode)
    ap = api.FFTPlan(n, n, mode)
    Hr = api.filter_tensor(sc.range_replica, n, mode)
    Ha = api.filter_tensor(sc.azimuth_replica, n, mode)
    bufs = [[torch.empty_like(echo0) for _ in range(3)] for _ in range(2)]

    def frame(i):
        rc, rct, img = bufs[i]
        rp.range_compress(echoes[i], Hr, out=rc)
        api.corner_turn(rc, fmt, out=rct)
        ap.azimuth_compress(rct, Ha, out=img)

    for i in range(2):
        frame(i)
    torch.cuda.synchronize()
    eager = [bufs[i][2].clone() for i in range(2)]
    assert not torch.equal(eager[0], eager[1])
    side = torch.cuda.Stream()

    def both():
        main = torch.cuda.current_stream()
        side.wait_stream(main)
        frame(0)
        with torch.cuda.stream(side):
            frame(1)
        main.wait_stream(side)

    g = _capture(both)
    for k in range(3):
        for b in bufs:
            b[2].zero_()
            b[0].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i in range(2):
            assert torch.equal(bufs[i][2], eager[i]), f"replay {k} frame {i}"
        frame(0)  # eager work between replays
        torch.cuda.synchronize()
