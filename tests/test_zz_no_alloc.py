"""The no-allocation entropy entry point (GPU tier): sar_image_entropy_noalloc
through the C ABI against sar_image_entropy (the plan-based entry point with
the same kernels) and the FP64 oracle, on two calls in a row, the second with
a smaller image, then at the largest grid (1024 workgroups) and the smallest
input, and its argument checks."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2605_28451_amd import _lib, scenes
from paper_2605_28451_amd.autofocus import AutofocusPlan, image_entropy_noalloc
from tests.gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu


def _image(seed, rows, n):
    g = scenes.gaussian_rows(seed, rows, n)
    g[:, : n // 8] *= 30.0  # a few bright columns: entropy well below its maximum
    g[0, :5] = 0.0          # exact zeros: 0 ln 0 = 0
    return g


def _device_fp32(x):
    return torch.from_numpy(np.stack([x.real, x.imag], -1).astype(np.float32)).cuda().contiguous()


def test_noalloc_entropy_equals_plan_entropy_twice():
    need_gpu()
    plan = AutofocusPlan(1024, 64, "fp32")
    for k, (rows, n) in enumerate(((512, 1024), (37, 256))):
        announce(f"no-alloc entropy call {k}: {rows}x{n}")
        x = _image(70 + k, rows, n)
        img = _device_fp32(x)
        got = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
        st = _lib.load().sar_image_entropy_noalloc(ctypes.c_void_p(img.data_ptr()), img.numel() // 2,
                                                   ctypes.c_void_p(got.data_ptr()),
                                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == _lib.OK
        want = plan.entropy_stats(img)
        torch.cuda.synchronize()
        # same kernels, same grid, same fixed-order sums: bitwise equal
        assert torch.equal(got, want), (k, got, want)
        xq = np.stack([x.real, x.imag], -1).astype(np.float32).astype(np.float64)
        e_ref = oracle.entropy(xq[..., 0] + 1j * xq[..., 1])
        assert abs(got[2].item() - e_ref) <= 1e-6 * abs(e_ref), (k, got[2].item(), e_ref)


def test_noalloc_entropy_largest_grid_and_one_value():
    need_gpu()
    announce("no-alloc entropy: 1024-workgroup grid, then one value")
    x = _image(72, 2048, 1024)  # 2^21 values: the 1024-workgroup cap of the scratch
    img = _device_fp32(x)
    plan = AutofocusPlan(1024, 8, "fp32")
    a = image_entropy_noalloc(img)
    b = plan.entropy_stats(img)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    one = _device_fp32(np.array([[3.0 + 4.0j]]))
    s = image_entropy_noalloc(one).cpu().numpy()
    # one value: p = 1, E = 0 up to the FP32 logarithm of |I|^2 (about 1 ulp)
    assert s[0] == 25.0 and abs(s[2]) <= 1e-6


def test_noalloc_entropy_rejects_bad_arguments():
    need_gpu()
    lib = _lib.load()
    img = torch.zeros((4, 2), dtype=torch.float32, device="cuda")
    stats = torch.zeros(3, dtype=torch.float64, device="cuda")
    p, q = ctypes.c_void_p(img.data_ptr()), ctypes.c_void_p(stats.data_ptr())
    assert lib.sar_image_entropy_noalloc(p, 0, q, None) == _lib.EINVAL
    assert lib.sar_image_entropy_noalloc(None, 4, q, None) == _lib.EINVAL
    assert lib.sar_image_entropy_noalloc(p, 4, None, None) == _lib.EINVAL
    assert lib.sar_image_entropy_noalloc(p, (1 << 40) + 1, q, None) == _lib.EINVAL
    assert b"2^40" in lib.bfp_last_error()
