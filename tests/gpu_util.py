"""Shared helpers for the GPU tiers (imported only by tests)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_28451_amd.metrics import sqnr_db
from paper_2605_28451_amd import api, scenes

MODES = ["fp32", "fp16", "fp16_fp32", "fp16_mul_fp32_acc", "e4m3", "e5m2"]
FP16_MODES = ["fp16", "fp16_fp32", "fp16_mul_fp32_acc"]

# minimum forward-FFT SQNR (dB) vs the FP64 oracle on the storage-rounded
# input, N = 4096, complex N(0,1) rows, about 3 dB under the measured values
# (FP32 138.3, pure FP16 60.5, FP16 storage / FP32 compute 68.9, FP16
# multiply / FP32 accumulate 67.5, E4M3 31.5, E5M2 25.6).  Pure FP16 also
# meets the paper's 55 dB; FP16 storage with FP32 arithmetic rounds only at
# the LDS exchanges and the output; FP32 is the same-GPU reference path.
FWD_SQNR_MIN = {"fp32": 135.0, "fp16": 57.5, "fp16_fp32": 66.0, "fp16_mul_fp32_acc": 64.5,
                "e4m3": 28.5, "e5m2": 22.5}
# round trip (forward, then BFP inverse): measured FP32 134.9, FP16 57.6,
# FP16 storage 66.4, FP16 multiply 64.7, E4M3 31.9, E5M2 25.9
ROUNDTRIP_SQNR_MIN = {"fp32": 131.5, "fp16": 54.5, "fp16_fp32": 63.0, "fp16_mul_fp32_acc": 61.5,
                      "e4m3": 28.5, "e5m2": 22.5}


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if api.device_count() < 1:
        pytest.fail("GPU visible but no gfx950 device: the HIP path cannot run")


def upload(x, fmt):
    return api.to_device(x, fmt)


def download(t, fmt):
    torch.cuda.synchronize()
    return api.to_host(t, fmt)


def rand_rows(rows, n, seed, scale=1.0):
    return scale * scenes.gaussian_rows(seed, rows, n)


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
