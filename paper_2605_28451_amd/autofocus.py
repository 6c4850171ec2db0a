"""Entropy autofocus on the differentiable azimuth-compression chain.

``AzimuthFocus`` and ``ImageEntropy`` are torch.autograd.Functions whose
forward and backward passes are the HIP kernels of libbfpfft.so (the
adjoint of the azimuth chain is the same block-floating-point chain with the
conjugated filter).  ``entropy_and_grad`` is the fused path used in the
optimisation loop: the phasor table, the forward compression with its
entropy sums and their total, and, on the same phasor table, the fused
entropy gradient + adjoint + per-pulse partial rows and their fixed-order
sum: five kernel launches.
"""
import ctypes

import torch

from . import _lib
from ._lib import FLAG_AUTOFOCUS, check
from .api import FFTPlan, _check_storage, _ptr, _stream


def image_entropy_noalloc(img, stats=None, stream=None):
    """(S, Q, E) of an FP32 image with no plan and no device allocation by the
    library (its partial sums live in a library-owned device array; calls on
    one GPU must not overlap).  `stats`: 3 float64 on the device, or None."""
    count = img.numel() // 2
    _check_storage(img, "fp32", count, "image")
    if stats is None:
        stats = torch.empty(3, dtype=torch.float64, device=img.device)
    check(_lib.load().sar_image_entropy_noalloc(_ptr(img), count, _ptr(stats), _stream(stream)),
          "sar_image_entropy_noalloc")
    return stats


class AutofocusPlan(FFTPlan):
    """Azimuth plan (n = pulses, batch = range bins) with the autofocus workspace."""

    def __init__(self, n_az: int, n_range: int, precision="fp16_fp32", flags: int = 0):
        super().__init__(n_az, n_range, precision, flags | FLAG_AUTOFOCUS)

    def image(self, rc_t, h_az, phase, out=None, stream=None):
        return self.azimuth_compress(rc_t, h_az, out=out, phase=phase, out_fp32=True, stream=stream)

    def entropy_stats(self, img, stats=None, stream=None):
        count = img.numel() // 2
        _check_storage(img, "fp32", count, "image")
        if stats is None:
            stats = torch.empty(3, dtype=torch.float64, device=img.device)
        check(_lib.load().sar_image_entropy(self._h, _ptr(img), count, _ptr(stats), _stream(stream)),
              "sar_image_entropy")
        return stats

    def image_and_entropy(self, rc_t, h_az, phase, out=None, stats=None, stream=None):
        """The image (FP32) and its entropy stats (S, Q, E) in one pass."""
        rows = rc_t.numel() // (2 * self.n)
        _check_storage(rc_t, self.fmt, rows * self.n, "rc_t")
        _check_storage(h_az, self.filter_fmt, self.n, "filter")
        if out is None:
            out = torch.empty((rows, self.n, 2), dtype=torch.float32, device=rc_t.device)
        _check_storage(out, "fp32", rows * self.n, "image")
        if stats is None:
            stats = torch.empty(3, dtype=torch.float64, device=rc_t.device)
        if phase is not None and (phase.dtype != torch.float32 or phase.numel() != self.n
                                  or not phase.is_cuda):
            raise ValueError("phase: n_az float32 device values")
        check(_lib.load().sar_azimuth_image_entropy(self._h, _ptr(rc_t), _ptr(out), _ptr(h_az),
                                                    _ptr(phase), rows, _ptr(stats),
                                                    _stream(stream)), "sar_azimuth_image_entropy")
        return out, stats

    def entropy_grad(self, img, stats, scale=None, out=None, stream=None):
        count = img.numel() // 2
        if out is None:
            out = torch.empty_like(img)
        check(_lib.load().sar_entropy_grad(_ptr(img), _ptr(stats), _ptr(scale), _ptr(out), count,
                                           _stream(stream)), "sar_entropy_grad")
        return out

    def phase_grad(self, rc_t, g, h_az, phase, stats=None, out=None, stream=None):
        """dL/dphase from dL/dI (stats None) or, fused, from the image and its
        entropy stats (L = entropy).  phase None: the plan's phasor table as
        the last call with a phase vector (image_and_entropy, image) left it."""
        rows = rc_t.numel() // (2 * self.n)
        _check_storage(rc_t, self.fmt, rows * self.n, "rc_t")
        _check_storage(g, "fp32", rows * self.n, "gradient/image")
        _check_storage(h_az, self.filter_fmt, self.n, "filter")
        if out is None:
            out = torch.empty(self.n, dtype=torch.float32, device=rc_t.device)
        check(_lib.load().sar_azimuth_phase_grad(self._h, _ptr(rc_t), _ptr(g), _ptr(stats),
                                                 _ptr(h_az), _ptr(phase), _ptr(out), rows,
                                                 _stream(stream)), "sar_azimuth_phase_grad")
        return out


class AzimuthFocus(torch.autograd.Function):
    """I = A_az(rc_t . exp(i phase)) as FP32 pairs; gradient w.r.t. phase."""

    @staticmethod
    def forward(ctx, phase, plan, rc_t, h_az):
        img = plan.image(rc_t, h_az, phase.detach().contiguous())
        ctx.save_for_backward(phase)
        ctx.plan, ctx.rc_t, ctx.h_az = plan, rc_t, h_az
        return img

    @staticmethod
    def backward(ctx, grad_img):
        (phase,) = ctx.saved_tensors
        g = ctx.plan.phase_grad(ctx.rc_t, grad_img.contiguous(), ctx.h_az, phase.detach().contiguous())
        return g, None, None, None


class ImageEntropy(torch.autograd.Function):
    """E = -sum p ln p of an FP32-pair image; returns a 0-d float64 tensor."""

    @staticmethod
    def forward(ctx, img, plan):
        stats = plan.entropy_stats(img)
        ctx.save_for_backward(img, stats)
        ctx.plan = plan
        return stats[2].clone()

    @staticmethod
    def backward(ctx, gE):
        img, stats = ctx.saved_tensors
        scale = gE.detach().reshape(1).to(torch.float32).contiguous()
        return ctx.plan.entropy_grad(img, stats, scale=scale), None


def entropy_and_grad(plan, rc_t, h_az, phase, img=None, stats=None, grad=None):
    """Fused path: (E as a device float64 scalar tensor, dE/dphase)."""
    img, stats = plan.image_and_entropy(rc_t, h_az, phase, out=img, stats=stats)
    grad = plan.phase_grad(rc_t, img, h_az, None, stats=stats, out=grad)  # the same phasor table
    return stats[2], grad, img


def cosine_schedule(steps: int, lr_max: float = 2.5, lr_min: float = 0.02):
    """lr_k = lr_min + (lr_max - lr_min) (1 + cos(pi (k - 1) / steps)) / 2, k = 1..steps:
    large steps first (a phase error of several radians across the
    aperture), small ones at the end."""
    import math
    return [lr_min + (lr_max - lr_min) * 0.5 * (1.0 + math.cos(math.pi * (k - 1) / steps))
            for k in range(1, steps + 1)]


class PhaseAdam:
    """Adam on a device phase vector (Kingma & Ba, 2015), moments and step
    count on the device (the library's sar_autofocus_adam), so the update
    needs no host round trip and can be captured in a graph."""

    def __init__(self, phase, lr=0.3, betas=(0.9, 0.999), eps=1e-8, lr_schedule=None):
        if phase.dtype != torch.float32 or not phase.is_cuda or not phase.is_contiguous():
            raise ValueError("phase: contiguous float32 device tensor")
        self.phase = phase
        self.lr, self.betas, self.eps = float(lr), (float(betas[0]), float(betas[1])), float(eps)
        self.schedule = None
        if lr_schedule is not None:
            # step k uses lr_schedule[min(k, len) - 1], read on the device
            self.schedule = torch.as_tensor(lr_schedule, dtype=torch.float32).to(phase.device).contiguous()
        self.m = torch.zeros_like(phase)
        self.v = torch.zeros_like(phase)
        self.count = torch.zeros(1, dtype=torch.int32, device=phase.device)

    def step(self, grad, stream=None):
        if grad.dtype != torch.float32 or grad.numel() != self.phase.numel() or not grad.is_cuda:
            raise ValueError("grad: float32 device tensor of the phase's size")
        lib = _lib.load()
        if self.schedule is not None:
            check(lib.sar_autofocus_adam_schedule(_ptr(self.phase), _ptr(grad), _ptr(self.m), _ptr(self.v),
                                                  _ptr(self.count), self.phase.numel(), _ptr(self.schedule),
                                                  self.schedule.numel(), self.betas[0], self.betas[1],
                                                  self.eps, _stream(stream)), "sar_autofocus_adam_schedule")
        else:
            check(lib.sar_autofocus_adam(_ptr(self.phase), _ptr(grad), _ptr(self.m), _ptr(self.v),
                                         _ptr(self.count), self.phase.numel(), self.lr,
                                         self.betas[0], self.betas[1], self.eps, _stream(stream)),
                  "sar_autofocus_adam")


class AutofocusLoop:
    """Entropy autofocus by Adam: one iteration is the image and its entropy,
    the fused phase gradient and the Adam step, all library kernels on the
    current stream.  Each step() runs `iterations_per_step` iterations; with
    graph=True they are captured once in a HIP graph (buffers preallocated
    here) and each step() replays it.  A replay carries a fixed cost on the
    device, so several iterations per replay run faster; the results are the
    same bits either way."""

    def __init__(self, plan, rc_t, h_az, phase, lr=0.3, graph=True, lr_schedule=None,
                 iterations_per_step=1):
        n = plan.n
        rows = rc_t.numel() // (2 * n)
        if int(iterations_per_step) < 1:
            raise ValueError("iterations_per_step must be >= 1")
        self.k = int(iterations_per_step)
        self.plan, self.rc_t, self.h_az, self.phase = plan, rc_t, h_az, phase
        self.opt = PhaseAdam(phase, lr=lr, lr_schedule=lr_schedule)
        self.img = torch.empty((rows, n, 2), dtype=torch.float32, device=rc_t.device)
        self.stats = torch.empty(3, dtype=torch.float64, device=rc_t.device)
        self.grad = torch.empty(n, dtype=torch.float32, device=rc_t.device)
        self.graph = None
        if graph:
            # one uncaptured pass of every kernel of the iteration on a side
            # stream (its outputs are overwritten by every replay; the Adam
            # launch goes to a throwaway state, so the optimiser's own state
            # is untouched), then the capture of one iteration
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(s):
                entropy_and_grad(plan, rc_t, h_az, phase, img=self.img, stats=self.stats,
                                 grad=self.grad)
                PhaseAdam(torch.zeros_like(phase), lr=lr, lr_schedule=lr_schedule).step(self.grad)
                s.synchronize()
                with torch.cuda.graph(g, stream=s):
                    for _ in range(self.k):
                        self._iteration()
            torch.cuda.current_stream().wait_stream(s)
            self.graph = g

    def _iteration(self):
        entropy_and_grad(self.plan, self.rc_t, self.h_az, self.phase, img=self.img, stats=self.stats,
                         grad=self.grad)
        self.opt.step(self.grad)

    def step(self):
        """iterations_per_step iterations; afterwards img and stats hold the
        image and entropy at the phase before the last update."""
        if self.graph is not None:
            self.graph.replay()
        else:
            for _ in range(self.k):
                self._iteration()

    def entropy(self):
        """Entropy of the image at the current phase (runs the forward pass)."""
        self.plan.image_and_entropy(self.rc_t, self.h_az, self.phase, out=self.img, stats=self.stats)
        return self.stats[2]
