"""torch.autograd.Function wrappers of the ARM, upsampling and synthesis
modules, whose forward and hand-written backward run in the library's HIP
kernels (see cc_arm_fwd_bwd / cc_ups_* / cc_syn_* in include/coolchic.h).

    mods = Modules(mc, H, W)               # workspace state for one shape
    bits = arm_rate(yhat, params, mods)    # total bits of the quantised latents
    zhat = upsample(yhat, params, mods)    # [L, H, W]
    xhat = synthesis(zhat, params, mods)   # [3, H, W]

Tensors are float32 on the GPU; `params` is the full decoder parameter
vector and each module returns the gradient of its own part (zeros
elsewhere).  A module's backward uses the workspace written by its forward, so
each Modules object serves one graph at a time.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib
from ._lib import check, lib
from .encoder import Encoder


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Modules:
    """Workspace (one state slab) for modules of one decoder shape and size."""

    def __init__(self, mc, H: int, W: int, precision: str = "fp32"):
        img = torch.zeros(3, H, W)
        self.enc = Encoder(mc, img, 1.0, 0, precision=precision)
        self.h = self.enc.handle
        self.n_lat, self.n_par = self.enc.n_lat, self.enc.n_par
        self.L, self.H, self.W = mc.L, H, W


def _f32(t):
    return t.detach().to(device="cuda", dtype=torch.float32).contiguous()


class ArmRate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, yhat, params, mods):
        y, p = _f32(yhat), _f32(params)
        need = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
        gy = torch.zeros_like(y) if need else None
        gp = torch.zeros_like(p) if need else None
        bits = C.c_double()
        check(lib().cc_arm_fwd_bwd(mods.h, _p(y), _p(p), C.byref(bits), _p(gy), _p(gp), _stream()))
        ctx.save_for_backward(*( [gy, gp] if need else [] ))
        return torch.tensor(bits.value, dtype=torch.float32, device="cuda")

    @staticmethod
    def backward(ctx, g):
        gy, gp = ctx.saved_tensors
        return g * gy, g * gp, None


class Upsample(torch.autograd.Function):
    @staticmethod
    def forward(ctx, yhat, params, mods):
        y, p = _f32(yhat), _f32(params)
        z = torch.empty(mods.L, mods.H, mods.W, device="cuda", dtype=torch.float32)
        check(lib().cc_ups_fwd(mods.h, _p(y), _p(p), _p(z), _stream()))
        ctx.mods = mods
        ctx.n_par = p.numel()
        return z

    @staticmethod
    def backward(ctx, gz):
        mods = ctx.mods
        gy = torch.empty(mods.n_lat, device="cuda", dtype=torch.float32)
        gp = torch.zeros(ctx.n_par, device="cuda", dtype=torch.float32)
        check(lib().cc_ups_bwd(mods.h, _p(_f32(gz)), _p(gy), _p(gp), _stream()))
        return gy, gp, None


class Synthesis(torch.autograd.Function):
    @staticmethod
    def forward(ctx, zhat, params, mods):
        z, p = _f32(zhat), _f32(params)
        x = torch.empty(3, mods.H, mods.W, device="cuda", dtype=torch.float32)
        check(lib().cc_syn_fwd(mods.h, _p(z), _p(p), _p(x), _stream()))
        ctx.mods = mods
        ctx.n_par = p.numel()
        return x

    @staticmethod
    def backward(ctx, gx):
        mods = ctx.mods
        gz = torch.empty(mods.L, mods.H, mods.W, device="cuda", dtype=torch.float32)
        gp = torch.zeros(ctx.n_par, device="cuda", dtype=torch.float32)
        check(lib().cc_syn_bwd(mods.h, _p(_f32(gx)), _p(gz), _p(gp), _stream()))
        return gz, gp, None


def arm_rate(yhat, params, mods):
    return ArmRate.apply(yhat, params, mods)


def upsample(yhat, params, mods):
    return Upsample.apply(yhat, params, mods)


def synthesis(zhat, params, mods):
    return Synthesis.apply(zhat, params, mods)
