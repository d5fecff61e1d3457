"""Python front end of the encode step: one ``Encoder`` per image.

Device memory (the state slab, images) comes from PyTorch's allocator and
work runs on PyTorch's current HIP stream; every step of the path runs in the
library's kernels through the C ABI.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import CC_BF16_FUSED, CC_FP32_PLAIN, CC_HARD, CC_SOFT, check, lib

PRECISIONS = {"fp32": CC_FP32_PLAIN, "bf16": CC_BF16_FUSED}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return C.c_void_p(a.ctypes.data)


def step_params(t: int, lr: float, T: float, sigma: float, quant: str = "soft",
                update_latents: bool = True) -> _lib.cc_step_params:
    p = _lib.cc_step_params()
    p.t = int(t)
    p.lr = float(lr)
    p.temperature = float(T)
    p.sigma = float(sigma)
    p.quant_mode = CC_SOFT if quant == "soft" else CC_HARD
    p.update_latents = 1 if update_latents else 0
    return p


def schedule(t: int, n_iter: int, lr0=1e-2, lr1=1e-5, T0=0.35, T1=0.08, s0=0.22, s1=0.15,
             cosine_lr=True):
    """Table I schedules mapped linearly onto an n_iter budget (t from 1):
    cosine learning rate, linear softround temperature and noise std."""
    a = 0.0 if n_iter <= 1 else (t - 1) / (n_iter - 1)
    lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * a)) if cosine_lr else lr0
    return lr, T0 + (T1 - T0) * a, s0 + (s1 - s0) * a


def set_branch_overlap(enable: bool) -> bool:
    """Run the rate branch of every following step concurrently with the
    distortion branch (the default) or in order on one stream; returns the
    previous setting."""
    return bool(lib().cc_set_branch_overlap(1 if enable else 0))


def state_bytes(mc, H: int, W: int, precision: str = "fp32") -> int:
    cfg = _lib.make_config(mc, PRECISIONS[precision])
    n = lib().cc_state_bytes(C.byref(cfg), H, W)
    if n == 0:
        check(_lib.CC_EINVAL)
    return int(n)


class Encoder:
    """Device-resident encoder state of one image (latents, decoder
    parameters, Adam moments, scratch) in one slab."""

    def __init__(self, mc, image, lam: float, seed: int, latents=None, params=None,
                 precision: str = "fp32", slab: Optional[torch.Tensor] = None,
                 optimizer: str = "adam"):
        if not torch.cuda.is_available():
            raise RuntimeError("the encode step needs a HIP GPU")
        self.mc = mc
        self.precision = precision
        self.cfg = _lib.make_config(mc, PRECISIONS[precision])
        img = torch.as_tensor(image, dtype=torch.float32)
        if img.dim() != 3 or img.shape[0] != 3:
            raise ValueError("image must be [3, H, W]")
        self.H, self.W = int(img.shape[1]), int(img.shape[2])
        self.img = img.to("cuda").contiguous()
        L = lib()
        nbytes = L.cc_state_bytes(C.byref(self.cfg), self.H, self.W)
        if nbytes == 0:
            check(_lib.CC_EINVAL)
        self.nbytes = int(nbytes)
        self.slab = slab if slab is not None else torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        if self.slab.numel() < self.nbytes:
            raise ValueError("slab too small")
        self.n_lat = int(L.cc_n_latents(C.byref(self.cfg), self.H, self.W))
        self.n_par = int(L.cc_n_params(C.byref(self.cfg)))
        lat = None if latents is None else np.ascontiguousarray(latents, dtype=np.float32)
        par = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        if lat is not None and lat.size != self.n_lat:
            raise ValueError(f"latents: {lat.size} values, need {self.n_lat}")
        if par is not None and par.size != self.n_par:
            raise ValueError(f"params: {par.size} values, need {self.n_par}")
        h = C.c_void_p()
        check(L.cc_init_state(C.byref(self.cfg), self.H, self.W, C.c_void_p(self.img.data_ptr()),
                              float(lam), int(seed) & 0xFFFFFFFFFFFFFFFF, _ptr(lat), _ptr(par),
                              C.c_void_p(self.slab.data_ptr()), self.nbytes, _stream(),
                              C.byref(h)))
        self.handle = h
        self.lam = float(lam)
        self.seed = int(seed)
        self.optimizer = "adam"
        if optimizer != "adam":
            self.set_optimizer(optimizer)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().cc_free_state(h)
            except Exception:
                pass
            self.handle = None

    # ------------------------------------------------------------ steps --
    def step(self, t: int, lr: float, T: float, sigma: float, quant: str = "soft",
             update_latents: bool = True, sync: bool = True):
        """One encoding iteration; returns (loss, bits, mse) when sync."""
        p = step_params(t, lr, T, sigma, quant, update_latents)
        out = (C.c_double * 3)() if sync else None
        check(lib().cc_encode_step(self.handle, C.byref(p), out, _stream()))
        return tuple(out) if sync else None

    def eval_loss(self, t: int, T: float, sigma: float, quant: str = "soft"):
        p = step_params(t, 0.0, T, sigma, quant)
        out = (C.c_double * 3)()
        check(lib().cc_eval_loss(self.handle, C.byref(p), out, _stream()))
        return tuple(out)

    def rd_eval(self):
        r = _lib.cc_rd_result()
        check(lib().cc_rd_eval(self.handle, C.byref(r), _stream()))
        return dict(bits=r.bits, bpp=r.bpp, mse=r.mse, psnr=r.psnr, loss=r.loss)

    def set_launch_shape(self, arm_wgs: int = 0, syn_chunks_per_wg: int = 0,
                         res_tiles_per_wg: int = 0):
        """Launch shape of the tunable kernels (0 keeps a value)."""
        check(lib().cc_set_launch_shape(self.handle, int(arm_wgs), int(syn_chunks_per_wg),
                                        int(res_tiles_per_wg), _stream()))

    def launch_shape(self) -> dict:
        v = [C.c_int(0) for _ in range(4)]
        check(lib().cc_get_launch_shape(self.handle, *[C.byref(x) for x in v]))
        return dict(arm_wgs=v[0].value, syn_chunks_per_wg=v[1].value,
                    res_tiles_per_wg=v[2].value, arm_bands=v[3].value)

    def nn_quantize(self):
        """Choose the quantisation steps and Exp-Golomb orders of the decoder
        parameters by rate-distortion cost and leave the state with the
        quantised decoder (Section IV-E)."""
        r = _lib.cc_nnq_result()
        check(lib().cc_nn_quantize(self.handle, C.byref(r), _stream()))
        subs = ("arm", "syn", "ups", "ifce")
        return dict(step_index={a: tuple(r.step_index[i]) for i, a in enumerate(subs)},
                    step={a: tuple(r.step[i]) for i, a in enumerate(subs)},
                    kappa={a: tuple(r.kappa[i]) for i, a in enumerate(subs)},
                    nn_bits=r.nn_bits, bits=r.bits, mse=r.mse, psnr=r.psnr, loss=r.loss)

    def decode(self) -> torch.Tensor:
        out = torch.empty(3, self.H, self.W, dtype=torch.float32, device="cuda")
        check(lib().cc_decode(self.handle, C.c_void_p(out.data_ptr()), _stream()))
        return out

    def set_precision(self, precision: str):
        check(lib().cc_set_precision(self.handle, PRECISIONS[precision]))
        self.precision = precision

    def set_optimizer(self, optimizer: str):
        """Decoder-parameter optimiser: "adam" or "soap" (selecting SOAP
        clears its state; the next step initialises it)."""
        kinds = {"adam": _lib.CC_OPT_ADAM, "soap": _lib.CC_OPT_SOAP}
        check(lib().cc_set_optimizer(self.handle, kinds[optimizer], _stream()))
        self.optimizer = optimizer

    def soap_factor_size(self) -> int:
        return int(lib().cc_soap_factor_size(C.byref(self.cfg)))

    def get_soap_state(self):
        nf = self.soap_factor_size()
        m = np.empty(self.n_par, np.float32)
        v = np.empty(self.n_par, np.float32)
        p = np.empty(nf, np.float32)
        q = np.empty(nf, np.float32)
        calls = C.c_int()
        check(lib().cc_get_soap_state(self.handle, _ptr(m), _ptr(v), _ptr(p), _ptr(q),
                                      C.byref(calls), _stream()))
        return dict(m=m, v=v, p=p, q=q, calls=int(calls.value))

    def set_soap_state(self, m=None, v=None, p=None, q=None, calls: int = 0):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float32)
                for a in (m, v, p, q)]
        check(lib().cc_set_soap_state(self.handle, *[_ptr(a) for a in arrs], int(calls),
                                      _stream()))

    # ------------------------------------------------------------ state --
    def get_state(self):
        lat = np.empty(self.n_lat, np.float32)
        par = np.empty(self.n_par, np.float32)
        m = np.empty(self.n_lat + self.n_par, np.float32)
        v = np.empty(self.n_lat + self.n_par, np.float32)
        t = C.c_int64()
        check(lib().cc_get_state(self.handle, _ptr(lat), _ptr(par), _ptr(m), _ptr(v),
                                 C.byref(t), _stream()))
        return dict(latents=lat, params=par, m=m, v=v, t=int(t.value))

    def set_state(self, latents=None, params=None, m=None, v=None, t: int = 0):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float32)
                for a in (latents, params, m, v)]
        check(lib().cc_set_state(self.handle, *[_ptr(a) for a in arrs], int(t), _stream()))

    def debug_read(self, name: str, count: int) -> np.ndarray:
        out = np.empty(count, np.float32)
        check(lib().cc_debug_read(self.handle, name.encode(), _ptr(out), count, _stream()))
        return out

    def grad(self) -> np.ndarray:
        g = np.empty(self.n_lat + self.n_par, np.float32)
        check(lib().cc_get_grad(self.handle, _ptr(g), _stream()))
        return g


def step_batch(encoders: Sequence[Encoder], params: Sequence[_lib.cc_step_params],
               sync: bool = True):
    """One iteration for every encoder in one set of launches; returns a list
    of (loss, bits, mse) when sync."""
    n = len(encoders)
    hs = (C.c_void_p * n)(*[e.handle.value for e in encoders])
    ps = (_lib.cc_step_params * n)(*params)
    out = (C.c_double * (3 * n))() if sync else None
    rc = lib().cc_encode_step_batch(hs, n, ps, out, _stream())
    if rc == _lib.CC_ENONFINITE and sync:
        # every state's totals were read; the caller finds the non-finite ones
        return [tuple(out[3 * i:3 * i + 3]) for i in range(n)]
    check(rc)
    if not sync:
        return None
    return [tuple(out[3 * i:3 * i + 3]) for i in range(n)]
