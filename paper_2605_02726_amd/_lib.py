"""ctypes binding of libcoolchic.so (argument marshalling only).

Every call forwards to the C ABI declared in include/coolchic.h; all
arithmetic runs in the library's HIP kernels.  Loading fails loudly when the
library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcoolchic.so")

CC_OK, CC_EINVAL, CC_ENOMEM, CC_EDEVICE, CC_ENONFINITE, CC_ESTATE = 0, -1, -2, -3, -4, -5
CC_SOFT, CC_HARD = 0, 1
CC_FP32_PLAIN, CC_BF16_FUSED = 0, 1
CC_OPT_ADAM, CC_OPT_SOAP = 0, 1
CC_MAX_BATCH = 32

ERRORS = {CC_EINVAL: "EINVAL", CC_ENOMEM: "ENOMEM", CC_EDEVICE: "EDEVICE",
          CC_ENONFINITE: "ENONFINITE", CC_ESTATE: "ESTATE"}


class CCError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class cc_config(C.Structure):
    _fields_ = [("L", C.c_int), ("n_spatial", C.c_int), ("n_ifce_feat", C.c_int),
                ("n_ifce_grids", C.c_int), ("arm_hidden", C.c_int * 2), ("arm_stab", C.c_int),
                ("n_syn_hidden", C.c_int), ("syn_hidden", C.c_int * 2), ("syn_stab", C.c_int),
                ("n_res", C.c_int), ("logscale_min", C.c_float), ("logscale_max", C.c_float),
                ("p_min", C.c_float), ("precision", C.c_int), ("n_hyper", C.c_int),
                ("hyper_first", C.c_int),
                ("ups_conv", C.c_int)]


class cc_step_params(C.Structure):
    _fields_ = [("t", C.c_int64), ("lr", C.c_float), ("temperature", C.c_float),
                ("sigma", C.c_float), ("quant_mode", C.c_int), ("update_latents", C.c_int)]


class cc_rd_result(C.Structure):
    _fields_ = [("bits", C.c_double), ("bpp", C.c_double), ("mse", C.c_double),
                ("psnr", C.c_double), ("loss", C.c_double)]


class cc_nnq_result(C.Structure):
    _fields_ = [("step_index", (C.c_int * 2) * 4), ("step", (C.c_double * 2) * 4),
                ("kappa", (C.c_int * 2) * 4), ("nn_bits", C.c_double), ("bits", C.c_double),
                ("mse", C.c_double), ("psnr", C.c_double), ("loss", C.c_double)]


_lib = None

# (name, restype, argtypes)
_PROTOS = [
    ("cc_config_supported", C.c_int, [C.POINTER(cc_config), C.c_int, C.c_int]),
    ("cc_n_latents", C.c_int64, [C.POINTER(cc_config), C.c_int, C.c_int]),
    ("cc_n_params", C.c_int, [C.POINTER(cc_config)]),
    ("cc_state_bytes", C.c_size_t, [C.POINTER(cc_config), C.c_int, C.c_int]),
    ("cc_timing_every", C.c_int, [C.c_int]),
    ("cc_arm_band_plan", C.c_int, [C.POINTER(cc_config), C.c_int, C.c_int, C.c_int,
                                   C.POINTER(C.c_int), C.POINTER(C.c_int), C.c_void_p, C.c_void_p]),
    ("cc_init_state", C.c_int, [C.POINTER(cc_config), C.c_int, C.c_int, C.c_void_p, C.c_double,
                                C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                C.c_void_p, C.POINTER(C.c_void_p)]),
    ("cc_encode_step", C.c_int, [C.c_void_p, C.POINTER(cc_step_params), C.c_void_p, C.c_void_p]),
    ("cc_encode_step_batch", C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(cc_step_params),
                                       C.c_void_p, C.c_void_p]),
    ("cc_eval_loss", C.c_int, [C.c_void_p, C.POINTER(cc_step_params), C.c_void_p, C.c_void_p]),
    ("cc_rd_eval", C.c_int, [C.c_void_p, C.POINTER(cc_rd_result), C.c_void_p]),
    ("cc_rd_eval_noalloc", C.c_int, [C.c_void_p, C.POINTER(cc_rd_result), C.c_void_p]),
    ("cc_nn_quantize", C.c_int, [C.c_void_p, C.POINTER(cc_nnq_result), C.c_void_p]),
    ("cc_decode", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("cc_get_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.POINTER(C.c_int64), C.c_void_p]),
    ("cc_set_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                               C.c_int64, C.c_void_p]),
    ("cc_get_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("cc_set_precision", C.c_int, [C.c_void_p, C.c_int]),
    ("cc_set_optimizer", C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    ("cc_soap_factor_size", C.c_int64, [C.POINTER(cc_config)]),
    ("cc_get_soap_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_int), C.c_void_p]),
    ("cc_set_soap_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                    C.c_int, C.c_void_p]),
    ("cc_debug_read", C.c_int, [C.c_void_p, C.c_char_p, C.c_void_p, C.c_int64, C.c_void_p]),
    ("cc_arm_fwd_bwd", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                 C.c_void_p, C.c_void_p, C.c_void_p]),
    ("cc_ups_fwd", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("cc_ups_bwd", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("cc_syn_fwd", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("cc_syn_bwd", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("cc_timing_enable", C.c_int, [C.c_char_p]),
    ("cc_set_branch_overlap", C.c_int, [C.c_int]),
    ("cc_set_launch_shape", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_void_p]),
    ("cc_get_launch_shape", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                      C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("cc_arm_fused_available", C.c_int, [C.c_void_p]),
    ("cc_timing_read", C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    ("cc_free_state", None, [C.c_void_p]),
    ("cc_last_error", C.c_char_p, []),
]

EXPORTED = [n for n, _, _ in _PROTOS]


def lib():
    """The loaded library; raises if it is missing (build it first with
    ``python -m paper_2605_02726_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python -m paper_2605_02726_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _PROTOS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc: int):
    if rc != CC_OK:
        raise CCError(rc, lib().cc_last_error().decode(errors="replace"))


def make_config(mc, precision: int = CC_FP32_PLAIN) -> cc_config:
    """cc_config from a workloads.ModelConfig (or anything with its fields)."""
    c = cc_config()
    c.L = mc.L
    c.n_spatial = mc.n_spatial
    c.n_ifce_feat = mc.n_ifce_feat
    c.n_ifce_grids = mc.n_ifce_grids
    if len(mc.arm_hidden) != 2:
        raise ValueError("the ARM has two hidden layers")
    c.arm_hidden[0], c.arm_hidden[1] = mc.arm_hidden
    c.arm_stab = int(mc.arm_stab)
    c.n_syn_hidden = len(mc.syn_hidden)
    for i, w in enumerate(mc.syn_hidden[:2]):
        c.syn_hidden[i] = w
    c.syn_stab = int(mc.syn_stab)
    c.n_res = mc.n_res
    c.logscale_min = mc.logscale_min
    c.logscale_max = mc.logscale_max
    c.n_hyper = int(getattr(mc, "n_hyper", 0))
    c.hyper_first = int(getattr(mc, "hyper_first", 4))
    c.ups_conv = int(getattr(mc, "ups_conv", 0))
    c.p_min = mc.p_min
    c.precision = precision
    return c
