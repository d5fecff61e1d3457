"""cc_rd_eval_noalloc: the hard-quantised rate-distortion evaluation with its
scratch in the library's static device array instead of the state slab.

Checked through the C ABI against cc_rd_eval on the same state (same kernels
in the same order, so the results must be equal bit for bit), on two calls
in a row with the second on a smaller image, in both precisions; the state
slab must be left as it was; a state whose evaluation needs more scratch
than the array holds is refused before anything runs.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2605_02726_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _enc(mc, H, W, seed, precision):
    from paper_2605_02726_amd.encoder import Encoder
    img = wl.image_large(seed) if (H, W) == (512, 768) else wl.synth_image(H, W, seed)
    return Encoder(mc, torch.from_numpy(img), 1e-3, seed, wl.random_latents(mc, H, W, seed),
                   wl.init_params(mc, seed, arm_out_zero=False), precision=precision)


def _rd(fn, enc):
    from paper_2605_02726_amd import _lib
    r = _lib.cc_rd_result()
    rc = fn(enc.handle, C.byref(r), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, (r.bits, r.bpp, r.mse, r.psnr, r.loss)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_rd_eval_equals_rd_eval(precision):
    from paper_2605_02726_amd._lib import lib
    L = lib()
    mc = wl.config_hop()
    # the larger image first, then a smaller one: the second call must not
    # see anything the first left in the shared array
    for H, W, seed in ((512, 768, 2), (128, 192, 12)):
        enc = _enc(mc, H, W, seed, precision)
        enc.step(1, 1e-2, 0.35, 0.22)            # a state that is not the initial one
        before = torch.clone(enc.slab)
        rc, got = _rd(L.cc_rd_eval_noalloc, enc)
        assert rc == 0, L.cc_last_error()
        assert torch.equal(enc.slab, before), "the no-allocation evaluation wrote to the state slab"
        rc, ref = _rd(L.cc_rd_eval, enc)
        assert rc == 0
        print(f"[{precision} {H}x{W}] noalloc {got} vs rd_eval {ref}", flush=True)
        assert got == ref
        # and again, after the slab's own scratch has been written by cc_rd_eval
        rc, again = _rd(L.cc_rd_eval_noalloc, enc)
        assert rc == 0 and again == ref


def test_noalloc_rejects_oversized_state():
    from paper_2605_02726_amd._lib import CC_ENOMEM, lib
    L = lib()
    mc = wl.config_hop()
    enc = _enc(mc, 2048, 2048, 5, "fp32")
    rc, _ = _rd(L.cc_rd_eval_noalloc, enc)
    assert rc == CC_ENOMEM
    assert b"scratch" in L.cc_last_error()
