"""Hyperlatent grids (Section III-A.3) on the GPU beyond the first-step
parity cases: a 300-iteration 128x192 encode with and without hyperlatents
against the FP64 oracle's results of the same runs
(tests/golden/hyper_encode_128x192_300.json), and batched steps of
hyperlatent states bitwise equal to the same states stepped alone.

Trajectory criterion (as for the 512x768 trajectory): the rate-distortion
cost J = MSE + lambda bpp within 1% of the oracle's, bits within 2%, PSNR
within 0.2%."""
import json
import os

import numpy as np
import pytest
import torch

from paper_2605_02726_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("name", ["plain", "hyper"])
def test_short_encode_against_the_oracle(name, precision):
    from paper_2605_02726_amd.encoder import Encoder, schedule
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "hyper_encode_128x192_300.json")))
    mc = wl.config_hop_hyper() if name == "hyper" else wl.config_hop()
    H, W, seed, lam, n = 128, 192, 6, 1e-3, gold["n_iter"]
    enc = Encoder(mc, torch.from_numpy(wl.synth_image(H, W, seed)), lam, seed,
                  np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, seed),
                  precision=precision)
    for t in range(1, n + 1):
        enc.step(t, *schedule(t, n), sync=False)
    rd = enc.rd_eval()
    ref = gold[name]
    j = rd["mse"] + lam * rd["bits"] / (H * W)
    jr = ref["mse"] + lam * ref["bits"] / (H * W)
    print(f"[{name}] bits {rd['bits']:.1f} vs {ref['bits']:.1f}, psnr {rd['psnr']:.4f} vs "
          f"{ref['psnr']:.4f}, J {j:.6f} vs {jr:.6f} ({j / jr - 1:+.2e})", flush=True)
    assert abs(j / jr - 1.0) <= 1e-2
    assert rd["bits"] == pytest.approx(ref["bits"], rel=2e-2)
    assert rd["psnr"] == pytest.approx(ref["psnr"], rel=2e-3)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_hyper_batch_equals_alone(precision):
    from paper_2605_02726_amd.encoder import Encoder, step_batch, step_params
    mc = wl.config_hop_hyper()
    alone, batch = [], []
    for H, W, s in ((128, 192, 61), (64, 320, 62)):
        img = torch.from_numpy(wl.synth_image(H, W, s))
        lat = wl.random_latents(mc, H, W, s)
        par = wl.init_params(mc, s, arm_out_zero=False)
        alone.append(Encoder(mc, img, 1e-3, s, lat, par, precision=precision))
        batch.append(Encoder(mc, img, 1e-3, s, lat, par, precision=precision))
    for t in (1, 2, 3):
        ra = [e.step(t, 1e-2, 0.3, 0.2) for e in alone]
        rb = step_batch(batch, [step_params(t, 1e-2, 0.3, 0.2)] * 2)
        assert ra == rb
    for a, b in zip(alone, batch):
        sa, sb = a.get_state(), b.get_state()
        for k in ("latents", "params", "m", "v"):
            assert np.array_equal(sa[k], sb[k]), k


@pytest.mark.parametrize("mk", [wl.config_hop_hyper, wl.config_hop_conv])
def test_multi_stage_driver_on_the_gpu(mk):
    """The multi-stage driver (warm-up candidates in one batch, main stage,
    hard-round stage with frozen latents) with the hyperlatent and the Conv
    refinement decoders: latents sized by the library (hyperlatent grids
    included), every stage runs, and the final cost is below the best
    warm-up cost."""
    from paper_2605_02726_amd.encode import GpuBackend, StagePlan, encode
    mc = mk()
    H, W = 64, 128
    img = wl.synth_image(H, W, 71)
    be = GpuBackend(mc, img, 1e-3, precision="bf16")
    plan = StagePlan(candidates=(3, 2), warmup_iters=20, main_iters=60, hard_iters=10)
    res = encode(be, [wl.init_params(mc, 80 + i) for i in range(3)], plan)
    assert res.handle.n_lat == wl.n_latents(mc, H, W)
    stages = [h["stage"] for h in res.history]
    assert stages == ["warm-up", "warm-up", "main", "hard"]
    first = res.history[0]["costs"]
    print("warm-up costs", first, "final", res.rd, flush=True)
    assert res.rd["loss"] < min(first)
