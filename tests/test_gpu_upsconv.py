"""The upsampling Conv refinement on the GPU: with identity taps it computes
the plain upsampling (same totals; gradients within the FP32 rule); a batch
equals each state alone, bitwise; the Conv tap gradients follow the oracle
over a few steps of Adam; a 300-iteration encode follows the oracle's."""
import numpy as np
import pytest
import torch

from oracle import coolchic_ref as R
from paper_2605_02726_amd import workloads as wl

from gpu_util import outliers, segments

pytestmark = pytest.mark.gpu


def _enc(mc, H, W, seed, precision, jitter=0.0):
    from paper_2605_02726_amd.encoder import Encoder
    return Encoder(mc, torch.from_numpy(wl.synth_image(H, W, seed)), 1e-3, seed,
                   wl.random_latents(mc, H, W, seed),
                   wl.init_params(mc, seed, arm_out_zero=False, conv_jitter=jitter),
                   precision=precision)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_identity_taps_equal_the_plain_upsampling(precision):
    H, W, seed = 128, 192, 31
    plain, conv = wl.config_hop(), wl.config_hop_conv()
    a, b = _enc(plain, H, W, seed, precision), _enc(conv, H, W, seed, precision)
    ra, rb = a.step(1, 1e-2, 0.3, 0.2), b.step(1, 1e-2, 0.3, 0.2)
    assert ra == rb
    ga, gb = a.grad(), b.grad()
    offs = wl.conv_taps_offsets(conv)
    n_lat = wl.n_latents(plain, H, W)
    c0 = n_lat + offs[0]
    gb_plain = np.concatenate([gb[:c0], gb[c0 + 4 * len(offs):]])
    n_bad, worst = outliers(gb_plain, ga.astype(np.float64), 1e-5, segments(plain, H, W))
    print(f"[{precision}] {n_bad} outside 1e-5; worst {worst}", flush=True)
    assert n_bad == 0


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_conv_batch_equals_alone(precision):
    from paper_2605_02726_amd.encoder import schedule, step_batch, step_params
    mc = wl.config_hop_conv()
    shapes = ((128, 192, 41), (64, 320, 42), (192, 64, 43))
    alone = [_enc(mc, H, W, s, precision, 0.15) for H, W, s in shapes]
    batch = [_enc(mc, H, W, s, precision, 0.15) for H, W, s in shapes]
    for t in range(1, 4):
        lr, T, sg = schedule(t, 20)
        ra = [e.step(t, lr, T, sg) for e in alone]
        rb = step_batch(batch, [step_params(t, lr, T, sg)] * 3)
        assert ra == rb
    for x, y in zip(alone, batch):
        sx, sy = x.get_state(), y.get_state()
        for k in ("latents", "params", "m", "v"):
            assert np.array_equal(sx[k], sy[k]), k


def test_conv_taps_follow_the_oracle_over_steps():
    from paper_2605_02726_amd.encoder import schedule
    mc = wl.config_hop_conv()
    H, W, seed = 64, 128, 44
    enc = _enc(mc, H, W, seed, "fp32", 0.15)
    lat = wl.random_latents(mc, H, W, seed)
    par = wl.init_params(mc, seed, arm_out_zero=False, conv_jitter=0.15)
    ost = R.OracleState(mc.as_dict(), H, W, wl.synth_image(H, W, seed), 1e-3, seed, lat, par)
    offs = np.array(wl.conv_taps_offsets(mc))
    idx = (offs[:, None] + np.arange(4)[None, :]).reshape(-1)
    for t in range(1, 6):
        lr, T, sg = schedule(t, 50)
        lg = enc.step(t, lr, T, sg)[0]
        lo = ost.step(t, lr, T, sg)[0]
        assert lg == pytest.approx(lo, rel=1e-4)
    got = enc.get_state()["params"][idx].astype(np.float64)
    ref = ost.theta[ost.n_lat:][idx]
    print("conv taps", np.max(np.abs(got - ref)), flush=True)
    assert np.allclose(got, ref, rtol=0, atol=1e-5)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_short_encode_against_the_oracle(precision):
    """300 iterations of a 128x192 encode from identity taps against the FP64
    oracle's results (tests/golden/conv_encode_128x192_300.json), with the
    trajectory criterion of the hyperlatent encode: J within 1%, bits within
    2%, PSNR within 0.2%."""
    import json
    import os
    from paper_2605_02726_amd.encoder import Encoder, schedule
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "conv_encode_128x192_300.json")))
    mc = wl.config_hop_conv()
    H, W, seed, lam, n = 128, 192, 6, 1e-3, gold["n_iter"]
    enc = Encoder(mc, torch.from_numpy(wl.synth_image(H, W, seed)), lam, seed,
                  np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, seed),
                  precision=precision)
    for t in range(1, n + 1):
        enc.step(t, *schedule(t, n), sync=False)
    rd = enc.rd_eval()
    ref = gold["conv"]
    j = rd["mse"] + lam * rd["bits"] / (H * W)
    jr = ref["mse"] + lam * ref["bits"] / (H * W)
    taps = enc.get_state()["params"][np.array(wl.conv_taps_offsets(mc))[:, None] + np.arange(4)]
    print(f"bits {rd['bits']:.1f} vs {ref['bits']:.1f}, psnr {rd['psnr']:.4f} vs {ref['psnr']:.4f}, "
          f"J {j:.6f} vs {jr:.6f} ({j / jr - 1:+.2e}); taps max diff "
          f"{np.max(np.abs(taps - np.array(gold['conv_taps']))):.2e}", flush=True)
    assert abs(j / jr - 1.0) <= 1e-2
    assert rd["bits"] == pytest.approx(ref["bits"], rel=2e-2)
    assert rd["psnr"] == pytest.approx(ref["psnr"], rel=2e-3)
