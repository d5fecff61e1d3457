"""1,000-iteration trajectory of the 512x768 workload against the stored FP64
oracle trajectory (tests/golden/trajectory_512x768_1000.json, written by
tests/golden/make_trajectory.py from the oracle alone).

Criterion: after the 1,000 iterations, the hard-quantised total rate (bits)
and PSNR within 0.1% of the oracle's, for the plain FP32 and the fused BF16
forms.  The checkpoints on the way are printed, not asserted: Adam's first
moments turn rounding-level gradient differences into +-lr steps, and
mid-course totals of even the FP32 form wander by a few tenths of a percent
from the FP64 trajectory before the schedules anneal them back together.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_2605_02726_amd import workloads as wl

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "trajectory_512x768_1000.json")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_trajectory_totals_within_0p1_percent(precision):
    from paper_2605_02726_amd.encoder import Encoder, schedule
    gold = json.load(open(GOLD))
    n_iter = gold["n_iter"]
    mc = wl.config_hop()
    H, W = 512, 768
    enc = Encoder(mc, torch.from_numpy(wl.image_large(2)), 1e-3, 2,
                  np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, 2),
                  precision=precision)
    worst = 0.0
    for t in range(1, n_iter + 1):
        lr, T, s = schedule(t, n_iter)
        enc.step(t, lr, T, s, sync=False)
        if str(t) in gold["rd_eval"]:
            rd = enc.rd_eval()
            ref = gold["rd_eval"][str(t)]
            eb = rd["bits"] / ref["bits"] - 1.0
            ep = rd["psnr"] / ref["psnr"] - 1.0
            print(f"[{precision}] t={t}: bits {rd['bits']:.1f} vs {ref['bits']:.1f} ({eb:+.2e}), "
                  f"psnr {rd['psnr']:.4f} vs {ref['psnr']:.4f} ({ep:+.2e})", flush=True)
            if t == n_iter:
                worst = max(abs(eb), abs(ep))
    assert worst <= 1e-3
