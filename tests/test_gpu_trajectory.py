"""1,000-iteration trajectory of the 512x768 workload against the stored FP64
oracle trajectory (tests/golden/trajectory_512x768_1000.json, written by
tests/golden/make_trajectory.py from the oracle alone).

Per step the GPU holds the parity rules (first steps, trained states); over
1,000 Adam iterations rounding differences grow into a different path
through a flat valley of the cost.  How far correct implementations end
apart was measured on the oracle itself (same script), which forms the
reference family: the trajectory with every gradient element multiplied by
(1 + rel xi) per step, rel = 1e-6 (seeds 1-3) and rel = 1e-5 (seeds 11, 12:
the size of the split-BF16 products' rounding), and with theta, m, v rounded
to FP32 after every update.  The family ends with total bits up to 0.64%
away from the reference, PSNR up to 0.058%, and the rate-distortion cost
J = MSE + lambda bpp (the objective) in [-0.28%, +0.045%]: the end point is
bimodal, a second basin lying about 0.3% lower in J (reached by the oracle
with seed 11, and by the GPU in either form depending on rounding).  Total
bits alone cannot be held to 0.1%, and a single J tolerance narrower than
the basin spacing cannot be two-sided.

The GPU runs the trajectory in eight launch shapes that change only the
order of the synthesis and residual weight-gradient partial sums (different
rounding, same arithmetic).  Criteria after the 1,000 iterations,
hard-quantised:
  * every run: PSNR within 0.1% and bits within 1% of the reference, and J
    within the family's range widened by 0.1% on each side;
  * the mean J of the runs inside the family's range widened by 0.05% (the
    spread of a basin's end points: GPU runs in the upper basin end up to
    0.08% above the reference, the family's up to 0.045%); two-sided, so an
    offset of the GPU arithmetic larger than the basin spacing shows here,
    and smaller systematic errors are the per-step parity tests' to find.
Gradient noise of BF16 size (rel = 1e-3, *_perturbed_4.json) moves the
oracle's J by -0.44%, outside that range: the BF16 form keeps split operands
(about 16 significant bits) in every product, its weight gradients included.
The checkpoints on the way are printed.
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
# (synthesis-adjoint chunks per workgroup, residual-adjoint tiles per
# workgroup): 0 keeps the default
SHAPES = [(0, 0), (6, 1), (24, 1), (9, 2), (4, 1), (10, 1), (16, 1), (32, 1)]
# the reference family: noise-perturbed and FP32-storage oracle runs
FAMILY = ["perturbed_1", "perturbed_2", "perturbed_3", "perturbed_11", "perturbed_12", "fp32storage"]


def _j(r, hw):
    return r["mse"] + 1e-3 * r["bits"] / hw


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_trajectory_psnr_and_cost_two_sided(precision):
    from paper_2605_02726_amd.encoder import Encoder, schedule
    gold = json.load(open(GOLD))
    n_iter = gold["n_iter"]
    mc = wl.config_hop()
    H, W = 512, 768
    hw = H * W
    img = torch.from_numpy(wl.image_large(2))
    par = wl.init_params(mc, 2)
    finals = []
    for syn, res in SHAPES:
        enc = Encoder(mc, img, 1e-3, 2, np.zeros(wl.n_latents(mc, H, W), np.float32), par,
                      precision=precision)
        if syn:
            enc.set_launch_shape(0, syn, res)
        for t in range(1, n_iter + 1):
            lr, T, s = schedule(t, n_iter)
            enc.step(t, lr, T, s, sync=False)
            if str(t) in gold["rd_eval"] and t in (250, 500, 750, n_iter):
                rd = enc.rd_eval()
                ref = gold["rd_eval"][str(t)]
                print(f"[{precision} {syn}/{res}] t={t}: bits {rd['bits'] / ref['bits'] - 1:+.2e} "
                      f"psnr {rd['psnr'] / ref['psnr'] - 1:+.2e} "
                      f"J {_j(rd, hw) / _j(ref, hw) - 1:+.2e}", flush=True)
        finals.append(rd)
        del enc
    ref = gold["rd_eval"][str(n_iter)]
    fam = []
    for tag in FAMILY:
        g = json.load(open(GOLD.replace(".json", f"_{tag}.json")))
        fam.append(_j(g["rd_eval"][str(n_iter)], hw) / _j(ref, hw) - 1)
    lo, hi = min(fam + [0.0]), max(fam + [0.0])
    ej = np.array([_j(r, hw) / _j(ref, hw) - 1 for r in finals])
    eb = np.array([r["bits"] / ref["bits"] - 1 for r in finals])
    ep = np.array([r["psnr"] / ref["psnr"] - 1 for r in finals])
    print(f"[{precision}] final J {ej} (mean {ej.mean():+.2e}), bits {eb}, psnr {ep}; "
          f"oracle family J in [{lo:+.2e}, {hi:+.2e}]", flush=True)
    assert np.all(np.abs(ep) <= 1e-3)
    assert np.all(np.abs(eb) <= 1e-2)
    assert np.all(ej >= lo - 1e-3) and np.all(ej <= hi + 1e-3)
    assert lo - 5e-4 <= ej.mean() <= hi + 5e-4
