"""The two branches of an iteration run concurrently (rate branch on the
library's second stream) or in order: the results must be bitwise the same,
for single and batched steps, both forms, evaluations and the hard stage."""
import numpy as np
import pytest
import torch

from paper_2605_02726_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _run(overlap, precision, quant):
    from paper_2605_02726_amd.encoder import (Encoder, schedule, set_branch_overlap, step_batch,
                                              step_params)
    prev = set_branch_overlap(overlap)
    try:
        mc = wl.config_hop()
        encs = []
        for H, W, s in ((128, 192, 51), (64, 320, 52), (192, 64, 53)):
            encs.append(Encoder(mc, torch.from_numpy(wl.synth_image(H, W, s)), 1e-3, s,
                                wl.random_latents(mc, H, W, s), wl.init_params(mc, s, arm_out_zero=False),
                                precision=precision))
        res = []
        for t in range(1, 6):
            lr, T, sg = schedule(t, 20)
            res.append(encs[0].step(t, lr, T, sg, quant=quant))
            ps = [step_params(t, lr, T, sg, quant=quant)] * 2
            res.extend(step_batch(encs[1:], ps))
        res.append(encs[0].eval_loss(6, 0.3, 0.2))
        rd = encs[1].rd_eval()
        res.append((rd["bits"], rd["mse"]))
        states = [e.get_state() for e in encs]
        return res, states
    finally:
        set_branch_overlap(prev)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("quant", ["soft", "hard"])
def test_overlapped_branches_are_bitwise_serial(precision, quant):
    ra, sa = _run(True, precision, quant)
    rb, sb = _run(False, precision, quant)
    assert ra == rb
    for a, b in zip(sa, sb):
        for k in ("latents", "params", "m", "v"):
            assert np.array_equal(a[k], b[k]), k
