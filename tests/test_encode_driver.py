"""Stage logic of the multi-stage encoder (Section IV-D): warm-up selection by
rate-distortion cost, main-stage schedules, frozen latents in the hard-round
stage.  Runs on the CPU with the FP64 oracle standing in for the GPU backend
(test infrastructure only)."""
import numpy as np
import pytest

from oracle import coolchic_ref as R
from paper_2605_02726_amd import workloads as wl
from paper_2605_02726_amd.encode import StagePlan, encode, main_schedule


class OracleBackend:
    def __init__(self, mc, image, lam):
        self.mc, self.image, self.lam = mc, image, lam
        self.calls = []

    def create(self, seed, params):
        _, H, W = self.image.shape
        return R.OracleState(self.mc.as_dict(), H, W, self.image, self.lam, seed,
                             np.zeros(wl.n_latents(self.mc, H, W), np.float32), params)

    def step_batch(self, handles, specs):
        self.calls.append((len(handles), specs[0]))
        for h, (t, lr, T, s, quant, upd) in zip(handles, specs):
            h.step(t, lr, T if quant == "soft" else 1.0, s, quant=quant, update_latents=upd)

    def rd_eval(self, h):
        return h.rd_eval()

    def latents(self, h):
        return h.theta[:h.n_lat].copy()


def test_stages_select_the_best_candidates_and_freeze_latents():
    mc = wl.config_tiny()
    img = wl.synth_image(16, 16, 3)
    be = OracleBackend(mc, img, 1e-2)
    plan = StagePlan(candidates=(3, 2), warmup_iters=3, main_iters=4, hard_iters=2)
    params = [wl.init_params(mc, 10 + i) for i in range(3)]
    res = encode(be, params, plan, seeds=[10, 11, 12])
    w1, w2 = res.history[0], res.history[1]
    assert len(w1["costs"]) == 3 and len(w1["kept"]) == 2
    assert w1["costs"][w1["kept"][0]] == min(w1["costs"])
    assert len(w2["costs"]) == 2 and len(w2["kept"]) == 1
    # batched warm-up calls: 3 candidates, then 2; then single-state stages
    sizes = [n for n, _ in be.calls]
    assert sizes == [3] * 3 + [2] * 3 + [1] * 4 + [1] * 2
    # the hard stage uses true rounding and leaves the latents alone
    assert [s[4] for _, s in be.calls[-2:]] == ["hard", "hard"]
    assert [s[5] for _, s in be.calls[-2:]] == [False, False]
    main_lat = res.history[2]
    assert res.rd["bits"] > 0 and np.isfinite(res.rd["loss"])


def test_hard_stage_keeps_latents_fixed():
    mc = wl.config_tiny()
    img = wl.synth_image(16, 16, 4)
    be = OracleBackend(mc, img, 1e-2)
    plan = StagePlan(candidates=(), warmup_iters=0, main_iters=3, hard_iters=0)
    res = encode(be, [wl.init_params(mc, 1)], plan, seeds=[1])
    before = be.latents(res.handle)
    for i in range(3):
        be.step_batch([res.handle], [(10 + i, 1e-3, 1.0, 0.0, "hard", False)])
    assert np.array_equal(be.latents(res.handle), before)


def test_main_schedule_endpoints():
    p = StagePlan()
    assert main_schedule(1, 100, p) == (p.lr0, p.T0, p.s0)
    lr, T, s = main_schedule(100, 100, p)
    assert lr == pytest.approx(p.lr1) and T == pytest.approx(p.T1) and s == pytest.approx(p.s1)
