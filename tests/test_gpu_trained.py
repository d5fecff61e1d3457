"""Per-step parity from trained states (Sections IV-A to IV-C: one encoding
iteration = quantisation proxy, rate + distortion, gradient, Adam).

The first-step cases start from initial or random states.  Here the oracle
trains a 64x128 image with the workload's decoder for a 400-iteration budget
(Table I schedules mapped onto it: cosine learning rate 1e-2 -> 1e-5,
temperature 0.35 -> 0.08, noise 0.22 -> 0.15), and its state (latents,
parameters, Adam moments, t) at t = 150 and at the end (t = 400, where the
latents are large, many log-scales sit at their clamp and the temperature is
low) is loaded into the GPU state.  The GPU then takes the next iteration
and is held to the same rules as from a fresh state: FP32 totals within
1e-5 and every gradient element within 1e-5 (|oracle| + rms) plus the slack
of near-threshold decisions; BF16 totals within 1e-3 and every element
within 2e-2 (|oracle| + rms) plus the slack of the decisions near threshold
at BF16 resolution; the Adam update of the parameters as the oracle's update
of the oracle gradient within the image of those tolerances.
"""
import numpy as np
import pytest
import torch

from oracle import coolchic_ref as R
from paper_2605_02726_amd import workloads as wl

from gpu_util import decision_slack, fp32_eval_slack, outliers, segments, slack_outliers

pytestmark = pytest.mark.gpu

H, W, SEED, LAM, N_ITER = 64, 128, 31, 1e-3, 400
STATES = (150, 400)
_CACHE = {}


def _trained():
    """Oracle states along one 400-iteration run (computed once)."""
    if not _CACHE:
        torch.set_num_threads(max(1, min(16, torch.get_num_threads())))
        mc = wl.config_hop()
        img = wl.synth_image(H, W, SEED)
        st = R.OracleState(mc.as_dict(), H, W, img, LAM, SEED,
                           np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, SEED))
        for t in range(1, N_ITER + 1):
            st.step(t, *R.schedule(t, N_ITER))
            if t in STATES:
                _CACHE[t] = (st.theta.copy(), st.m.copy(), st.v.copy())
        _CACHE["mc"], _CACHE["img"] = mc, img
    return _CACHE


def _gpu_after(precision, t0):
    from paper_2605_02726_amd.encoder import Encoder
    c = _trained()
    mc, img = c["mc"], c["img"]
    theta, m, v = c[t0]
    n_lat = wl.n_latents(mc, H, W)
    th32 = theta.astype(np.float32)
    enc = Encoder(mc, torch.from_numpy(img), LAM, SEED, th32[:n_lat], th32[n_lat:],
                  precision=precision)
    enc.set_state(m=m.astype(np.float32), v=v.astype(np.float32), t=t0)
    # the last budget step has no successor: step N_ITER again from the end
    t = t0 + 1 if t0 < N_ITER else t0
    lr, T, s = R.schedule(t, N_ITER)
    tot = enc.step(t, lr, T, s)
    return mc, img, th32.astype(np.float64), m.astype(np.float32).astype(np.float64), \
        v.astype(np.float32).astype(np.float64), (t, lr, T, s), tot, enc.grad(), enc.get_state()


@pytest.mark.parametrize("t0", STATES)
@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_step_from_trained_state(precision, t0):
    mc, img, theta, m, v, (t, lr, T, s), tot, g, st = _gpu_after(precision, t0)
    ref = R.loss_and_grad(mc.as_dict(), H, W, theta, img, LAM, "soft", T, s, SEED, t)
    rtol, ttol, tau = (1e-5, 1e-5, 3e-6) if precision == "fp32" else (2e-2, 1e-3, 3e-5)
    segs = segments(mc, H, W)
    n_lat = wl.n_latents(mc, H, W)
    lat = theta[:n_lat]
    print(f"[{precision} t={t}] |latent| max {np.abs(lat).max():.2f}; loss {tot[0]:.9g} vs "
          f"{ref[0]:.9g}; bits {tot[1]:.9g} vs {ref[1]:.9g}; mse {tot[2]:.9g} vs {ref[2]:.9g}",
          flush=True)
    for a, b in zip(tot, ref[:3]):
        assert a == pytest.approx(b, rel=ttol)
    n_plain, worst = outliers(g, ref[3], rtol, segs)
    slack = np.zeros_like(ref[3])
    n_bad, n_near, n_used = 0, 0, 0
    n_fp32 = 0
    if n_plain:
        _, slack, n_near, n_used = decision_slack(mc, H, W, theta, img, LAM, "soft", T, s, SEED,
                                                  t, tau=tau, max_sites=64)
        n_bad, worst = slack_outliers(g, ref[3], slack, rtol, segs)
        n_fp32 = n_bad
        if n_bad:
            # what FP32 evaluation of the same formulas deviates by here
            slack = slack + fp32_eval_slack(mc, H, W, theta, img, LAM, "soft", T, s, SEED, t, segs)
            n_bad, worst = slack_outliers(g, ref[3], slack, rtol, segs)
    print(f"[{precision} t={t}] gradient: {n_plain} of {g.size} outside the plain rule; "
          f"{n_near} near-threshold decisions ({n_used} used); {n_fp32} outside with their slack, "
          f"{n_bad} also outside the FP32-evaluation slack; worst {worst}", flush=True)
    assert n_bad == 0
    # Adam on the decoder parameters: the GPU's new parameters against the
    # oracle's Adam update of the oracle gradient, within the image of the
    # gradient tolerance delta through the update's derivative in g
    gref = ref[3][n_lat:]
    delta = slack[n_lat:].copy()
    for name, sl in segs:
        if sl.start >= n_lat:
            q = slice(sl.start - n_lat, sl.stop - n_lat)
            delta[q] += rtol * (np.abs(gref[q]) + np.sqrt(np.mean(gref[q] ** 2)))
    b1, b2 = 1 - R.BETA1 ** t, 1 - R.BETA2 ** t
    m2 = R.BETA1 * m[n_lat:] + (1 - R.BETA1) * gref
    v2 = R.BETA2 * v[n_lat:] + (1 - R.BETA2) * gref * gref
    sq = np.sqrt(v2 / b2)
    new_ref = theta[n_lat:] - lr * (m2 / b1) / (sq + R.EPS)
    # |d step / d g| <= lr ((1-beta1)/b1 + |m_hat| (1-beta2) (|g| + delta) / (b2 sqrt(v_hat))) / (sqrt(v_hat) + eps)
    sens = lr * ((1 - R.BETA1) / b1 + np.abs(m2 / b1) * (1 - R.BETA2) * (np.abs(gref) + delta) /
                 (b2 * np.maximum(sq, 1e-30) * (sq + R.EPS))) / (sq + R.EPS)
    bound = 2 * sens * delta + 2.4e-7 * (np.abs(new_ref) + lr) + 1e-12
    got = st["params"].astype(np.float64)
    n_upd = int(np.sum(np.abs(got - new_ref) > bound))
    print(f"[{precision} t={t}] parameter update: {n_upd} of {gref.size} outside the bound",
          flush=True)
    assert n_upd == 0
