"""GPU encode step (plain FP32 form) against the FP64 CPU oracle.

Rule (per element, per step from the same state): |gpu - oracle| <=
rtol |oracle| + rtol rms(oracle over the tensor), rtol = 1e-5; loss, bits and
MSE totals within 1e-5 relative.  A ReLU, clamp or probability-floor
decision whose argument lies within rounding of its threshold may go either
way in FP32: the oracle recomputes the gradient with each such decision
inverted on its own, and the sum of the resulting changes is added to the
tolerance of each element (decision_slack).
"""
import numpy as np
import pytest
import torch

from oracle import coolchic_ref as R
from paper_2605_02726_amd import workloads as wl

from gpu_util import (_oracle_grad, decision_slack, latent_flip_slack, outlier_indices, outliers,
                      param_flip_slack, segments, slack_outliers, unexplained_outliers)

pytestmark = pytest.mark.gpu

RTOL = 1e-5


def _encoder(mc, img, lam, seed, lat, par, precision="fp32"):
    from paper_2605_02726_amd.encoder import Encoder
    return Encoder(mc, torch.from_numpy(img), lam, seed, lat, par, precision=precision)


def _with_conv(mc):
    mc.ups_conv = 1
    return mc


CASES = {
    # name: (config, H, W, image seed, random state?)
    "small_init": (wl.config_small, 64, 64, 1, False),
    "small_random": (wl.config_small, 64, 64, 11, True),
    "hop_128x192_random": (wl.config_hop, 128, 192, 12, True),
    "tiny_64x32_random": (wl.config_tiny, 64, 32, 13, True),
    "hop_512x768_init": (wl.config_hop, 512, 768, 2, False),
    "hop_320x1088_random": (wl.config_hop, 320, 1088, 14, True),   # ragged against every tile
    # the 18 + 6 reading of the workload's ARM context (24-wide context)
    "hop_s18_128x192_random": (wl.config_hop_s18, 128, 192, 23, True),
    "hop_s18_512x768_init": (wl.config_hop_s18, 512, 768, 2, False),
    # hyperlatent grids (1/16 .. 1/64) feeding the IFCEs
    "hop_hyper_128x192_random": (wl.config_hop_hyper, 128, 192, 19, True),
    "hop_hyper_512x768_init": (wl.config_hop_hyper, 512, 768, 2, False),
    # Table II presets (with their hyperlatent grids)
    "LOP_64x128_random": (lambda: wl.config_preset("LOP"), 64, 128, 15, True),
    "MOP_64x128_random": (lambda: wl.config_preset("MOP"), 64, 128, 16, True),
    "HOP_64x128_random": (lambda: wl.config_preset("HOP"), 64, 128, 17, True),
    "VHOP_64x128_random": (lambda: wl.config_preset("VHOP"), 64, 128, 18, True),
    # upsampling Conv refinement (random taps; identity taps at init)
    "hop_conv_128x192_random": (wl.config_hop_conv, 128, 192, 20, True),
    "hop_conv_512x768_init": (wl.config_hop_conv, 512, 768, 2, False),
    "tiny_conv_64x32_random": (lambda: _with_conv(wl.config_tiny()), 64, 32, 21, True),
    # both: hyperlatent grids and the Conv refinement
    "hop_hyper_conv_128x192_random": (lambda: _with_conv(wl.config_hop_hyper()), 128, 192, 22, True),
}


def _state(case):
    mk, H, W, seed, rnd = CASES[case]
    mc = mk()
    img = wl.image_large(seed) if (H, W) == (512, 768) else wl.synth_image(H, W, seed)
    if rnd:
        lat = wl.random_latents(mc, H, W, seed, scale=2.0)
        par = wl.init_params(mc, seed, arm_out_zero=False, conv_jitter=0.15)
    else:
        lat = np.zeros(wl.n_latents(mc, H, W), np.float32)
        par = wl.init_params(mc, seed)
    return mc, H, W, img, lat, par, seed


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("quant", ["soft", "hard"])
def test_first_step_gradient_and_totals(case, quant):
    mc, H, W, img, lat, par, seed = _state(case)
    lam, t, T, sigma = 1e-3, 1, 0.35, 0.22
    enc = _encoder(mc, img, lam, seed, lat, par)
    loss, bits, mse = enc.step(t, 1e-2, T, sigma, quant=quant)
    g = enc.grad()
    ref = R.loss_and_grad(mc.as_dict(), H, W, np.concatenate([lat, par]).astype(np.float64),
                          img, lam, quant, T, sigma, seed, t)
    print(f"[{case}/{quant}] loss {loss:.9g} vs {ref[0]:.9g}; bits {bits:.9g} vs {ref[1]:.9g}; "
          f"mse {mse:.9g} vs {ref[2]:.9g}", flush=True)
    assert loss == pytest.approx(ref[0], rel=RTOL)
    assert bits == pytest.approx(ref[1], rel=RTOL)
    assert mse == pytest.approx(ref[2], rel=RTOL)
    gref = ref[3]
    theta = np.concatenate([lat, par]).astype(np.float64)
    n_plain, worst = outliers(g, gref, RTOL, segments(mc, H, W))
    n_bad, n_near, n_used = 0, 0, 0
    if n_plain:   # only then are the decision slacks needed
        _, slack, n_near, n_used = decision_slack(mc, H, W, theta, img, lam, quant, T, sigma,
                                                  seed, t)
        n_bad, worst = slack_outliers(g, gref, slack, RTOL, segments(mc, H, W))
    print(f"[{case}/{quant}] gradient: {n_plain} of {g.size} outside the plain rule; {n_near} "
          f"near-threshold decisions ({n_used} flipped one by one); {n_bad} outside with their "
          f"slack; worst {worst}", flush=True)
    assert n_bad == 0


@pytest.mark.parametrize("case", ["small_random", "hop_128x192_random"])
def test_adam_update_matches_oracle(case):
    """After one step the new latents/parameters and moments follow Adam of
    the oracle gradient.  Adam's first step moves every coordinate by about
    lr * sign(g), so coordinates whose oracle gradient is below the gradient
    tolerance may legitimately move the other way: they are allowed 2 lr."""
    mc, H, W, img, lat, par, seed = _state(case)
    lam, lr = 1e-3, 1e-2
    enc = _encoder(mc, img, lam, seed, lat, par)
    enc.step(1, lr, 0.35, 0.22)
    st = enc.get_state()
    ost = R.OracleState(mc.as_dict(), H, W, img, lam, seed, lat, par)
    ost.step(1, lr, 0.35, 0.22)
    got = np.concatenate([st["latents"], st["params"]]).astype(np.float64)
    g = ost.last_grad
    segs = segments(mc, H, W)
    # gradient tolerance per element (rule + decision slack), then its image
    # through the first Adam step lr g / (|g| + eps), plus FP32 rounding of
    # the update; where the tolerance reaches |g| the sign itself is open
    tol = np.zeros_like(g)
    for _, sl in segs:
        rms = np.sqrt(np.mean(g[sl] ** 2))
        tol[sl] = RTOL * (np.abs(g[sl]) + rms)
    eps = 1e-8
    open_sign = tol >= np.abs(g)
    _, slack, _, _ = decision_slack(mc, H, W, np.concatenate([lat, par]).astype(np.float64), img,
                                    lam, "soft", 0.35, 0.22, seed, 1)
    # a decision slack on the gradient opens the sign like a small gradient does
    open_sign |= slack >= np.abs(g)
    # |g/(|g|+eps) - g'/(|g'|+eps)| for same-sign g, g' with |g - g'| <= delta
    delta = tol + slack
    lo = np.maximum(np.abs(g) - delta, 0.0)
    bound = np.where(open_sign, 2 * lr,
                     lr * eps * delta / ((np.abs(g) + eps) * (lo + eps)) +
                     2.4e-7 * (np.abs(ost.theta) + lr))
    err = np.abs(got - ost.theta)
    bad = np.nonzero(err > bound)[0]
    print(f"[{case}] open-sign fraction {float(np.mean(open_sign)):.2e}; {len(bad)} outside: "
          f"{[(int(i), float(err[i]), float(bound[i])) for i in bad[:5]]}", flush=True)
    assert len(bad) == 0
    m_ref = ost.m
    m_tol = 1e-5 * (np.abs(m_ref) + float(np.sqrt(np.mean(m_ref ** 2)))) + 0.1 * slack + 1e-12
    assert np.all(np.abs(st["m"] - m_ref) <= m_tol)


@pytest.mark.parametrize("case", ["small_random", "hop_128x192_random", "tiny_64x32_random",
                                  "hop_conv_128x192_random"])
def test_rd_eval_and_decode(case):
    mc, H, W, img, lat, par, seed = _state(case)
    enc = _encoder(mc, img, 4e-3, seed, lat, par)
    rd = enc.rd_eval()
    xd = enc.decode().cpu().numpy()
    ost = R.OracleState(mc.as_dict(), H, W, img, 4e-3, seed, lat, par)
    ref = ost.rd_eval()
    xr = ost.decode()
    print(f"[{case}] bits {rd['bits']:.9g} vs {ref['bits']:.9g} psnr {rd['psnr']:.6f} vs "
          f"{ref['psnr']:.6f}", flush=True)
    for key in ("bits", "mse", "loss", "bpp"):
        assert rd[key] == pytest.approx(ref[key], rel=RTOL)
    assert rd["psnr"] == pytest.approx(ref["psnr"], abs=1e-4)
    rms = float(np.sqrt(np.mean(xr ** 2)))
    assert np.max(np.abs(xd - xr) / (np.abs(xr) + rms)) <= RTOL


def test_small_ten_step_trajectory():
    """The 64x64 workload: 10 iterations, constant lr 1e-2, T and sigma
    scheduled; per-step totals follow the oracle's own FP64 trajectory."""
    mc, H, W, img, lat, par, seed = _state("small_init")
    enc = _encoder(mc, img, 1e-3, seed, lat, par)
    ost = R.OracleState(mc.as_dict(), H, W, img, 1e-3, seed, lat, par)
    worst = 0.0
    for t in range(1, 11):
        _, T, s = R.schedule(t, 10)
        a = enc.step(t, 1e-2, T, s)
        b = ost.step(t, 1e-2, T, s)
        rel = max(abs(a[i] - b[i]) / abs(b[i]) for i in range(3))
        worst = max(worst, rel)
        print(f"t={t}: loss {a[0]:.9g} vs {b[0]:.9g} bits {a[1]:.9g} vs {b[1]:.9g} rel {rel:.2e}",
              flush=True)
    assert worst < 1e-4


def test_batch_equals_alone_bitwise():
    """Two images of different sizes stepped in one batched launch give the
    same bits as each stepped alone (per-image fixed-order reductions)."""
    from paper_2605_02726_amd.encoder import step_batch, step_params
    mc = wl.config_hop()
    shapes = [(64, 128, 21), (128, 64, 22)]
    alone, batch = [], []
    for H, W, s in shapes:
        img = wl.synth_image(H, W, s)
        lat = wl.random_latents(mc, H, W, s)
        par = wl.init_params(mc, s, arm_out_zero=False)
        alone.append(_encoder(mc, img, 1e-3, s, lat, par))
        batch.append(_encoder(mc, img, 1e-3, s, lat, par))
    for t in (1, 2, 3):
        ra = [e.step(t, 1e-2, 0.3, 0.2) for e in alone]
        rb = step_batch(batch, [step_params(t, 1e-2, 0.3, 0.2)] * 2)
        assert ra == rb
    for a, b in zip(alone, batch):
        sa, sb = a.get_state(), b.get_state()
        for k in ("latents", "params", "m", "v"):
            assert np.array_equal(sa[k], sb[k])


def test_deterministic_repeat():
    mc, H, W, img, lat, par, seed = _state("hop_128x192_random")
    outs = []
    for _ in range(2):
        enc = _encoder(mc, img, 1e-3, seed, lat, par)
        r = [enc.step(t, 1e-2, 0.3, 0.2) for t in (1, 2)]
        outs.append((r, enc.grad(), enc.get_state()["params"]))
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][2], outs[1][2])


def test_hard_stage_freezes_latents():
    mc, H, W, img, lat, par, seed = _state("small_random")
    enc = _encoder(mc, img, 1e-3, seed, lat, par)
    enc.step(1, 1e-2, 0.3, 0.2, quant="hard", update_latents=False)
    st = enc.get_state()
    assert np.array_equal(st["latents"], lat)
    assert not np.array_equal(st["params"], par)


def test_gpu_gradient_matches_finite_differences():
    """Central differences of the GPU's own FP64-reduced loss (same noise)
    against its hand-written gradient, on random decoder parameters."""
    mc, H, W, img, lat, par, seed = _state("hop_128x192_random")
    enc = _encoder(mc, img, 1e-2, seed, lat, par)
    enc.step(1, 0.0, 0.35, 0.22)          # lr 0: state unchanged, gradient kept
    g = enc.grad()
    st = enc.get_state()
    rng = np.random.default_rng(0)
    n_lat = enc.n_lat
    idx = rng.choice(enc.n_par, size=60, replace=False)
    ok, tried = 0, 0
    for i in idx:
        gi = float(g[n_lat + i])
        h = 1e-2 * max(1.0, abs(float(st["params"][i])))
        vals = []
        for sgn in (1, -1):
            p = st["params"].copy()
            p[i] += sgn * h
            enc.set_state(params=p)
            vals.append(enc.eval_loss(1, 0.35, 0.22)[0])
        enc.set_state(params=st["params"])
        fd = (vals[0] - vals[1]) / (2 * h)
        tried += 1
        if abs(fd - gi) <= 2e-2 * max(abs(fd), abs(gi)) + 1e-6:
            ok += 1
    print(f"FD agreement {ok}/{tried}", flush=True)
    assert ok >= 0.9 * tried


_LARGEST = {}


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_largest_serving_image(precision):
    """2048x2048, the largest side of the serving trace (4.2 Mpixel, 5.6 M
    latents), from a random state: totals and every gradient element against
    the oracle.  At this size about a thousand ReLU, clamp and floor
    decisions sit within rounding of their thresholds, too many to recompute
    the whole oracle once per decision.  Every latent element outside the
    per-element rule must lie inside the footprint of such a decision
    (`unexplained_outliers`; the footprints cover about 0.5% of grid 0) and
    hold the rule plus the first-order change those decisions can make to it
    (`latent_flip_slack`: each ARM decision's rate term recomputed with the
    decision inverted, synthesis ReLUs bounded through the largest upsampling
    weight), and every decoder-parameter element must hold the rule plus the
    first-order slack of those decisions (`param_flip_slack`).  FP32: rtol 1e-5, decisions
    within 3e-6 of the layer's rms; BF16: rtol 2e-2, decisions within 3e-5
    (the resolution of its split operands)."""
    mc = wl.config_hop()
    H = W = 2048
    seed = 21
    img = wl.synth_image(H, W, seed)
    lat = wl.random_latents(mc, H, W, seed, scale=2.0)
    par = wl.init_params(mc, seed, arm_out_zero=False)
    lam, t, T, sigma = 1e-3, 1, 0.35, 0.22
    enc = _encoder(mc, img, lam, seed, lat, par, precision=precision)
    loss, bits, mse = enc.step(t, 1e-2, T, sigma)
    g = enc.grad()
    theta = np.concatenate([lat, par]).astype(np.float64)
    if "ref" not in _LARGEST:     # one oracle run (~20 s, ~15 GB) serves both forms
        tot, cap = {}, {}
        gref, sites = _oracle_grad(mc, H, W, theta, img, lam, "soft", T, sigma, seed, t, 3e-5,
                                   set(), totals=tot, capture=cap)
        _LARGEST["ref"] = (tot, gref, sites, cap)
    tot, gref, sites, cap = _LARGEST["ref"]
    rtol, tol_tot = (RTOL, RTOL) if precision == "fp32" else (2e-2, 1e-3)
    if precision == "fp32":   # decisions within 3e-6 of the layer's rms
        sites = [e for e in sites if e[0] < 0.1]
    print(f"[2048x2048/{precision}] loss {loss:.9g} vs {tot['loss']:.9g}; bits {bits:.9g} vs "
          f"{tot['bits']:.9g}; mse {mse:.9g} vs {tot['mse']:.9g}", flush=True)
    assert loss == pytest.approx(tot["loss"], rel=tol_tot)
    assert bits == pytest.approx(tot["bits"], rel=tol_tot)
    assert mse == pytest.approx(tot["mse"], rel=tol_tot)
    segs = segments(mc, H, W)
    n_lat = enc.n_lat
    bad = outlier_indices(g, gref, rtol, segs)
    bad_lat = bad[bad < n_lat]
    left = unexplained_outliers(mc, H, W, bad_lat, sites)
    slack = np.zeros(g.size)
    # latents outside the rule: each must hold it plus the first-order change
    # that the near-threshold decisions around it can make
    for e, v in latent_flip_slack(mc, H, W, theta, lam, sites, cap, bad_lat).items():
        slack[e] = v
    lsegs = [sg for sg in segs if sg[1].start < n_lat]
    n_lat_bad, lworst = slack_outliers(g, gref, slack, rtol, lsegs)
    psegs = [sg for sg in segs if sg[1].start >= n_lat]
    n_par_bad, worst = slack_outliers(g, gref, slack, rtol, psegs)
    if n_par_bad:   # only then are the decisions' parameter terms needed
        slack[n_lat:] = param_flip_slack(mc, H, W, theta, lam, sites, cap)
        n_par_bad, worst = slack_outliers(g, gref, slack, rtol, psegs)
    print(f"[2048x2048/{precision}] {len(bad)} of {g.size} elements outside the rule, "
          f"{len(sites)} near-threshold decisions; latents outside every footprint: "
          f"{len(left)} {left[:8]}; latents outside rule + slack: {n_lat_bad} {lworst}; "
          f"parameters outside rule + slack: {n_par_bad} {worst}", flush=True)
    assert not left
    assert n_lat_bad == 0
    assert n_par_bad == 0
