"""Pins of the oracle's gradient (central finite differences in FP64), of its
Adam update (closed forms, Kingma and Ba), of rd_eval / decode and of the
schedules (Table I)."""
import math

import numpy as np
import pytest
import torch

from oracle import coolchic_ref as R
from oracle.philox import latent_noise
from paper_2605_02726_amd import workloads as wl

DT = torch.float64


def _loss_fn(cfg, H, W, img, lam, quant, T, sigma, seed, t):
    noise = R.noise_pyramid(cfg, H, W, seed, t) if quant == "soft" else None
    imgt = torch.tensor(img, dtype=DT)

    def f(theta_np):
        with torch.no_grad():
            return float(R.forward(cfg, H, W, torch.tensor(theta_np), imgt, lam, quant, T,
                                   sigma, noise)["loss"])
    return f


def _fd_check(mc, H, W, quant, n_coords, seed, lat_scale, lam=0.01, T=0.3, sigma=0.2):
    cfg = mc.as_dict()
    img = wl.synth_image(H, W, seed)
    theta = np.concatenate([wl.random_latents(mc, H, W, seed, scale=lat_scale),
                            wl.init_params(mc, seed, arm_out_zero=False, scale=1.5)]).astype(np.float64)
    if quant == "hard":
        # keep latents away from the rounding steps, where Q is flat
        n_lat = wl.n_latents(mc, H, W)
        theta[:n_lat] = np.round(theta[:n_lat]) + 0.25
    _, _, _, g = R.loss_and_grad(cfg, H, W, theta, img, lam, quant, T, sigma, seed, 3)
    f = _loss_fn(cfg, H, W, img, lam, quant, T, sigma, seed, 3)
    rng = np.random.default_rng(seed + 1)
    n_lat = wl.n_latents(mc, H, W)
    idx = rng.choice(len(theta), size=min(n_coords, len(theta)), replace=False)
    if quant == "hard":
        idx = idx[idx >= n_lat]    # hard rounding has no useful latent derivative
    checked = 0
    for i in idx:
        fds = []
        for h in (1e-6 * max(1.0, abs(theta[i])), 2.5e-7 * max(1.0, abs(theta[i]))):
            tp, tm = theta.copy(), theta.copy()
            tp[i] += h
            tm[i] -= h
            fds.append((f(tp) - f(tm)) / (2 * h))
        fd = fds[1]
        # two step sizes that disagree reveal a kink (ReLU, clamp, floor,
        # probability floor) within reach of the stencil: skip the coordinate
        if abs(fds[0] - fds[1]) > 2e-6 * max(1.0, abs(fd)) + 1e-8:
            continue
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-8), f"coordinate {i}"
        checked += 1
    assert checked >= 0.8 * len(idx)


@pytest.mark.parametrize("quant", ["soft", "hard"])
def test_gradient_matches_central_differences_tiny(quant):
    _fd_check(wl.config_tiny(), 16, 16, quant, 400, 3, lat_scale=2.0)


@pytest.mark.parametrize("quant", ["soft", "hard"])
def test_gradient_matches_central_differences_small(quant):
    _fd_check(wl.config_small(), 64, 64, quant, 120, 4, lat_scale=1.5)


def test_gradient_matches_central_differences_hop_shape():
    # the 512x768 layer shapes on a 64x64 image (IFCE + both stabilizers)
    _fd_check(wl.config_hop(), 64, 64, "soft", 120, 5, lat_scale=1.5)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    th = rng.normal(size=100)
    g = rng.normal(size=100) * np.logspace(-6, 2, 100)
    th2, m, v = R.adam(th, g, np.zeros(100), np.zeros(100), 1, 0.01)
    assert np.allclose(th2, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_second_step_closed_form_and_mask():
    g1, g2, th = 0.3, -0.7, 1.0
    th1, m1, v1 = R.adam(np.array([th]), np.array([g1]), np.zeros(1), np.zeros(1), 1, 0.1)
    th2, m2, v2 = R.adam(th1, np.array([g2]), m1, v1, 2, 0.1)
    mh = (0.09 * g1 + 0.1 * g2) / (1 - 0.81)
    vh = (0.999 * 0.001 * g1 * g1 + 0.001 * g2 * g2) / (1 - 0.999 ** 2)
    assert th2[0] == pytest.approx(th1[0] - 0.1 * mh / (math.sqrt(vh) + 1e-8), rel=1e-13)
    mask = np.array([False, True])
    t3, m3, v3 = R.adam(np.array([1.0, 2.0]), np.array([5.0, 5.0]), np.zeros(2), np.zeros(2),
                        1, 0.1, mask)
    assert t3[0] == 1.0 and m3[0] == 0.0 and v3[0] == 0.0 and t3[1] != 2.0


def test_state_step_decreases_loss_and_freezes_latents():
    mc = wl.config_small()
    H = W = 64
    st = R.OracleState(mc.as_dict(), H, W, wl.image_small(1), 1e-3, 1,
                       np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, 1))
    losses = [st.step(t, 1e-2, 0.3, 0.2)[0] for t in range(1, 6)]
    assert losses[-1] < losses[0]
    lat = st.theta[:st.n_lat].copy()
    st.step(6, 1e-2, 0.3, 0.2, quant="hard", update_latents=False)
    assert np.array_equal(st.theta[:st.n_lat], lat)


def test_decode_equals_hard_forward_synthesis():
    mc = wl.config_hop()
    cfg = mc.as_dict()
    H, W = 64, 128
    st = R.OracleState(cfg, H, W, wl.synth_image(H, W, 3), 1e-3, 3,
                       wl.random_latents(mc, H, W, 3), wl.init_params(mc, 3, arm_out_zero=False))
    out = R.forward(cfg, H, W, torch.from_numpy(st.theta), torch.from_numpy(st.img), 1e-3, "hard")
    assert np.array_equal(st.decode(), out["xhat"].detach().numpy())
    rd = st.rd_eval()
    assert rd["loss"] == pytest.approx(rd["mse"] + 1e-3 * rd["bits"] / (H * W), rel=1e-14)
    assert rd["psnr"] == pytest.approx(-10 * math.log10(rd["mse"]))


def test_soft_noise_enters_through_q_train():
    """The training loss at sigma = 0 equals the loss of the noise-free proxy;
    with noise it differs, and the same (seed, t) reproduces it exactly."""
    mc = wl.config_tiny()
    cfg = mc.as_dict()
    H = W = 16
    img = wl.synth_image(H, W, 8)
    theta = np.concatenate([wl.random_latents(mc, H, W, 8), wl.init_params(mc, 8, arm_out_zero=False)])
    a = R.loss_and_grad(cfg, H, W, theta, img, 0.01, "soft", 0.3, 0.0, 8, 1)[0]
    b = R.loss_and_grad(cfg, H, W, theta, img, 0.01, "soft", 0.3, 0.2, 8, 1)[0]
    c = R.loss_and_grad(cfg, H, W, theta, img, 0.01, "soft", 0.3, 0.2, 8, 1)[0]
    d = R.loss_and_grad(cfg, H, W, theta, img, 0.01, "soft", 0.3, 0.2, 8, 2)[0]
    assert a != b and b == c and b != d
    n = latent_noise(8, 1, 0, 256)
    assert np.array_equal(R.noise_pyramid(cfg, H, W, 8, 1)[0].reshape(-1).numpy(), n)


def test_schedule_endpoints():
    lr, T, s = R.schedule(1, 1000)
    assert (lr, T, s) == (1e-2, 0.35, 0.22)
    lr, T, s = R.schedule(1000, 1000)
    assert lr == pytest.approx(1e-5) and T == pytest.approx(0.08) and s == pytest.approx(0.15)
    lr, _, _ = R.schedule(500, 999)
    assert lr == pytest.approx(0.5 * (1e-2 + 1e-5))
