"""The decision footprints used to excuse FP32 outliers at large sizes
(tests/gpu_util.py: unexplained_outliers) are conservative: inverting one
near-threshold decision in the oracle changes latent-gradient elements only
inside that decision's footprint.  CPU only (oracle against itself)."""
import numpy as np
import pytest

from paper_2605_02726_amd import workloads as wl

from gpu_util import (_oracle_grad, outlier_indices, param_flip_slack, segments,
                      unexplained_outliers)


def test_single_flips_stay_inside_their_footprints():
    mc = wl.config_hop()
    H, W, seed = 128, 192, 12
    img = wl.synth_image(H, W, seed)
    lat = wl.random_latents(mc, H, W, seed, scale=2.0)
    par = wl.init_params(mc, seed, arm_out_zero=False)
    theta = np.concatenate([lat, par]).astype(np.float64)
    args = (mc, H, W, theta, img, 1e-3, "soft", 0.35, 0.22, seed, 1)
    # a wide threshold band, so that every kind of decision has candidates
    g0, sites = _oracle_grad(*args, 3e-3, set())
    n_lat = wl.n_latents(mc, H, W)
    segs = [sg for sg in segments(mc, H, W) if sg[1].start < n_lat]
    picked = {}
    for s in sorted(sites):
        kind = s[1][:2] if s[1][0] == "arm" else s[1][:1]
        picked.setdefault(kind, s)
    assert len(picked) >= 3, picked.keys()
    moved = 0
    for kind, site in picked.items():
        g1, _ = _oracle_grad(*args, 3e-3, {(site[1], site[2])})
        bad = outlier_indices(g1[:n_lat], g0[:n_lat], 1e-8, segs)   # FP64 order noise ~1e-9
        moved += len(bad) > 0
        left = unexplained_outliers(mc, H, W, bad, [site])
        print(kind, site, len(bad), "elements moved", flush=True)
        assert not left, (kind, site, left[:5])
    assert moved >= 3


def test_param_flip_slack_is_each_flips_exact_parameter_change():
    """For single inverted decisions of every kind, the per-position
    recomputation reproduces the full oracle's change of the decoder-parameter
    gradient (up to FP64 reduction order), except the upsampling taps, whose
    share it leaves out by construction."""
    mc = wl.config_hop()
    H, W, seed = 128, 192, 12
    img = wl.synth_image(H, W, seed)
    lat = wl.random_latents(mc, H, W, seed, scale=2.0)
    par = wl.init_params(mc, seed, arm_out_zero=False)
    theta = np.concatenate([lat, par]).astype(np.float64)
    args = (mc, H, W, theta, img, 1e-3, "soft", 0.35, 0.22, seed, 1)
    cap = {}
    g0, sites = _oracle_grad(*args, 3e-3, set(), capture=cap)
    n_lat = wl.n_latents(mc, H, W)
    ups = np.zeros(len(par), bool)
    pos = 0
    for name, shape, _ in wl.param_spec(mc):
        n = int(np.prod(shape))
        ups[pos:pos + n] = name.startswith("ups.")
        pos += n
    picked = {}
    for s in sorted(sites):
        kind = s[1][:2] if s[1][0] == "arm" else s[1][:1]
        picked.setdefault(kind, s)
    checked = 0
    for kind, site in picked.items():
        g1, _ = _oracle_grad(*args, 3e-3, {(site[1], site[2])})
        exact = np.abs(g1[n_lat:] - g0[n_lat:])
        est = param_flip_slack(mc, H, W, theta, 1e-3, [site], cap)
        scale = np.abs(g0[n_lat:]).max()
        err = np.abs(exact - est)[~ups].max()
        print(kind, site[1], f"max change {exact[~ups].max():.3e}, mismatch {err:.3e}", flush=True)
        assert err <= 1e-9 * scale
        checked += exact[~ups].max() > 1e-9 * scale
    assert checked >= 3


def test_latent_flip_slack_bounds_each_flips_latent_change():
    """For single inverted decisions of every kind, the latent-gradient slack
    equals the full oracle's change of every latent-gradient element for ARM
    decisions (the position's own rate term is the only one that moves) and
    bounds it for synthesis ReLUs (first order through the largest upsampling
    weight)."""
    from gpu_util import latent_flip_slack
    mc = wl.config_hop()
    H, W, seed = 128, 192, 12
    img = wl.synth_image(H, W, seed)
    lat = wl.random_latents(mc, H, W, seed, scale=2.0)
    par = wl.init_params(mc, seed, arm_out_zero=False)
    theta = np.concatenate([lat, par]).astype(np.float64)
    args = (mc, H, W, theta, img, 1e-3, "soft", 0.35, 0.22, seed, 1)
    cap = {}
    g0, sites = _oracle_grad(*args, 3e-3, set(), capture=cap)
    n_lat = wl.n_latents(mc, H, W)
    scale = np.abs(g0[:n_lat]).max()
    picked = {}
    for s in sorted(sites):
        kind = s[1][:2] if s[1][0] == "arm" else s[1][:1]
        picked.setdefault(kind, s)
    checked = 0
    for kind, site in picked.items():
        g1, _ = _oracle_grad(*args, 3e-3, {(site[1], site[2])})
        exact = np.abs(g1[:n_lat] - g0[:n_lat])
        elems = np.nonzero(exact > 1e-12 * scale)[0]
        est = latent_flip_slack(mc, H, W, theta, 1e-3, [site], cap, elems)
        e_arr = np.array([est[int(e)] for e in elems]) if len(elems) else np.zeros(0)
        x_arr = exact[elems]
        print(kind, site[1], f"{len(elems)} elements moved, max change {x_arr.max() if len(elems) else 0:.3e}, "
              f"max slack {e_arr.max() if len(elems) else 0:.3e}", flush=True)
        if site[1][0] == "syn":
            assert np.all(x_arr <= e_arr * (1 + 1e-3) + 1e-10 * scale)
        else:
            assert np.all(np.abs(x_arr - e_arr) <= 1e-9 * scale + 1e-6 * x_arr)
        checked += len(elems) > 0
    assert checked >= 3
