"""Pins of the oracle's optional upsampling Conv refinement (Section III-B:
the upsampling is built from symmetric separable convolutions and transposed
convolutions): the 7-tap filter against SciPy's 1-D convolution with
replicated edges, the identity taps against the plain upsampling, the
pyramid structure, constants under normalised taps, the gradient against
central differences, and the parameter layout of the quantiser and SOAP."""
import numpy as np
import pytest
import scipy.ndimage
import torch

from oracle import coolchic_ref as R
from oracle import nnq as Q
from oracle import soap as S
from paper_2605_02726_amd import workloads as wl

DT = torch.float64


def _k7(c):
    return np.array([c[3], c[2], c[1], c[0], c[1], c[2], c[3]])


@pytest.mark.parametrize("dim", [1, 2])
def test_conv1d_is_scipy_convolution_with_replicated_edges(dim):
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 9, 5))           # sides shorter and longer than the kernel
    c = rng.normal(size=4)
    got = R.conv1d(torch.tensor(x), R.conv_taps(torch.tensor(c)), dim).numpy()
    ref = scipy.ndimage.convolve1d(x, _k7(c), axis=dim, mode="nearest")
    assert np.allclose(got, ref, atol=1e-13)


def test_conv1d_on_a_single_sample_sums_the_taps():
    c = np.array([0.5, 0.2, -0.1, 0.05])
    x = torch.tensor([[[3.0]]], dtype=DT)
    got = float(R.conv1d(x, R.conv_taps(torch.tensor(c)), 2))
    assert got == pytest.approx(3.0 * (c[0] + 2 * (c[1] + c[2] + c[3])), rel=1e-15)


def _grids(cfg, H, W, seed):
    rng = np.random.default_rng(seed)
    return [torch.tensor(rng.normal(size=(h, w))) for h, w in R.grid_shapes(cfg, H, W)]


def test_identity_taps_reduce_to_the_plain_upsampling():
    plain = wl.config_tiny()
    conv = wl.config_tiny()
    conv.ups_conv = 1
    Pp = R.unpack_params(plain.as_dict(), torch.tensor(wl.init_params(plain, 1), dtype=DT))
    Pc = R.unpack_params(conv.as_dict(), torch.tensor(wl.init_params(conv, 1), dtype=DT))
    for j in range(1, plain.L):
        assert torch.equal(Pc[f"ups.{j}.conv"], torch.tensor([1.0, 0.0, 0.0, 0.0], dtype=DT))
    g = _grids(plain.as_dict(), 16, 24, 2)
    assert torch.equal(R.upsample(conv.as_dict(), Pc, g), R.upsample(plain.as_dict(), Pp, g))


def test_conv_pyramid_structure_and_constants():
    """zhat channel g is grid g taken through (Conv_j, then TConv_j) for
    j = g .. 1, with the Conv done by SciPy; taps with c0 + 2 (c1 + c2 + c3)
    = 1 and the bicubic transposed convolution keep constant grids constant."""
    mc = wl.config_tiny()
    mc.ups_conv = 1
    cfg = mc.as_dict()
    rng = np.random.default_rng(3)
    P = R.unpack_params(cfg, torch.tensor(wl.init_params(mc, 1), dtype=DT))
    for j in range(1, cfg["L"]):
        P[f"ups.{j}"][:] = torch.tensor(rng.normal(size=4))
        P[f"ups.{j}.conv"][:] = torch.tensor(rng.normal(size=4))
    grids = _grids(cfg, 16, 8, 4)
    z = R.upsample(cfg, P, grids)
    for g in range(cfg["L"]):
        t = grids[g].numpy()
        for j in range(g, 0, -1):
            k = _k7(P[f"ups.{j}.conv"].numpy())
            t = scipy.ndimage.convolve1d(scipy.ndimage.convolve1d(t, k, axis=0, mode="nearest"),
                                         k, axis=1, mode="nearest")
            u = R.up_taps(P[f"ups.{j}"])
            t = R.up1d(R.up1d(torch.tensor(t)[None], u, 1), u, 2)[0].numpy()
        assert np.allclose(z[g].numpy(), t, atol=1e-12)
    P = R.unpack_params(cfg, torch.tensor(wl.init_params(mc, 1), dtype=DT))
    for j in range(1, cfg["L"]):
        c = rng.normal(size=3) * 0.1
        P[f"ups.{j}.conv"][:] = torch.tensor([1.0 - 2.0 * c.sum(), *c])
    flat = [torch.full(s, 0.7, dtype=DT) for s in R.grid_shapes(cfg, 16, 8)]
    assert torch.allclose(R.upsample(cfg, P, flat), torch.full((cfg["L"], 16, 8), 0.7, dtype=DT),
                          atol=1e-12)


def test_gradient_of_the_conv_taps_matches_central_differences():
    mc = wl.config_tiny()
    mc.ups_conv = 1
    cfg = mc.as_dict()
    H = W = 16
    img = wl.synth_image(H, W, 5)
    rng = np.random.default_rng(5)
    par = wl.init_params(mc, 5, arm_out_zero=False).astype(np.float64)
    offs = wl.conv_taps_offsets(mc)
    for o in offs:
        par[o:o + 4] += rng.normal(size=4) * 0.2
    n_lat = wl.n_latents(mc, H, W)
    theta = np.concatenate([wl.random_latents(mc, H, W, 5, scale=1.5), par])
    _, _, _, g = R.loss_and_grad(cfg, H, W, theta, img, 0.01, "soft", 0.3, 0.2, 5, 3)
    noise = R.noise_pyramid(cfg, H, W, 5, 3)
    imgt = torch.tensor(img, dtype=DT)

    def f(th):
        with torch.no_grad():
            return float(R.forward(cfg, H, W, torch.tensor(th), imgt, 0.01, "soft", 0.3, 0.2,
                                   noise)["loss"])
    idx = [n_lat + o + t for o in offs for t in range(4)]
    for i in idx:
        h = 1e-6 * max(1.0, abs(theta[i]))
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        assert g[i] == pytest.approx((f(tp) - f(tm)) / (2 * h), rel=1e-5, abs=1e-9), i


def test_layout_quantiser_groups_and_soap_tensors():
    mc = wl.config_hop_conv()
    cfg = mc.as_dict()
    assert wl.n_params(mc) == 2247 == R.n_params(cfg)
    names = [n for n, _, _ in wl.param_spec(mc)]
    assert names == list(R.unpack_params(cfg, torch.zeros(R.n_params(cfg), dtype=DT)).keys())
    offs = wl.conv_taps_offsets(mc)
    assert offs == [offs[0] + 4 * i for i in range(mc.L - 1)]
    w, b = Q.groups(cfg)["ups"]
    assert set(range(offs[0], offs[0] + 24)) <= set(w.tolist()) and b.size == 0
    lay = S.tensors(cfg)
    assert [(n, s) for n, s, _ in lay] == [(n, tuple(s)) for n, s, _ in wl.param_spec(mc)]
