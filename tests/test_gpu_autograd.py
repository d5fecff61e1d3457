"""torch.autograd.Function wrappers (ARM rate, upsampling, synthesis) with
hand-written HIP backward kernels, against the FP64 oracle's modules (value
and autograd gradient) and against central finite differences of the
wrappers' own forward.  Rule as in the step parity tests: per element
|gpu - oracle| <= 1e-5 (|oracle| + rms(oracle tensor)), values within 1e-5."""
import numpy as np
import pytest
import torch

from oracle import coolchic_ref as R
from paper_2605_02726_amd import workloads as wl

pytestmark = pytest.mark.gpu
RTOL = 1e-5
DT = torch.float64


def _case(mk=wl.config_hop, H=64, W=128, seed=41):
    mc = mk()
    rng = np.random.default_rng(seed)
    yhat = np.round(rng.normal(scale=2.0, size=wl.n_latents(mc, H, W))).astype(np.float32)
    yhat += rng.uniform(-0.4, 0.4, size=yhat.shape).astype(np.float32)   # training-like values
    par = wl.init_params(mc, seed, arm_out_zero=False, conv_jitter=0.15)
    return mc, H, W, yhat, par


def _close(a, b, name):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    rms = float(np.sqrt(np.mean(b * b))) if b.size else 0.0
    r = np.abs(a - b) / (RTOL * (np.abs(b) + rms) + 1e-300)
    print(f"{name}: worst ratio {float(r.max()):.3f}", flush=True)
    assert float(r.max()) <= 1.0, name


@pytest.mark.parametrize("mk", [wl.config_hop, wl.config_small, wl.config_hop_conv])
def test_modules_match_oracle(mk):
    from paper_2605_02726_amd.autograd import Modules, arm_rate, synthesis, upsample
    mc, H, W, yhat, par = _case(mk)
    cfg = mc.as_dict()
    mods = Modules(mc, H, W)
    y = torch.tensor(yhat, device="cuda", requires_grad=True)
    p = torch.tensor(par, device="cuda", requires_grad=True)
    # ARM rate
    bits = arm_rate(y, p, mods)
    bits.backward()
    gy, gp = y.grad.cpu().numpy(), p.grad.cpu().numpy()
    yo = torch.tensor(yhat.astype(np.float64), requires_grad=True)
    po = torch.tensor(par.astype(np.float64), requires_grad=True)
    P = R.unpack_params(cfg, po)
    bo, _, _ = R.rate_bits(cfg, P, R.split_latents(cfg, H, W, yo))
    bo.backward()
    assert float(bits) == pytest.approx(float(bo), rel=RTOL)
    _close(gy, yo.grad.numpy(), "arm d/dyhat")
    n_arm = sum(int(np.prod(s)) for n, s, _ in wl.param_spec(mc) if n.startswith(("arm.", "ifce.")))
    _close(gp[:n_arm], po.grad.numpy()[:n_arm], "arm d/dparams")
    assert np.all(gp[n_arm:] == 0)
    # upsampling + synthesis with an MSE head
    y.grad = None
    p.grad = None
    img = torch.tensor(wl.synth_image(H, W, 5), device="cuda")
    z = upsample(y, p, mods)
    x = synthesis(z, p, mods)
    loss = ((x - img) ** 2).mean()
    loss.backward()
    yo = torch.tensor(yhat.astype(np.float64), requires_grad=True)
    po = torch.tensor(par.astype(np.float64), requires_grad=True)
    P = R.unpack_params(cfg, po)
    zo = R.upsample(cfg, P, R.split_latents(cfg, H, W, yo))
    xo = R.synthesis(cfg, P, zo)
    lo = ((xo - torch.tensor(wl.synth_image(H, W, 5), dtype=DT)) ** 2).mean()
    lo.backward()
    _close(z.detach().cpu().numpy(), zo.detach().numpy(), "zhat")
    _close(x.detach().cpu().numpy(), xo.detach().numpy(), "xhat")
    assert float(loss) == pytest.approx(float(lo), rel=RTOL)
    _close(y.grad.cpu().numpy(), yo.grad.numpy(), "dist d/dyhat")
    _close(p.grad.cpu().numpy()[n_arm:], po.grad.numpy()[n_arm:], "ups+syn d/dparams")


@pytest.mark.parametrize("mk,H,W", [(wl.config_tiny, 40, 56), (wl.config_tiny, 8, 8),
                                    (wl.config_tiny, 24, 72), (wl.config_hop, 64, 1088),
                                    (lambda: wl.ModelConfig(L=8), 128, 384)])
def test_upsampling_forward_every_tile_shape(mk, H, W):
    """zhat of the upsampling forward (per-level launches over the fine
    levels, one workgroup per source grid for the coarse ones) against the
    oracle: images smaller than a 16 x 16 adjoint tile and ragged against it
    (L = 4), a wide strip (L = 7), and eight grids (L = 8)."""
    from paper_2605_02726_amd.autograd import Modules, upsample
    mc, H, W, yhat, par = _case(mk, H, W, seed=43)
    cfg = mc.as_dict()
    mods = Modules(mc, H, W)
    with torch.no_grad():
        z = upsample(torch.tensor(yhat, device="cuda"), torch.tensor(par, device="cuda"), mods)
    P = R.unpack_params(cfg, torch.tensor(par.astype(np.float64)))
    zo = R.upsample(cfg, P, R.split_latents(cfg, H, W, torch.tensor(yhat.astype(np.float64))))
    _close(z.cpu().numpy(), zo.numpy(), "zhat")


def test_module_gradients_match_finite_differences():
    """Central differences of the wrappers' own forward (FP32, evaluated in
    double from the GPU outputs) against their backward, on random
    coordinates of the decoder parameters."""
    from paper_2605_02726_amd.autograd import Modules, synthesis, upsample
    mc, H, W, yhat, par = _case()
    mods = Modules(mc, H, W)
    img = torch.tensor(wl.synth_image(H, W, 6), device="cuda")
    y = torch.tensor(yhat, device="cuda")
    p = torch.tensor(par, device="cuda", requires_grad=True)

    def f(pp):
        with torch.no_grad():
            x = synthesis(upsample(y, pp, mods), pp, mods)
            return float(((x.double() - img.double()) ** 2).sum())

    x = synthesis(upsample(y, p, mods), p, mods)
    ((x - img) ** 2).sum().backward()
    g = p.grad.cpu().numpy()
    rng = np.random.default_rng(3)
    n_arm = sum(int(np.prod(s)) for n, s, _ in wl.param_spec(mc) if n.startswith(("arm.", "ifce.")))
    idx = rng.choice(np.arange(n_arm, mods.n_par), size=40, replace=False)
    ok = 0
    for i in idx:
        h = 1e-2 * max(1.0, abs(float(par[i])))
        pp = torch.tensor(par, device="cuda")
        pp[i] += h
        fp = f(pp)
        pp[i] -= 2 * h
        fm = f(pp)
        fd = (fp - fm) / (2 * h)
        if abs(fd - g[i]) <= 1e-2 * max(abs(fd), abs(g[i])) + 1e-4:
            ok += 1
    print(f"FD agreement {ok}/{len(idx)}", flush=True)
    assert ok >= 0.9 * len(idx)
