"""A non-finite loss marks the state and every later call reports it.

The oracle's loss becomes NaN when any parameter or latent is NaN (a NaN
pre-activation stays NaN through its ReLU); the GPU step must report
CC_ENONFINITE on that step and on every call after it, until the state is
replaced through cc_set_state.
"""
import numpy as np
import pytest
import torch

from oracle import coolchic_ref as R
from paper_2605_02726_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _poisoned(mc, H, W, lat, par, where):
    lat, par = lat.copy(), par.copy()
    if where == "latent":
        lat[(H // 2) * W + W // 3] = np.nan
        return lat, par
    pos = 0
    for name, shape, _ in wl.param_spec(mc):
        if name == where:
            par[pos + 1] = np.nan
            return lat, par
        pos += int(np.prod(shape))
    raise KeyError(where)


# first ARM and synthesis layers (behind a ReLU), the ARM output bias (mu),
# an IFCE weight, an upsampling tap, a residual weight and one latent
WHERE = ["arm.0.w", "arm.2.b", "ifce.0.w", "ups.2", "syn.0.w", "res.1.w", "latent"]


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
@pytest.mark.parametrize("where", WHERE)
def test_nonfinite_is_reported_and_sticky(precision, where):
    from paper_2605_02726_amd._lib import CC_ENONFINITE, CCError
    from paper_2605_02726_amd.encoder import Encoder
    mc = wl.config_hop()
    H, W, seed = 64, 128, 41
    img = wl.synth_image(H, W, seed)
    lat = wl.random_latents(mc, H, W, seed)
    par = wl.init_params(mc, seed, arm_out_zero=False)
    lat_bad, par_bad = _poisoned(mc, H, W, lat, par, where)
    # the oracle's loss is not finite either
    ref = R.loss_and_grad(mc.as_dict(), H, W, np.concatenate([lat_bad, par_bad]).astype(np.float64),
                          img, 1e-3, "soft", 0.35, 0.22, seed, 2)
    assert not np.isfinite(ref[0])

    enc = Encoder(mc, torch.from_numpy(img), 1e-3, seed, lat, par, precision=precision)
    assert np.isfinite(enc.step(1, 1e-2, 0.35, 0.22)[0])
    enc.set_state(latents=lat_bad, params=par_bad)
    with pytest.raises(CCError) as e:
        enc.step(2, 1e-2, 0.35, 0.22)
    assert e.value.code == CC_ENONFINITE
    # the next calls report the stored error, synchronous or not
    for sync in (True, False):
        with pytest.raises(CCError) as e:
            enc.step(3, 1e-2, 0.35, 0.22, sync=sync)
        assert e.value.code == CC_ENONFINITE
    # a finite state clears it
    enc.set_state(latents=lat, params=par, m=np.zeros(enc.n_lat + enc.n_par, np.float32),
                  v=np.zeros(enc.n_lat + enc.n_par, np.float32))
    assert np.isfinite(enc.step(1, 1e-2, 0.35, 0.22)[0])
