"""Helpers shared by the GPU parity tests (comparison rules, oracle runs)."""
import numpy as np

from oracle import coolchic_ref as R
from paper_2605_02726_amd import workloads as wl


def segments(mc, H, W):
    """(name, slice) of theta = [latents, params]: one entry per latent grid
    and per parameter tensor."""
    out = []
    pos = 0
    for k in range(mc.L):
        n = (H >> k) * (W >> k)
        out.append((f"grid{k}", slice(pos, pos + n)))
        pos += n
    for name, shape, _ in wl.param_spec(mc):
        n = int(np.prod(shape))
        out.append((name, slice(pos, pos + n)))
        pos += n
    return out


def mixed_excess(a, b, rtol, segs):
    """Largest |a - b| / (rtol (|b| + rms(b_segment))) over all elements: the
    per-element rule |a-b| <= rtol |b| + rtol rms(segment) holds when <= 1.
    Returns (ratio, name of the worst segment, index)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    worst = (0.0, "", -1)
    for name, sl in segs:
        bb, aa = b[sl], a[sl]
        if bb.size == 0:
            continue
        rms = float(np.sqrt(np.mean(bb * bb)))
        den = rtol * (np.abs(bb) + rms)
        den = np.where(den > 0, den, 1e-300)
        r = np.abs(aa - bb) / den
        i = int(np.argmax(r))
        if r[i] > worst[0]:
            worst = (float(r[i]), name, sl.start + i)
    return worst


def oracle_state(mc, H, W, img, lam, seed, latents, params):
    return R.OracleState(mc.as_dict(), H, W, img, lam, seed, latents, params)
