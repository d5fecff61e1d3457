"""Seeded synthetic inputs for the Cool-chic encode step.

This module is the only code shared by the GPU path and its CPU checker: it
draws images, initial decoder parameters and serving traces from numpy PCG64
seeds.  It holds none of the method's arithmetic (no quantisation, entropy
model, upsampling or synthesis), imports nothing else from this package, and
is safe to import on a machine without a GPU.

The images stand in for the natural photographs of the Kodak and CLIC20
professional-validation sets used in the paper (Section VI-A), which are not
available here: a 1/f-spectrum Gaussian field gives the power-law spectrum of
natural images, and pasted constant-colour rectangles give sharp edges.

The flat parameter vector follows one documented order (shared interface, see
``param_spec``):

  ARM      for each layer: W [out, in] row-major, then b [out];
           then, with the ARM stabilizer, Ws [2, in], bs [2]
  IFCE     for grid k = 0 .. n_ifce_grids-1: W [F, L-k-1 + n_hyper], b [F]
  upsample for level j = 1 .. L-1: the 4 free taps (h0, h1, h2, h3) of the
           symmetric 8-tap kernel (h0 h1 h2 h3 h3 h2 h1 h0); then, with the
           Conv refinement, for level j = 1 .. L-1 the 4 free taps
           (c0, c1, c2, c3) of the symmetric 7-tap kernel (c3 c2 c1 c0 c1 c2 c3)
  synthesis for each 1x1 layer: W [out, in], b [out];
           then, with the synthesis stabilizer, Ws [3, L], bs [3];
           then for each residual 3x3 layer: W [3, 3, 3, 3] (out, in, ky, kx), b [3]
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import List

import numpy as np

# Keys cubic kernel (a = -0.75) sampled at distances 1.75, 1.25, 0.75, 0.25:
# the bicubic interpolation taps for a factor-2 upsampling, used to initialise
# every learned upsampling level.  All four values are exact dyadic fractions.
BICUBIC_TAPS = (-0.03515625, -0.10546875, 0.26171875, 0.87890625)
# Free taps (c0, c1, c2, c3) of the optional 7-tap upsampling Conv at start:
# the identity filter.
IDENTITY_CONV_TAPS = (1.0, 0.0, 0.0, 0.0)


@dataclass
class ModelConfig:
    """Decoder shape (Table II of the paper gives the named presets)."""
    L: int = 7                      # number of latent grids (1/1 .. 1/2^(L-1))
    n_spatial: int = 16             # causal spatial neighbours s
    n_ifce_feat: int = 0            # inter-feature context size F
    n_ifce_grids: int = 0           # grids 0 .. n_ifce_grids-1 use an IFCE
    arm_hidden: List[int] = field(default_factory=lambda: [16, 16])
    arm_stab: int = 0
    syn_hidden: List[int] = field(default_factory=lambda: [24, 24])
    syn_stab: int = 0
    n_res: int = 1
    logscale_min: float = -4.6
    logscale_max: float = 5.0
    p_min: float = 2.0 ** -16
    n_hyper: int = 0                # hyperlatent grids, resolutions 1/2^b .. 1/2^(b+n_hyper-1)
    hyper_first: int = 4            # b
    ups_conv: int = 0               # 1: each upsampling level filters its input (7-tap Conv) first

    def as_dict(self):
        return asdict(self)


def config_small() -> ModelConfig:
    """64x64 workload: s=16 neighbours, no IFCE, ARM 16->16->16->2,
    synthesis 7->24->24->3 plus one residual 3x3 layer, no stabilizers."""
    return ModelConfig()


def config_hop() -> ModelConfig:
    """512x768 workload: s=24 spatial + F=6 inter-feature context on grids
    1/1, 1/2, 1/4; ARM 30->24->24->2 with stabilizer; synthesis 7->40->3 with
    stabilizer and two residual 3x3 layers (2,223 decoder parameters)."""
    return ModelConfig(L=7, n_spatial=24, n_ifce_feat=6, n_ifce_grids=3,
                       arm_hidden=[24, 24], arm_stab=1,
                       syn_hidden=[40], syn_stab=1, n_res=2)


def config_hop_s18() -> ModelConfig:
    """The other reading of the 512x768 workload's ARM: 18 spatial
    neighbours + F=6 inter-feature context, so that the context is 24 wide
    (ARM 24->24->24->2 with stabilizer); the rest as config_hop (2,067
    decoder parameters)."""
    c = config_hop()
    c.n_spatial = 18
    return c


# Table II presets for images below 10^6 pixels (7 latent grids, hyperlatent
# grids 1/16 .. 1/64): inter-feature context F on the 1/1, 1/2, 1/4 grids,
# spatial context s, two ARM hidden layers of the given width, one 1x1
# synthesis hidden layer, the number of 3x3 post-filters; both linear
# stabilizers.
PRESETS = {
    "LOP": dict(F=2, s=6, arm=8, syn=8, res=1),
    "MOP": dict(F=4, s=10, arm=10, syn=16, res=2),
    "HOP": dict(F=6, s=14, arm=20, syn=48, res=2),
    "VHOP": dict(F=6, s=20, arm=26, syn=64, res=2),
}


def config_preset(name: str, hyper: bool = True) -> ModelConfig:
    p = PRESETS[name]
    return ModelConfig(L=7, n_spatial=p["s"], n_ifce_feat=p["F"], n_ifce_grids=3,
                       arm_hidden=[p["arm"], p["arm"]], arm_stab=1,
                       syn_hidden=[p["syn"]], syn_stab=1, n_res=p["res"],
                       n_hyper=3 if hyper else 0, hyper_first=4)


def config_hop_hyper() -> ModelConfig:
    """The 512x768 workload's decoder with three hyperlatent grids (1/16,
    1/32, 1/64) feeding the IFCEs."""
    c = config_hop()
    c.n_hyper, c.hyper_first = 3, 4
    return c


def config_hop_conv() -> ModelConfig:
    """The 512x768 workload's decoder with the upsampling Conv refinement
    (6 levels x 4 more taps: 2,247 decoder parameters)."""
    c = config_hop()
    c.ups_conv = 1
    return c


def conv_taps_offsets(cfg: ModelConfig):
    """Offsets of every level's Conv taps in the decoder-parameter vector."""
    out, pos = [], 0
    for name, shape, _ in param_spec(cfg):
        if name.endswith(".conv"):
            out.append(pos)
        pos += int(np.prod(shape))
    return out


def config_tiny() -> ModelConfig:
    """A small shape with every feature switched on, for brute-force tests."""
    return ModelConfig(L=4, n_spatial=6, n_ifce_feat=2, n_ifce_grids=2,
                       arm_hidden=[5, 4], arm_stab=1, syn_hidden=[6],
                       syn_stab=1, n_res=2)


def param_spec(cfg: ModelConfig):
    """List of (name, shape, fan_in) in flat-vector order."""
    spec = []
    ctx = cfg.n_spatial + cfg.n_ifce_feat
    widths = [ctx] + list(cfg.arm_hidden) + [2]
    for i in range(len(widths) - 1):
        spec.append((f"arm.{i}.w", (widths[i + 1], widths[i]), widths[i]))
        spec.append((f"arm.{i}.b", (widths[i + 1],), widths[i]))
    if cfg.arm_stab:
        spec.append(("arm.stab.w", (2, ctx), ctx))
        spec.append(("arm.stab.b", (2,), ctx))
    for k in range(cfg.n_ifce_grids):
        nin = cfg.L - k - 1 + cfg.n_hyper
        spec.append((f"ifce.{k}.w", (cfg.n_ifce_feat, nin), nin))
        spec.append((f"ifce.{k}.b", (cfg.n_ifce_feat,), nin))
    for j in range(1, cfg.L):
        spec.append((f"ups.{j}", (4,), 0))
    if cfg.ups_conv:
        for j in range(1, cfg.L):
            spec.append((f"ups.{j}.conv", (4,), 0))
    widths = [cfg.L] + list(cfg.syn_hidden) + [3]
    for i in range(len(widths) - 1):
        spec.append((f"syn.{i}.w", (widths[i + 1], widths[i]), widths[i]))
        spec.append((f"syn.{i}.b", (widths[i + 1],), widths[i]))
    if cfg.syn_stab:
        spec.append(("syn.stab.w", (3, cfg.L), cfg.L))
        spec.append(("syn.stab.b", (3,), cfg.L))
    for r in range(cfg.n_res):
        spec.append((f"res.{r}.w", (3, 3, 3, 3), 27))
        spec.append((f"res.{r}.b", (3,), 27))
    return spec


def n_params(cfg: ModelConfig) -> int:
    return sum(int(np.prod(s)) for _, s, _ in param_spec(cfg))


def grid_levels(cfg: ModelConfig):
    """Resolution level of every grid of the flat latent pyramid: the L
    latent grids, then the hyperlatent grids."""
    return list(range(cfg.L)) + [cfg.hyper_first + i for i in range(cfg.n_hyper)]


def n_latents(cfg: ModelConfig, H: int, W: int) -> int:
    return sum((H >> k) * (W >> k) for k in grid_levels(cfg))


def init_params(cfg: ModelConfig, seed: int, arm_out_zero: bool = True,
                scale: float = 1.0, conv_jitter: float = 0.0) -> np.ndarray:
    """Seeded initial decoder parameters (float32).

    Weights and biases ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in)) * scale; the last
    ARM layer (and the ARM stabilizer) are zero when ``arm_out_zero`` so that
    every latent starts with mu = 0 and log-scale = 0; upsampling taps start
    at the bicubic kernel, the upsampling Conv taps (if any) at the identity
    plus ``conv_jitter`` times standard normal draws.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    n_arm_layers = len(cfg.arm_hidden) + 1
    for name, shape, fan_in in param_spec(cfg):
        n = int(np.prod(shape))
        if name.startswith("ups."):
            if name.endswith(".conv"):
                taps = np.array(IDENTITY_CONV_TAPS) + (conv_jitter * rng.standard_normal(4)
                                                       if conv_jitter else 0.0)
            else:
                taps = np.array(BICUBIC_TAPS)
            out.append(taps.astype(np.float64))
            continue
        bound = scale / math.sqrt(fan_in)
        vals = rng.uniform(-bound, bound, size=n)
        if arm_out_zero and (name.startswith(f"arm.{n_arm_layers - 1}.")
                             or name.startswith("arm.stab.")):
            vals = np.zeros(n)
        out.append(vals)
    return np.concatenate(out).astype(np.float32)


def random_latents(cfg: ModelConfig, H: int, W: int, seed: int,
                   scale: float = 2.0) -> np.ndarray:
    """Seeded non-zero latents (float32) for tests that need a generic state."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (scale * rng.standard_normal(n_latents(cfg, H, W))).astype(np.float32)


def _one_over_f(rng, H, W):
    fy = np.fft.fftfreq(H)[:, None]
    fx = np.fft.fftfreq(W)[None, :]
    f = np.sqrt(fy * fy + fx * fx)
    xi = rng.standard_normal((H, W)) + 1j * rng.standard_normal((H, W))
    spec = xi / np.maximum(f, 1.0 / max(H, W))
    spec[0, 0] = 0.0
    z = np.real(np.fft.ifft2(spec))
    z = z - z.mean()
    return z / max(z.std(), 1e-12)


def synth_image(H: int, W: int, seed: int, n_rects: int = 0) -> np.ndarray:
    """[3, H, W] float32 in [0, 1]: a correlated-RGB 1/f field, optionally
    with ``n_rects`` constant-colour rectangles (sides U[16,128]) pasted in
    order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shared = _one_over_f(rng, H, W)
    img = np.empty((3, H, W))
    for c in range(3):
        img[c] = 0.5 + 0.25 * (0.8 * shared + 0.6 * _one_over_f(rng, H, W))
    for _ in range(n_rects):
        h = int(rng.integers(16, 129))
        w = int(rng.integers(16, 129))
        y0 = int(rng.integers(0, max(1, H - h + 1)))
        x0 = int(rng.integers(0, max(1, W - w + 1)))
        col = rng.uniform(0.0, 1.0, size=3)
        img[:, y0:y0 + h, x0:x0 + w] = col[:, None, None]
    return np.clip(img, 0.0, 1.0).astype(np.float32)


def image_small(seed: int = 1) -> np.ndarray:
    """64x64 RGB 1/f field."""
    return synth_image(64, 64, seed)


def image_large(seed: int = 2) -> np.ndarray:
    """512x768 RGB 1/f field with 32 pasted rectangles."""
    return synth_image(512, 768, seed, n_rects=32)


def batch_shapes(n: int = 16, seed: int = 100, lo: int = 256, hi: int = 1536,
                 step: int = 64):
    """Uneven image sizes for a batched encode: sides i.i.d. uniform over the
    multiples of ``step`` in [lo, hi]."""
    sides = np.arange(lo, hi + 1, step)
    rng = np.random.Generator(np.random.PCG64(seed))
    return [(int(rng.choice(sides)), int(rng.choice(sides))) for _ in range(n)]


@dataclass
class Request:
    rid: int
    arrival_s: float
    H: int
    W: int
    lam: float
    seed: int


def request_trace(n: int = 200, rate_hz: float = 8.0, seed: int = 7,
                  lo: int = 256, hi: int = 2048, step: int = 64,
                  lambdas=(1e-4, 4e-4, 1e-3, 4e-3)):
    """Poisson arrivals (exponential gaps of mean 1/rate_hz), sides uniform
    over multiples of ``step`` in [lo, hi], lambda uniform over ``lambdas``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sides = np.arange(lo, hi + 1, step)
    t = 0.0
    out = []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate_hz))
        out.append(Request(i, t, int(rng.choice(sides)), int(rng.choice(sides)),
                           float(rng.choice(lambdas)), 1000 + i))
    return out
