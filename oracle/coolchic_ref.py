"""Plain FP64 CPU oracle of one Cool-chic 5.0 encoding step.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this module; the product path never
does.  It shares no code with the GPU library: every formula below is written
from the paper's equations, in float64, with PyTorch CPU tensors and autograd
(autograd supplies the exact gradient of the written-out loss; library
primitives used as steps: matmul, 2-D convolution, tanh/exp/log).

Readings where the paper is silent (kept identical on the GPU side, written
independently there):
  * causal neighbours: the causal half-plane {dy < 0, or dy = 0 and dx < 0},
    ordered by (dy^2 + dx^2, dy, dx), first s kept; zero padding outside the
    grid;
  * IFCE: one linear layer with bias per grid k < n_ifce_grids; its input is
    the co-located value of every coarser grid j = k+1 .. L-1 after nearest
    upsampling, i.e. grid j at (y >> (j-k), x >> (j-k)), in ascending j,
    followed by every hyperlatent grid in the same way; F inter-feature slots
    are zero on the other grids;
  * hyperlatent grids (Section III-A.3): n_hyper extra grids of resolutions
    1/2^b ... 1/2^(b + n_hyper - 1) (b = hyper_first), placed after the L
    latent grids in the flat pyramid; the ARM codes them like the other grids
    (spatial context only, no IFCE of their own), the IFCEs take them as
    inputs, and the upsampling and synthesis never see them;
  * ARM output o = (mu, l) with l the log of the Laplace scale b,
    b = exp(clamp(l, logscale_min, logscale_max)); probability floor p_min;
  * the rate term of the loss is in bits per pixel: loss = MSE + lambda *
    R / (H W); MSE over the C x H x W values;
  * upsampling level j: symmetric 8-tap kernel (h0 h1 h2 h3 h3 h2 h1 h0) used
    as a stride-2 transposed convolution on rows then columns, replicate edge;
    T_{L-1} = yhat^(L-1), T_{j-1} = concat(yhat^(j-1), Up_j(T_j));
  * upsampling Conv refinement (optional, ups_conv = 1): before its
    transposed convolution, level j filters T_j with a symmetric separable
    7-tap kernel (c3 c2 c1 c0 c1 c2 c3) on rows then columns (stride 1,
    replicate edge, every channel), i.e. Up_j(T) = TConv_j(Conv_j(T)); its
    four taps follow the transposed convolutions' in the parameter vector,
    level by level, and start at (1, 0, 0, 0), the identity;
  * synthesis: ReLU after each hidden 1x1 layer, stabilizer added to the trunk
    output, then x <- x + Conv3x3(x) per residual layer (replicate padding,
    no activation);
  * hard quantisation rounds half to even; in the hard mode the backward pass
    treats the rounding as the identity (straight-through);
  * Adam: beta1 0.9, beta2 0.999, eps 1e-8, bias correction, one learning rate
    for latents and decoder parameters.
"""
from __future__ import annotations

import math
from typing import Dict, List, Sequence

import numpy as np
import torch
import torch.nn.functional as Fnn

from .philox import latent_noise

DT = torch.float64
LN2 = math.log(2.0)
BETA1, BETA2, EPS = 0.9, 0.999, 1e-8


# ---------------------------------------------------------------- shapes ----
def n_hyper(cfg: Dict) -> int:
    return int(cfg.get("n_hyper", 0))


def grid_levels(cfg: Dict):
    """Resolution level of every grid of the pyramid: the L latent grids
    0 .. L-1, then the hyperlatent grids b .. b + n_hyper - 1."""
    b = int(cfg.get("hyper_first", 0))
    return list(range(cfg["L"])) + [b + i for i in range(n_hyper(cfg))]


def grid_shapes(cfg: Dict, H: int, W: int):
    """A grid of level k has shape (H / 2^k, W / 2^k) (Section III-A.1, eq. 1,
    and Section III-A.3 for the hyperlatent grids)."""
    return [(H >> k, W >> k) for k in grid_levels(cfg)]


def ifce_inputs(cfg: Dict, k: int) -> int:
    """Inputs of the IFCE of grid k: the coarser latent grids and the
    hyperlatent grids."""
    return cfg["L"] - k - 1 + n_hyper(cfg)


def causal_offsets(s: int, radius: int = 8):
    """The first s causal neighbours (dy, dx) in decoding (raster) order."""
    cand = [(dy, dx) for dy in range(-radius, 1) for dx in range(-radius, radius + 1)
            if dy < 0 or (dy == 0 and dx < 0)]
    cand.sort(key=lambda o: (o[0] * o[0] + o[1] * o[1], o[0], o[1]))
    return cand[:s]


def unpack_params(cfg: Dict, flat) -> Dict[str, torch.Tensor]:
    """Split the flat parameter vector into named tensors (documented order:
    ARM layers, ARM stabilizer, IFCEs, upsampling taps, synthesis layers,
    synthesis stabilizer, residual layers)."""
    L = cfg["L"]
    ctx = cfg["n_spatial"] + cfg["n_ifce_feat"]
    shapes = []
    widths = [ctx] + list(cfg["arm_hidden"]) + [2]
    for i in range(len(widths) - 1):
        shapes += [(f"arm.{i}.w", (widths[i + 1], widths[i])), (f"arm.{i}.b", (widths[i + 1],))]
    if cfg["arm_stab"]:
        shapes += [("arm.stab.w", (2, ctx)), ("arm.stab.b", (2,))]
    for k in range(cfg["n_ifce_grids"]):
        shapes += [(f"ifce.{k}.w", (cfg["n_ifce_feat"], ifce_inputs(cfg, k))),
                   (f"ifce.{k}.b", (cfg["n_ifce_feat"],))]
    for j in range(1, L):
        shapes.append((f"ups.{j}", (4,)))
    if cfg.get("ups_conv", 0):
        for j in range(1, L):
            shapes.append((f"ups.{j}.conv", (4,)))
    widths = [L] + list(cfg["syn_hidden"]) + [3]
    for i in range(len(widths) - 1):
        shapes += [(f"syn.{i}.w", (widths[i + 1], widths[i])), (f"syn.{i}.b", (widths[i + 1],))]
    if cfg["syn_stab"]:
        shapes += [("syn.stab.w", (3, L)), ("syn.stab.b", (3,))]
    for r in range(cfg["n_res"]):
        shapes += [(f"res.{r}.w", (3, 3, 3, 3)), (f"res.{r}.b", (3,))]
    out, pos = {}, 0
    for name, shp in shapes:
        n = int(np.prod(shp))
        out[name] = flat[pos:pos + n].reshape(shp)
        pos += n
    if pos != flat.numel():
        raise ValueError(f"parameter vector has {flat.numel()} values, layout needs {pos}")
    return out


def n_params(cfg: Dict) -> int:
    """Number of decoder parameters, counted from the layer shapes."""
    L = cfg["L"]
    ctx = cfg["n_spatial"] + cfg["n_ifce_feat"]
    n = 0
    widths = [ctx] + list(cfg["arm_hidden"]) + [2]
    n += sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1))
    n += (2 * ctx + 2) if cfg["arm_stab"] else 0
    n += sum(cfg["n_ifce_feat"] * ifce_inputs(cfg, k) + cfg["n_ifce_feat"]
             for k in range(cfg["n_ifce_grids"]))
    n += 4 * (L - 1) * (2 if cfg.get("ups_conv", 0) else 1)   # TConv (and Conv) taps
    widths = [L] + list(cfg["syn_hidden"]) + [3]
    n += sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1))
    n += (3 * L + 3) if cfg["syn_stab"] else 0
    n += 84 * cfg["n_res"]
    return n


def split_latents(cfg: Dict, H: int, W: int, flat) -> List[torch.Tensor]:
    """Flat pyramid (grid 0 first, each grid row-major) -> list of 2-D grids."""
    out, pos = [], 0
    for h, w in grid_shapes(cfg, H, W):
        out.append(flat[pos:pos + h * w].reshape(h, w))
        pos += h * w
    return out


# ---------------------------------------------------------- quantisation ----
def softround(x, T: float):
    """s_T (Section IV-C, eq. softround)."""
    fl = torch.floor(x)
    d = x - fl - 0.5
    return fl + torch.tanh(d / T) / (2.0 * math.tanh(1.0 / (2.0 * T))) + 0.5


def q_train(y, T: float, sigma: float, noise):
    """Training proxy s_T(s_T(y) + n_sigma) (Section IV-C, eq. q-train)."""
    return softround(softround(y, T) + sigma * noise, T)


def q_hard(y):
    """Uniform scalar quantiser Q (Section IV-C); straight-through gradient."""
    return y + (torch.round(y) - y).detach()


def noise_pyramid(cfg, H, W, seed: int, t: int):
    return [torch.from_numpy(latent_noise(seed, t, k, h * w)).reshape(h, w)
            for k, (h, w) in enumerate(grid_shapes(cfg, H, W))]


# ---------------------------------------------------------- entropy model ---
def spatial_context(grid, offsets):
    """s_i: causal neighbours of every position of one grid, zero outside the
    grid (Section III-A.1).  Returns [h*w, s]."""
    h, w = grid.shape
    R = 8
    padded = Fnn.pad(grid[None, None], (R, R, R, 0))[0, 0]  # left, right, top, bottom
    cols = [padded[R + dy:R + dy + h, R + dx:R + dx + w].reshape(-1) for dy, dx in offsets]
    if not cols:
        return grid.new_zeros(h * w, 0)
    return torch.stack(cols, dim=1)


def ifce_input(cfg, grids, k: int):
    """r_i: co-located values of the coarser latent grids j = k+1..L-1, then
    of the hyperlatent grids, after nearest-neighbour upsampling to grid k
    (Sections III-A.2, III-A.3).  [h*w, ifce_inputs(cfg, k)]."""
    h, w = grids[k].shape
    ys = torch.arange(h)
    xs = torch.arange(w)
    levels = grid_levels(cfg)
    cols = []
    for j in list(range(k + 1, cfg["L"])) + list(range(cfg["L"], len(grids))):
        f = levels[j] - k
        cols.append(grids[j][(ys >> f)[:, None], (xs >> f)[None, :]].reshape(-1))
    return torch.stack(cols, dim=1)


def arm_context(cfg, P, grids, k: int):
    """c_i = concat(s_i, f_i) for every position of grid k."""
    s = spatial_context(grids[k], causal_offsets(cfg["n_spatial"]))
    F = cfg["n_ifce_feat"]
    if F == 0:
        return s
    if k < cfg["n_ifce_grids"]:
        r = ifce_input(cfg, grids, k)
        f = r @ P[f"ifce.{k}.w"].T + P[f"ifce.{k}.b"]
    else:
        f = s.new_zeros(s.shape[0], F)
    return torch.cat([s, f], dim=1)


def arm_mlp(cfg, P, c):
    """(mu, l) = f_psi(c): ReLU MLP plus the linear stabilizer (Sections
    III-A.1 and III-C)."""
    h = c
    n_layers = len(cfg["arm_hidden"]) + 1
    for i in range(n_layers):
        h = h @ P[f"arm.{i}.w"].T + P[f"arm.{i}.b"]
        if i < n_layers - 1:
            h = torch.relu(h)
    if cfg["arm_stab"]:
        h = h + c @ P["arm.stab.w"].T + P["arm.stab.b"]
    return h[:, 0], h[:, 1]


def laplace_cdf(x, mu, b):
    """CDF of Laplace(mu, b)."""
    d = x - mu
    lo = 0.5 * torch.exp(torch.clamp(d, max=0.0) / b)
    hi = 1.0 - 0.5 * torch.exp(-torch.clamp(d, min=0.0) / b)
    return torch.where(d < 0, lo, hi)


def laplace_bin_prob(yhat, mu, logscale, cfg):
    """p(yhat | c) = integral of the Laplace PDF over [yhat-1/2, yhat+1/2]
    (Section III-A.1, eq. laplace-distribution)."""
    b = torch.exp(torch.clamp(logscale, cfg["logscale_min"], cfg["logscale_max"]))
    return laplace_cdf(yhat + 0.5, mu, b) - laplace_cdf(yhat - 0.5, mu, b)


def latent_bits(yhat, mu, logscale, cfg):
    """-log2 of the bin probability, floored at p_min (rate, Section IV-A)."""
    p = laplace_bin_prob(yhat, mu, logscale, cfg)
    return -torch.log(torch.clamp(p, min=cfg["p_min"])) / LN2


def rate_bits(cfg, P, grids):
    """R = -log2 p(yhat) = sum over every latent of every grid (eq.
    factorized-probability).  Returns (total, per-grid list of per-position
    bits, per-grid (mu, l))."""
    total = 0.0
    per_grid, params = [], []
    for k in range(len(grids)):
        c = arm_context(cfg, P, grids, k)
        mu, ls = arm_mlp(cfg, P, c)
        bits = latent_bits(grids[k].reshape(-1), mu, ls, cfg)
        per_grid.append(bits)
        params.append((mu, ls))
        total = total + bits.sum()
    return total, per_grid, params


# -------------------------------------------------------------- synthesis ---
def up_taps(h):
    """8-tap symmetric kernel from its 4 free taps."""
    return torch.stack([h[0], h[1], h[2], h[3], h[3], h[2], h[1], h[0]])


def up1d(x, u, dim: int):
    """Stride-2 transposed convolution with the 8-tap kernel u along one axis,
    padding 3, replicate edge: out[o] = sum over taps t with o+3-t even of
    u[t] * x[clamp((o+3-t)/2, 0, n-1)]."""
    n = x.shape[dim]
    o = torch.arange(2 * n)
    out = 0.0
    for t in range(8):
        valid = ((o + 3 - t) % 2 == 0).to(DT)
        idx = torch.clamp(torch.div(o + 3 - t, 2, rounding_mode="floor"), 0, n - 1)
        g = torch.index_select(x, dim, idx)
        shape = [1] * x.dim()
        shape[dim] = 2 * n
        out = out + u[t] * valid.reshape(shape) * g
    return out


def conv_taps(c):
    """7-tap symmetric kernel (c3 c2 c1 c0 c1 c2 c3) from its 4 free taps."""
    return torch.stack([c[3], c[2], c[1], c[0], c[1], c[2], c[3]])


def conv1d(x, k, dim: int):
    """Stride-1 convolution with the 7-tap symmetric kernel k along one axis,
    replicate edge: out[o] = sum over a in -3..3 of k[a+3] x[clamp(o+a, 0, n-1)]."""
    n = x.shape[dim]
    o = torch.arange(n)
    out = 0.0
    for a in range(-3, 4):
        out = out + k[a + 3] * torch.index_select(x, dim, torch.clamp(o + a, 0, n - 1))
    return out


def upsample(cfg, P, grids):
    """zhat = f_upsilon(yhat), shape (L, H, W) (Section III-B); with the Conv
    refinement each level filters its input before the transposed
    convolution."""
    L = cfg["L"]
    T = grids[L - 1][None]
    for j in range(L - 1, 0, -1):
        if cfg.get("ups_conv", 0):
            k = conv_taps(P[f"ups.{j}.conv"])
            T = conv1d(conv1d(T, k, 1), k, 2)
        u = up_taps(P[f"ups.{j}"])
        T = up1d(up1d(T, u, 1), u, 2)
        T = torch.cat([grids[j - 1][None], T], dim=0)
    return T


def synthesis(cfg, P, z):
    """xhat = f_theta(zhat): 1x1 trunk + stabilizer, then residual 3x3 layers
    (Sections III-B and III-C)."""
    L, H, W = z.shape
    h = z.reshape(L, -1).T
    x0 = h
    n_layers = len(cfg["syn_hidden"]) + 1
    for i in range(n_layers):
        h = h @ P[f"syn.{i}.w"].T + P[f"syn.{i}.b"]
        if i < n_layers - 1:
            h = torch.relu(h)
    if cfg["syn_stab"]:
        h = h + x0 @ P["syn.stab.w"].T + P["syn.stab.b"]
    x = h.T.reshape(3, H, W)
    for r in range(cfg["n_res"]):
        xp = Fnn.pad(x[None], (1, 1, 1, 1), mode="replicate")
        x = x + Fnn.conv2d(xp, P[f"res.{r}.w"], P[f"res.{r}.b"])[0]
    return x


# ------------------------------------------------------------------ loss ----
def forward(cfg, H, W, theta, img, lam, quant: str, T=None, sigma=None, noise=None):
    """Rate-distortion cost D + lambda R / (H W) (Section IV-A, eq.
    training-loss).  theta = [latents, params] (float64).  Returns a dict."""
    n_lat = sum(h * w for h, w in grid_shapes(cfg, H, W))
    y = theta[:n_lat]
    P = unpack_params(cfg, theta[n_lat:])
    grids_y = split_latents(cfg, H, W, y)
    if quant == "soft":
        grids = [q_train(g, T, sigma, n) for g, n in zip(grids_y, noise)]
    elif quant == "hard":
        grids = [q_hard(g) for g in grids_y]
    else:
        raise ValueError(quant)
    bits, per_grid_bits, arm_out = rate_bits(cfg, P, grids)
    z = upsample(cfg, P, grids)
    xhat = synthesis(cfg, P, z)
    mse = torch.mean((xhat - img) ** 2)
    loss = mse + lam * bits / (H * W)
    return dict(loss=loss, bits=bits, mse=mse, xhat=xhat, zhat=z, grids=grids,
                per_grid_bits=per_grid_bits, arm_out=arm_out)


def loss_and_grad(cfg, H, W, theta_np, img_np, lam, quant, T=None, sigma=None,
                  seed=0, t=1):
    """Loss terms and d loss / d theta at theta (all float64 numpy)."""
    theta = torch.tensor(np.asarray(theta_np, dtype=np.float64), requires_grad=True)
    img = torch.tensor(np.asarray(img_np, dtype=np.float64))
    noise = noise_pyramid(cfg, H, W, seed, t) if quant == "soft" else None
    out = forward(cfg, H, W, theta, img, lam, quant, T, sigma, noise)
    out["loss"].backward()
    return (float(out["loss"].detach()), float(out["bits"].detach()),
            float(out["mse"].detach()), theta.grad.numpy().copy())


# ------------------------------------------------------------------ adam ----
def adam(theta, g, m, v, t: int, lr: float, mask=None):
    """One Adam update (Kingma and Ba) with bias correction; entries where
    mask is False keep theta, m and v (frozen latents in the hard stage)."""
    m2 = BETA1 * m + (1.0 - BETA1) * g
    v2 = BETA2 * v + (1.0 - BETA2) * g * g
    mh = m2 / (1.0 - BETA1 ** t)
    vh = v2 / (1.0 - BETA2 ** t)
    th2 = theta - lr * mh / (np.sqrt(vh) + EPS)
    if mask is not None:
        th2 = np.where(mask, th2, theta)
        m2 = np.where(mask, m2, m)
        v2 = np.where(mask, v2, v)
    return th2, m2, v2


class OracleState:
    """Encoder state: theta = [latents, params], Adam moments, last t."""

    def __init__(self, cfg, H, W, img, lam, seed, latents, params, optimizer="adam"):
        self.cfg, self.H, self.W = cfg, H, W
        # decoder-parameter optimiser: Adam, or SOAP (Section IV-B; oracle/soap.py)
        self.soap = None
        if optimizer == "soap":
            from .soap import SoapState
            self.soap = SoapState(cfg)
        elif optimizer != "adam":
            raise ValueError(optimizer)
        self.img = np.asarray(img, dtype=np.float64)
        self.lam, self.seed = float(lam), int(seed)
        self.n_lat = sum(h * w for h, w in grid_shapes(cfg, H, W))
        self.theta = np.concatenate([np.asarray(latents, np.float64),
                                     np.asarray(params, np.float64)])
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0
        self.last_grad = None

    def step(self, t: int, lr: float, T: float, sigma: float, quant="soft",
             update_latents=True):
        """One encoding iteration: quantisation proxy, rate + distortion,
        gradient, Adam (Sections IV-A to IV-D)."""
        loss, bits, mse, g = loss_and_grad(self.cfg, self.H, self.W, self.theta,
                                           self.img, self.lam, quant, T, sigma,
                                           self.seed, t)
        mask = None
        if not update_latents:
            mask = np.zeros(self.theta.shape, dtype=bool)
            mask[self.n_lat:] = True
        if self.soap is not None:
            # Adam on the latents, SOAP on the decoder parameters
            lat = np.zeros(self.theta.shape, dtype=bool)
            lat[:self.n_lat] = update_latents
            self.theta, self.m, self.v = adam(self.theta, g, self.m, self.v, t, lr, lat)
            self.theta[self.n_lat:] = self.soap.step(self.theta[self.n_lat:], g[self.n_lat:], lr)
        else:
            self.theta, self.m, self.v = adam(self.theta, g, self.m, self.v, t, lr, mask)
        self.t = t
        self.last_grad = g
        return loss, bits, mse

    def rd_eval(self):
        """Hard-quantised rate and distortion, no gradient."""
        with torch.no_grad():
            out = forward(self.cfg, self.H, self.W, torch.from_numpy(self.theta),
                          torch.from_numpy(self.img), self.lam, "hard")
        bits, mse = float(out["bits"]), float(out["mse"])
        return dict(bits=bits, bpp=bits / (self.H * self.W), mse=mse,
                    psnr=10.0 * math.log10(1.0 / mse) if mse > 0 else float("inf"),
                    loss=float(out["loss"]))

    def decode(self):
        """Decoded image: hard-quantised latents -> upsampling -> synthesis."""
        with torch.no_grad():
            th = torch.from_numpy(self.theta)
            P = unpack_params(self.cfg, th[self.n_lat:])
            grids = [torch.round(g) for g in split_latents(self.cfg, self.H, self.W, th[:self.n_lat])]
            return synthesis(self.cfg, P, upsample(self.cfg, P, grids)).numpy()


# ------------------------------------------------------------- schedules ----
def schedule(t: int, n_iter: int, lr0=1e-2, lr1=1e-5, T0=0.35, T1=0.08,
             s0=0.22, s1=0.15, cosine_lr=True):
    """Table I schedules mapped linearly onto an n_iter budget (t from 1):
    cosine learning rate lr0 -> lr1, linear temperature and noise std."""
    a = 0.0 if n_iter <= 1 else (t - 1) / (n_iter - 1)
    lr = lr1 + 0.5 * (lr0 - lr1) * (1.0 + math.cos(math.pi * a)) if cosine_lr else lr0
    return lr, T0 + (T1 - T0) * a, s0 + (s1 - s0) * a
