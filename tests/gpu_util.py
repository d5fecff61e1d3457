"""Helpers shared by the GPU parity tests (comparison rules, oracle runs)."""
import numpy as np
import torch

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


def outliers(a, b, rtol, segs, top=5):
    """Elements breaking |a-b| <= rtol (|b| + rms(b_segment)): their count
    and the worst few (ratio, segment, index, a, b)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ratio = np.zeros_like(b)
    names = np.empty(b.size, dtype=object)
    for name, sl in segs:
        bb = b[sl]
        if bb.size == 0:
            continue
        rms = float(np.sqrt(np.mean(bb * bb)))
        den = rtol * (np.abs(bb) + rms)
        ratio[sl] = np.abs(a[sl] - bb) / np.where(den > 0, den, 1e-300)
        names[sl] = name
    bad = np.nonzero(ratio > 1.0)[0]
    order = bad[np.argsort(-ratio[bad])][:top]
    return len(bad), [(float(ratio[i]), names[i], int(i), float(a[i]), float(b[i])) for i in order]





def _oracle_grad(mc, H, W, theta, img, lam, quant, T, sigma, seed, t, tau, flip):
    """Oracle loss gradient with chosen near-threshold decisions inverted.

    Decisions: ARM and synthesis ReLUs (pre-activation within tau * rms of the
    layer), ARM log-scale clamps (within tau of a bound), probability floors
    (within a relative 1e-4).  `flip` is a set of (tag, flat index) to invert;
    returns (gradient, list of (normalised distance, tag, index) of every
    near-threshold decision)."""
    import torch.nn.functional as Fnn
    cfg = mc.as_dict()
    th = torch.tensor(np.asarray(theta, np.float64), requires_grad=True)
    n_lat = sum((H >> k) * (W >> k) for k in range(mc.L))
    P = R.unpack_params(cfg, th[n_lat:])
    gy = R.split_latents(cfg, H, W, th[:n_lat])
    if quant == "soft":
        noise = R.noise_pyramid(cfg, H, W, seed, t)
        grids = [R.q_train(g, T, sigma, nz) for g, nz in zip(gy, noise)]
    else:
        grids = [R.q_hard(g) for g in gy]
    sites = []

    def mark(tag, dist, scale):
        d = (dist / scale).reshape(-1)
        idx = torch.nonzero(d < 1.0).reshape(-1)
        for i in idx.tolist():
            sites.append((float(d[i]), tag, i))
        m = torch.zeros(d.numel(), dtype=torch.bool)
        for (tg, i) in flip:
            if tg == tag:
                m[i] = True
        return m.reshape(dist.shape)

    def relu(x, tag):
        xd = x.detach()
        rms = float(torch.sqrt(torch.mean(xd * xd))) + 1e-300
        fl = mark(tag, xd.abs(), tau * rms)
        return torch.where(fl, torch.where(xd > 0, x * 0.0, x), torch.relu(x))

    bits = 0.0
    nl = len(mc.arm_hidden) + 1
    for k in range(mc.L):
        c = R.arm_context(cfg, P, grids, k)
        x = c
        for i in range(nl):
            x = x @ P[f"arm.{i}.w"].T + P[f"arm.{i}.b"]
            if i < nl - 1:
                x = relu(x, ("arm", k, i))
        if mc.arm_stab:
            x = x + c @ P["arm.stab.w"].T + P["arm.stab.b"]
        mu, ls = x[:, 0], x[:, 1]
        lsd = ls.detach()
        dist = torch.minimum((lsd - mc.logscale_min).abs(), (lsd - mc.logscale_max).abs())
        fl = mark(("clamp", k), dist, tau)
        inside = (lsd >= mc.logscale_min) & (lsd <= mc.logscale_max)
        lcl = torch.clamp(ls, mc.logscale_min, mc.logscale_max)
        lcl = torch.where(fl, torch.where(inside, lcl.detach(), ls), lcl)
        b = torch.exp(lcl)
        yk = grids[k].reshape(-1)
        p = R.laplace_cdf(yk + 0.5, mu, b) - R.laplace_cdf(yk - 0.5, mu, b)
        pd = p.detach()
        fl = mark(("floor", k), (pd / mc.p_min - 1.0).abs(), 1e-4)
        pc = torch.clamp(p, min=mc.p_min)
        pc = torch.where(fl, torch.where(pd >= mc.p_min, pc.detach(), p), pc)
        bits = bits + (-torch.log(pc) / R.LN2).sum()
    z = R.upsample(cfg, P, grids)
    h = z.reshape(mc.L, -1).T
    x0 = h
    ns = len(mc.syn_hidden) + 1
    for i in range(ns):
        h = h @ P[f"syn.{i}.w"].T + P[f"syn.{i}.b"]
        if i < ns - 1:
            h = relu(h, ("syn", i))
    if mc.syn_stab:
        h = h + x0 @ P["syn.stab.w"].T + P["syn.stab.b"]
    xh = h.T.reshape(3, H, W)
    for r in range(mc.n_res):
        xp = Fnn.pad(xh[None], (1, 1, 1, 1), mode="replicate")
        xh = xh + Fnn.conv2d(xp, P[f"res.{r}.w"], P[f"res.{r}.b"])[0]
    imgt = torch.tensor(np.asarray(img, np.float64))
    loss = torch.mean((xh - imgt) ** 2) + lam * bits / (H * W)
    loss.backward()
    return th.grad.numpy().copy(), sites


def decision_slack(mc, H, W, theta, img, lam, quant, T=None, sigma=None, seed=0, t=1,
                   tau=3e-6, max_sites=48):
    """Per-element slack for decisions that FP32 may take either way: the
    oracle gradient is recomputed with each near-threshold decision inverted
    on its own (the max_sites nearest ones), and the slack of an element is
    the sum over those decisions of |gradient change| (first-order union
    bound for any subset of them going the other way).
    Returns (plain gradient, slack, number of near decisions, number used)."""
    g0, sites = _oracle_grad(mc, H, W, theta, img, lam, quant, T, sigma, seed, t, tau, set())
    sites.sort(key=lambda e: e[0])
    slack = np.zeros_like(g0)
    used = sites[:max_sites]
    for _, tag, i in used:
        gi, _ = _oracle_grad(mc, H, W, theta, img, lam, quant, T, sigma, seed, t, tau, {(tag, i)})
        slack += np.abs(gi - g0)
    return g0, slack, len(sites), len(used)


def slack_outliers(g, gref, slack, rtol, segs, top=5):
    """Elements with |g - gref| > rtol (|gref| + rms(segment)) + slack."""
    a = np.asarray(g, np.float64)
    b = np.asarray(gref, np.float64)
    ratio = np.zeros_like(b)
    names = np.empty(b.size, dtype=object)
    for name, sl in segs:
        bb = b[sl]
        if bb.size == 0:
            continue
        rms = float(np.sqrt(np.mean(bb * bb)))
        den = rtol * (np.abs(bb) + rms) + slack[sl]
        ratio[sl] = np.abs(a[sl] - bb) / np.where(den > 0, den, 1e-300)
        names[sl] = name
    bad = np.nonzero(ratio > 1.0)[0]
    order = bad[np.argsort(-ratio[bad])][:top]
    return len(bad), [(float(ratio[i]), names[i], int(i), float(a[i]), float(b[i])) for i in order]
