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
    for k, lev in enumerate(wl.grid_levels(mc)):
        n = (H >> lev) * (W >> lev)
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


def outlier_indices(a, b, rtol, segs):
    """Indices of every element breaking |a-b| <= rtol (|b| + rms(b_segment))."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    bad = []
    for _, sl in segs:
        bb = b[sl]
        if bb.size == 0:
            continue
        rms = float(np.sqrt(np.mean(bb * bb)))
        r = np.abs(a[sl] - bb) > rtol * (np.abs(bb) + rms)
        bad.append(np.nonzero(r)[0] + sl.start)
    return np.concatenate(bad) if bad else np.zeros(0, np.int64)


def footprint_rects(mc, H, W, site):
    """Conservative footprint of one near-threshold decision on the latent
    grids, as rectangles (grid, y0, y1, x0, x1), bounds inclusive:
      ARM ReLU, log-scale clamp, probability floor at grid k, position (y, x):
        grid k rows y-4..y, columns x-4..x+4 (the position and every causal
        neighbour its context reads), and the IFCE parents
        (y >> (j-k), x >> (j-k)) on the coarser grids j;
      synthesis ReLU at pixel (y, x): grid 0 at (y, x) +-1 and grid j >= 1
        within +-4 of (y >> j, x >> j) (j stride-2 upsamplings, each reading
        inputs within +-2 of half its output index, add up to less than 4)."""
    L = mc.L
    levels = wl.grid_levels(mc)
    _, tag, idx = site
    rects = []
    if tag[0] == "syn":
        p = idx // mc.syn_hidden[tag[1]]
        y, x = divmod(p, W)
        rects.append((0, y - 1, y + 1, x - 1, x + 1))
        for j in range(1, L):
            rects.append((j, (y >> j) - 4, (y >> j) + 4, (x >> j) - 4, (x >> j) + 4))
        return rects
    k = tag[1]
    pos = idx // mc.arm_hidden[tag[2]] if tag[0] == "arm" else idx
    y, x = divmod(pos, W >> levels[k])
    rects.append((k, y - 4, y, x - 4, x + 4))
    if k < mc.n_ifce_grids:
        for j in range(k + 1, len(levels)):
            f = levels[j] - k
            rects.append((j, y >> f, y >> f, x >> f, x >> f))
    return rects


def unexplained_outliers(mc, H, W, bad, sites):
    """Outlier elements that no near-threshold decision can reach (footprints
    of footprint_rects).  Decoder-parameter elements are never explained
    (every decision reaches them, so they are held to the plain rule).
    Returns the indices of `bad` that lie in no footprint."""
    levels = wl.grid_levels(mc)
    masks = [np.zeros((H >> lev, W >> lev), bool) for lev in levels]
    for site in sites:
        for (k, y0, y1, x0, x1) in footprint_rects(mc, H, W, site):
            h, w = masks[k].shape
            masks[k][max(y0, 0):min(y1, h - 1) + 1, max(x0, 0):min(x1, w - 1) + 1] = True
    starts = np.cumsum([0] + [(H >> lev) * (W >> lev) for lev in levels])
    out = []
    for e in np.asarray(bad).tolist():
        k = int(np.searchsorted(starts, e, side="right") - 1)
        if k >= len(levels):
            out.append(e)
            continue
        y, x = divmod(e - int(starts[k]), W >> levels[k])
        if not masks[k][y, x]:
            out.append(e)
    return out


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





def _oracle_grad(mc, H, W, theta, img, lam, quant, T, sigma, seed, t, tau, flip, totals=None,
                 capture=None):
    """Oracle loss gradient with chosen near-threshold decisions inverted.

    Decisions: ARM and synthesis ReLUs (pre-activation within tau * rms of the
    layer), ARM log-scale clamps (within tau of a bound), probability floors
    (within a relative 1e-4).  `flip` is a set of (tag, flat index) to invert;
    returns (gradient, list of (normalised distance, tag, index) of every
    near-threshold decision)."""
    import torch.nn.functional as Fnn
    cfg = mc.as_dict()
    th = torch.tensor(np.asarray(theta, np.float64), requires_grad=True)
    n_lat = wl.n_latents(mc, H, W)
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
    for k in range(len(grids)):
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
    if capture is not None:
        h.retain_grad()
    xh = h.T.reshape(3, H, W)
    for r in range(mc.n_res):
        xp = Fnn.pad(xh[None], (1, 1, 1, 1), mode="replicate")
        xh = xh + Fnn.conv2d(xp, P[f"res.{r}.w"], P[f"res.{r}.b"])[0]
    imgt = torch.tensor(np.asarray(img, np.float64))
    mse = torch.mean((xh - imgt) ** 2)
    loss = mse + lam * bits / (H * W)
    loss.backward()
    if totals is not None:
        totals.update(loss=float(loss), bits=float(bits), mse=float(mse))
    if capture is not None:   # for param_flip_slack and latent_flip_slack
        # d yhat / d y of every latent (elementwise; 1 for the hard rounding's
        # straight-through derivative)
        if quant == "soft":
            yd = th[:n_lat].detach().clone().requires_grad_(True)
            qs = [R.q_train(g, T, sigma, nz) for g, nz in zip(R.split_latents(cfg, H, W, yd), noise)]
            sum(q.sum() for q in qs).backward()
            dq = yd.grad.numpy().copy()
        else:
            dq = np.ones(n_lat)
        capture.update(grids=[g.detach() for g in grids], z=x0.detach(), go=h.grad.detach(), dq=dq)
    return th.grad.numpy().copy(), sites


def param_flip_slack(mc, H, W, theta, lam, sites, cap):
    """First-order bound of what near-threshold decisions can do to the
    decoder-parameter gradient, without one full oracle run per decision.

    A decision (ARM ReLU, log-scale clamp or probability floor at one latent
    position; synthesis ReLU at one pixel) changes only that position's own
    term of the parameter gradient, so the term is recomputed for that single
    position with the decision inverted (same inversion as _oracle_grad) and
    without, and the slack of a parameter is the sum over decisions of
    |change|.  `cap` comes from _oracle_grad(..., capture=cap): quantised
    grids, zhat per pixel and the gradient at the trunk output per pixel.
    Not included: what a changed pixel gradient does to the upsampling taps
    (one pixel's share of a tap gradient summed over a whole level)."""
    cfg = mc.as_dict()
    n_lat = wl.n_latents(mc, H, W)
    pt = torch.tensor(np.asarray(theta[n_lat:], np.float64), requires_grad=True)
    P = R.unpack_params(cfg, pt)
    grids = cap["grids"]
    offs = R.causal_offsets(mc.n_spatial)
    F, G, L = mc.n_ifce_feat, mc.n_ifce_grids, mc.L
    nl = len(mc.arm_hidden) + 1
    lmin, lmax, pmin = mc.logscale_min, mc.logscale_max, mc.p_min
    scale = lam / (H * W)

    def grad_of(v):
        g = torch.autograd.grad(v, pt, allow_unused=True)[0]
        return np.zeros(pt.numel()) if g is None else g.numpy()

    def inv_relu(x, u):
        xd = x.detach()
        m = torch.zeros_like(xd, dtype=torch.bool)
        m[0, u] = True
        return torch.where(m, torch.where(xd > 0, x * 0.0, x), torch.relu(x))

    def arm_term(k, pos, tag, u):
        gk = grids[k]
        h, w = gk.shape
        y, x = divmod(pos, w)
        s = torch.tensor([[float(gk[y + dy, x + dx]) if 0 <= y + dy < h and 0 <= x + dx < w
                           else 0.0 for dy, dx in offs]], dtype=torch.float64)
        c = s
        if F:
            if k < G:
                lev = wl.grid_levels(mc)
                r = torch.tensor([[float(grids[j][y >> (lev[j] - k), x >> (lev[j] - k)])
                                   for j in range(k + 1, len(grids))]], dtype=torch.float64)
                f = r @ P[f"ifce.{k}.w"].T + P[f"ifce.{k}.b"]
            else:
                f = s.new_zeros(1, F)
            c = torch.cat([s, f], dim=1)
        v = c
        for i in range(nl):
            v = v @ P[f"arm.{i}.w"].T + P[f"arm.{i}.b"]
            if i < nl - 1:
                v = inv_relu(v, u) if tag == ("arm", k, i) else torch.relu(v)
        if mc.arm_stab:
            v = v + c @ P["arm.stab.w"].T + P["arm.stab.b"]
        mu, ls = v[:, 0], v[:, 1]
        lcl = torch.clamp(ls, lmin, lmax)
        if tag == ("clamp", k):
            lsd = ls.detach()
            lcl = torch.where((lsd >= lmin) & (lsd <= lmax), lcl.detach(), ls)
        b = torch.exp(lcl)
        yk = gk.reshape(-1)[pos:pos + 1]
        p = R.laplace_cdf(yk + 0.5, mu, b) - R.laplace_cdf(yk - 0.5, mu, b)
        pc = torch.clamp(p, min=pmin)
        if tag == ("floor", k):
            pc = torch.where(p.detach() >= pmin, pc.detach(), p)
        return grad_of(scale * (-torch.log(pc) / R.LN2).sum())

    def syn_term(pix, tag, u):
        z = cap["z"][pix:pix + 1]
        v = z
        ns = len(mc.syn_hidden) + 1
        for i in range(ns):
            v = v @ P[f"syn.{i}.w"].T + P[f"syn.{i}.b"]
            if i < ns - 1:
                v = inv_relu(v, u) if tag == ("syn", i) else torch.relu(v)
        if mc.syn_stab:
            v = v + z @ P["syn.stab.w"].T + P["syn.stab.b"]
        return grad_of((v * cap["go"][pix:pix + 1]).sum())

    slack = np.zeros(pt.numel())
    for _, tag, idx in sites:
        if tag[0] == "syn":
            pix, u = divmod(idx, mc.syn_hidden[tag[1]])
            d = syn_term(pix, tag, u) - syn_term(pix, None, u)
        else:
            k = tag[1]
            pos, u = divmod(idx, mc.arm_hidden[tag[2]]) if tag[0] == "arm" else (idx, 0)
            d = arm_term(k, pos, tag, u) - arm_term(k, pos, None, u)
        slack += np.abs(d)
    return slack



def latent_flip_slack(mc, H, W, theta, lam, sites, cap, elems):
    """Per-element bound of what near-threshold decisions can do to the
    latent gradient, for the latent indices `elems` (the elements outside the
    plain rule), without one full oracle run per decision.

    ARM ReLU, log-scale clamp and probability-floor decisions at one latent
    position change only that position's rate term, whose gradient with
    respect to its inputs (the causal neighbours, the latent itself, the IFCE
    inputs) is recomputed with the decision inverted and without: exact to
    first order, times lambda / (H W) and d yhat / d y.  A synthesis ReLU at
    pixel p changes the gradient at the trunk input z(p) by dz (recomputed the
    same way); its share on a latent of grid c is bounded by |dz_c| times the
    largest weight of one grid-c latent in one upsampled pixel (an impulse
    through the oracle's upsampling, replicate edges included), times
    d yhat / d y.  Returns a dict {element: slack}."""
    cfg = mc.as_dict()
    n_lat = wl.n_latents(mc, H, W)
    P = {k: v.detach() for k, v in R.unpack_params(cfg, torch.tensor(np.asarray(theta[n_lat:], np.float64))).items()}
    grids = cap["grids"]
    dq = cap["dq"]
    levels = wl.grid_levels(mc)
    starts = np.cumsum([0] + [int(g.numel()) for g in grids])
    offs = R.causal_offsets(mc.n_spatial)
    F, G = mc.n_ifce_feat, mc.n_ifce_grids
    nl = len(mc.arm_hidden) + 1
    lmin, lmax, pmin = mc.logscale_min, mc.logscale_max, mc.p_min
    scale = lam / (H * W)
    want = set(int(e) for e in elems)
    out = {e: 0.0 for e in want}

    def where(e):
        k = int(np.searchsorted(starts, e, side="right") - 1)
        y, x = divmod(int(e - starts[k]), grids[k].shape[1])
        return k, y, x

    def in_footprint(site, e):
        k, y, x = where(e)
        return any(kk == k and y0 <= y <= y1 and x0 <= x <= x1
                   for (kk, y0, y1, x0, x1) in footprint_rects(mc, H, W, site))

    def arm_inputs_grad(k, pos, tag, u):
        gk = grids[k]
        h, w = gk.shape
        y, x = divmod(pos, w)
        idx, vals = [], []
        for dy, dx in offs:
            yy, xx = y + dy, x + dx
            inside = 0 <= yy < h and 0 <= xx < w
            idx.append(int(starts[k] + yy * w + xx) if inside else -1)
            vals.append(float(gk[yy, xx]) if inside else 0.0)
        ridx, rvals = [], []
        if F and k < G:
            for j in range(k + 1, len(grids)):
                sh = levels[j] - levels[k]
                yy, xx = y >> sh, x >> sh
                ridx.append(int(starts[j] + yy * grids[j].shape[1] + xx))
                rvals.append(float(grids[j][yy, xx]))
        s_t = torch.tensor([vals], dtype=torch.float64, requires_grad=True)
        own = torch.tensor([float(gk[y, x])], dtype=torch.float64, requires_grad=True)
        r_t = torch.tensor([rvals], dtype=torch.float64, requires_grad=True) if ridx else None
        c = s_t
        if F:
            f = (r_t @ P[f"ifce.{k}.w"].T + P[f"ifce.{k}.b"]) if r_t is not None else s_t.new_zeros(1, F)
            c = torch.cat([s_t, f], dim=1)
        v = c
        for i in range(nl):
            v = v @ P[f"arm.{i}.w"].T + P[f"arm.{i}.b"]
            if i < nl - 1:
                if tag == ("arm", k, i):
                    vd = v.detach()
                    m = torch.zeros_like(vd, dtype=torch.bool)
                    m[0, u] = True
                    v = torch.where(m, torch.where(vd > 0, v * 0.0, v), torch.relu(v))
                else:
                    v = torch.relu(v)
        if mc.arm_stab:
            v = v + c @ P["arm.stab.w"].T + P["arm.stab.b"]
        mu, ls = v[:, 0], v[:, 1]
        lcl = torch.clamp(ls, lmin, lmax)
        if tag == ("clamp", k):
            lsd = ls.detach()
            lcl = torch.where((lsd >= lmin) & (lsd <= lmax), lcl.detach(), ls)
        b = torch.exp(lcl)
        p = R.laplace_cdf(own + 0.5, mu, b) - R.laplace_cdf(own - 0.5, mu, b)
        pc = torch.clamp(p, min=pmin)
        if tag == ("floor", k):
            pc = torch.where(p.detach() >= pmin, pc.detach(), p)
        term = scale * (-torch.log(pc) / R.LN2).sum()
        leaves = [s_t, own] + ([r_t] if r_t is not None else [])
        grads = torch.autograd.grad(term, leaves, allow_unused=True)
        res = {}
        for ids, gr in zip([idx, [int(starts[k] + pos)], ridx], grads):
            if gr is None:
                continue
            for e, gv in zip(ids, gr.reshape(-1).tolist()):
                if e >= 0:
                    res[e] = res.get(e, 0.0) + gv
        return res

    def syn_dz(pix, tag, u):
        z = cap["z"][pix:pix + 1].clone().requires_grad_(True)
        v = z
        ns = len(mc.syn_hidden) + 1
        for i in range(ns):
            v = v @ P[f"syn.{i}.w"].T + P[f"syn.{i}.b"]
            if i < ns - 1:
                if tag == ("syn", i):
                    vd = v.detach()
                    m = torch.zeros_like(vd, dtype=torch.bool)
                    m[0, u] = True
                    v = torch.where(m, torch.where(vd > 0, v * 0.0, v), torch.relu(v))
                else:
                    v = torch.relu(v)
        if mc.syn_stab:
            v = v + z @ P["syn.stab.w"].T + P["syn.stab.b"]
        return torch.autograd.grad((v * cap["go"][pix:pix + 1]).sum(), z)[0].reshape(-1)

    wmax = None
    for site in sites:
        _, tag, i = site
        cover = [e for e in want if in_footprint(site, e)]
        if not cover:
            continue
        if tag[0] == "syn":
            if wmax is None:
                # largest weight of one latent of grid c in one upsampled pixel,
                # over impulses at a corner, an edge and the interior
                # (the same taps on a small 256x256 pyramid: the weights do not
                # depend on the image size)
                wmax = np.zeros(mc.L)
                hs = [(256 >> lev, 256 >> lev) for lev in levels]
                for c in range(mc.L):
                    for (yy, xx) in ((0, 0), (0, hs[c][1] // 2), (hs[c][0] // 2, hs[c][1] // 2)):
                        imp = [torch.zeros(sh, dtype=torch.float64) for sh in hs]
                        imp[c][yy, xx] = 1.0
                        zc = R.upsample(cfg, P, imp)
                        wmax[c] = max(wmax[c], float(zc[c].abs().max()))
            pix, u = divmod(i, mc.syn_hidden[tag[1]])
            d = (syn_dz(pix, tag, u) - syn_dz(pix, None, u)).abs().numpy()
            for e in cover:
                k, _, _ = where(e)
                if k < mc.L:
                    out[e] += float(d[k]) * wmax[k] * abs(float(dq[e]))
            continue
        k = tag[1]
        pos, u = divmod(i, mc.arm_hidden[tag[2]]) if tag[0] == "arm" else (i, 0)
        a = arm_inputs_grad(k, pos, tag, u)
        b = arm_inputs_grad(k, pos, None, u)
        for e in cover:
            out[e] += abs(a.get(e, 0.0) - b.get(e, 0.0)) * abs(float(dq[e]))
    return out

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


def fp32_eval_slack(mc, H, W, theta, img, lam, quant, T, sigma, seed, t, segs):
    """Resolution of FP32 arithmetic at this state: the oracle's own formulas
    evaluated in float32 (PyTorch CPU, same code, every tensor float32) against
    float64, as the largest deviation within each tensor of theta.  At
    trained states the Laplace rate at small scales b amplifies the rounding
    of mu, l and the context by 1/b, and sums with strong cancellation keep
    only the rounding of their terms, so an FP32 implementation of the exact
    arithmetic cannot hold 1e-5 there; this is the per-tensor slack such an
    implementation needs (applied only to elements outside the plain rule)."""
    cfg = mc.as_dict()

    def grad(dt):
        old = R.DT
        R.DT = dt
        try:
            th = torch.tensor(np.asarray(theta, np.float64), dtype=dt, requires_grad=True)
            noise = [n.to(dt) for n in R.noise_pyramid(cfg, H, W, seed, t)] if quant == "soft" else None
            out = R.forward(cfg, H, W, th, torch.tensor(np.asarray(img), dtype=dt), lam, quant, T,
                            sigma, noise)
            out["loss"].backward()
            return th.grad.double().numpy()
        finally:
            R.DT = old

    dev = np.abs(grad(torch.float32) - grad(torch.float64))
    slack = np.zeros_like(dev)
    for _, sl in segs:
        if sl.stop > sl.start:
            slack[sl] = dev[sl].max()
    return slack
