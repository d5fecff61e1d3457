"""Pins of the decoder-parameter quantisation and rate oracle
(oracle/nnq.py): Exp-Golomb code lengths against an explicit encoder and
decoder, the signed mapping, the quantiser, the submodule grouping, and the
successive choice against an independent evaluation of every candidate.
CPU only."""
import numpy as np
import pytest

from oracle import coolchic_ref as R
from oracle import nnq as Q
from paper_2605_02726_amd import workloads as wl


def eg_encode(u: int, k: int) -> str:
    """Order-k Exp-Golomb code (textbook): write u + 2^k in binary and
    prefix as many zeros as it has bits beyond k + 1."""
    b = bin(u + (1 << k))[2:]
    return "0" * (len(b) - 1 - k) + b


def eg_decode(bits: str, k: int):
    z = 0
    while bits[z] == "0":
        z += 1
    n = z + k + 1
    return int(bits[z:z + n], 2) - (1 << k), bits[z + n:]


def test_exp_golomb_lengths_match_an_explicit_encoder_and_decode_back():
    for k in range(7):
        us = np.arange(0, 2000)
        lens = Q.eg_bits(us, k)
        stream = ""
        for u, ln in zip(us.tolist(), lens.tolist()):
            c = eg_encode(u, k)
            assert len(c) == ln
            stream += c
        out = []
        while stream:
            v, stream = eg_decode(stream, k)
            out.append(v)
        assert out == us.tolist()


def test_signed_mapping_is_a_bijection():
    v = np.arange(-50, 51)
    u = Q.to_unsigned(v)
    assert sorted(u.tolist()) == list(range(101))
    assert Q.to_unsigned(np.array([0, 1, -1, 2, -2])).tolist() == [0, 1, 2, 3, 4]


def test_quantiser_rounds_half_to_even_and_is_exact_for_power_of_two_steps():
    st = 2.0 ** -3
    assert Q.quantise(np.array([2.5, 3.5, -2.5, 0.49]) * st, st).tolist() == [2, 4, -2, 0]
    p = np.random.default_rng(0).normal(size=1000) * 0.3
    q = Q.quantise(p, st)
    assert np.all(np.abs(p - st * q) <= st / 2)


@pytest.mark.parametrize("mk", [wl.config_hop, wl.config_small, wl.config_tiny])
def test_groups_partition_the_parameters(mk):
    mc = mk()
    g = Q.groups(mc.as_dict())
    allidx = np.concatenate([np.concatenate([w, b]) for w, b in g.values()])
    assert sorted(allidx.tolist()) == list(range(wl.n_params(mc)))
    assert g["ups"][1].size == 0
    names = [n for n, s, _ in wl.param_spec(mc)]
    off = np.cumsum([0] + [int(np.prod(s)) for _, s, _ in wl.param_spec(mc)])
    res0 = names.index("res.0.w") if "res.0.w" in names else None
    if res0 is not None:
        assert off[res0] in set(g["syn"][0].tolist())


def test_nn_rate_counts_the_explicit_codes():
    mc = wl.config_tiny()
    cfg = mc.as_dict()
    par = wl.init_params(mc, 7, arm_out_zero=False).astype(np.float64)
    choice = {"arm": (3, 5), "syn": (2, 7), "ups": (6, -1), "ifce": (0, 1)}
    pq, bits, kap = Q.apply(cfg, par, choice)
    g = Q.groups(cfg)
    ref = 0
    for sub, (iw, ib) in choice.items():
        for idx, ist, k in ((g[sub][0], iw, kap[sub][0]), (g[sub][1], ib, kap[sub][1])):
            if idx.size == 0 or ist < 0:
                continue
            q = np.rint(par[idx] / Q.STEPS[ist]).astype(int)
            assert np.array_equal(pq[idx], Q.STEPS[ist] * q)
            u = [2 * v - 1 if v > 0 else -2 * v for v in q.tolist()]
            lens = [sum(len(eg_encode(x, kk)) for x in u) for kk in Q.KAPPAS]
            assert sum(len(eg_encode(x, k)) for x in u) == min(lens)
            ref += min(lens)
    assert bits == ref


def test_each_choice_minimises_the_cost_over_its_candidates():
    mc = wl.config_tiny()
    cfg = mc.as_dict()
    H = W = 16
    img = wl.synth_image(H, W, 9)
    lat = np.round(wl.random_latents(mc, H, W, 9, scale=2.0)).astype(np.float64)
    par = wl.init_params(mc, 9, arm_out_zero=False).astype(np.float64)
    lam = 2e-2
    res = Q.select(cfg, H, W, lat, par, img, lam)
    g = Q.groups(cfg)
    fixed = {}
    for sub in Q.SUBMODULES:
        costs = {}
        for iw in range(len(Q.STEPS)):
            for ib in (range(len(Q.STEPS)) if g[sub][1].size else [-1]):
                trial = dict(fixed)
                trial[sub] = (iw, ib)
                pq, nb, _ = Q.apply(cfg, par, trial)
                theta = np.concatenate([lat, pq])
                import torch
                with torch.no_grad():
                    o = R.forward(cfg, H, W, torch.from_numpy(theta),
                                  torch.as_tensor(np.asarray(img, np.float64)), lam, "hard")
                costs[(iw, ib)] = float(o["mse"]) + lam * (float(o["bits"]) + nb) / (H * W)
        best = min(costs.values())
        assert costs[res["choice"][sub]] == best
        fixed[sub] = res["choice"][sub]
    assert res["cost"] == pytest.approx(
        res["mse"] + lam * (res["bits"] + res["nn_bits"]) / (H * W), rel=1e-12)
