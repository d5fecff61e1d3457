"""Quantisation and Exp-Golomb rate of the decoder parameters, and the choice
of their quantisation steps and Exp-Golomb orders by rate-distortion cost
(Section IV-E, "Neural network transmission"), FP64.

TEST INFRASTRUCTURE ONLY.  Only the tests may use this module; the product
path never does, and it shares no code with the GPU library.

The paper fixes: one pair of quantisation steps (weights, biases) and one
pair of Exp-Golomb orders per submodule (ARM, synthesis, upsampling, IFCE);
parameters quantised to integers and coded with Exp-Golomb; steps and orders
chosen submodule after submodule among a short list of candidates (e.g. 8
steps from 2^-8 to 2^-1) by D + lambda (R(latents) + R_NN), each candidate
evaluated by decoding with the quantised decoder.  Readings where it is
silent:
  * submodules: ARM = arm.* (stabilizer included); synthesis = syn.* and the
    residual layers res.*; upsampling = ups.* (its taps count as weights, it
    has no biases); IFCE = ifce.*; chosen in that order, each with the
    earlier ones quantised at their choice and the later ones unquantised;
  * steps: 2^-8 ... 2^-1 for weights and for biases independently (64
    pairs per submodule, 8 for the upsampling); q = rint(p / step) (ties to
    even), the decoder uses step * q;
  * integers to Exp-Golomb: v > 0 -> 2v - 1, v <= 0 -> -2v; an order-k code
    of u >= 0 takes 2 floor(log2(u + 2^k)) - k + 1 bits; the order of a group
    (submodule, weights or biases) is the one of 0..11 with the fewest bits
    (the smallest on ties);
  * R_NN counts the parameter codes of the quantised submodules; the cost of
    a candidate is MSE + lambda (R(latents) + R_NN) / (H W) (the loss
    normalisation of the encoder), with hard-quantised latents; ties go to
    the earlier candidate (weight step outer, bias step inner, ascending).
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np
import torch

from .coolchic_ref import forward, n_params, unpack_params

SUBMODULES = ("arm", "syn", "ups", "ifce")
STEPS = [2.0 ** -e for e in range(8, 0, -1)]
KAPPAS = list(range(12))


def groups(cfg: Dict) -> Dict[str, Tuple[np.ndarray, np.ndarray]]:
    """Parameter indices of every submodule: (weights, biases)."""
    out = {s: ([], []) for s in SUBMODULES}
    pos = 0
    for name, t in unpack_params(cfg, torch.zeros(n_params(cfg), dtype=torch.float64)).items():
        n = int(t.numel())
        head = name.split(".")[0]
        sub = "syn" if head == "res" else head
        is_bias = name.endswith(".b")
        out[sub][1 if is_bias else 0].extend(range(pos, pos + n))
        pos += n
    return {s: (np.array(w, dtype=np.int64), np.array(b, dtype=np.int64)) for s, (w, b) in out.items()}


def quantise(p: np.ndarray, step: float) -> np.ndarray:
    """Integer codes rint(p / step), ties to even."""
    return np.rint(np.asarray(p, np.float64) / step).astype(np.int64)


def to_unsigned(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, np.int64)
    return np.where(v > 0, 2 * v - 1, -2 * v)


def eg_bits(u: np.ndarray, k: int) -> np.ndarray:
    """Lengths of the order-k Exp-Golomb codes of non-negative integers:
    2 floor(log2(u + 2^k)) - k + 1, with the floor taken exactly."""
    x = np.asarray(u, np.int64).reshape(-1) + (1 << k)
    m = np.array([int(v).bit_length() - 1 for v in x], dtype=np.int64)
    return (2 * m - k + 1).reshape(np.shape(u))


def group_bits(codes: np.ndarray) -> Tuple[int, int]:
    """(fewest bits over the orders, the order reaching them)."""
    if codes.size == 0:
        return 0, 0
    u = to_unsigned(codes)
    best = None
    for k in KAPPAS:
        b = int(eg_bits(u, k).sum())
        if best is None or b < best[0]:
            best = (b, k)
    return best


def apply(cfg: Dict, params: np.ndarray, choice: Dict[str, Tuple[int, int]]):
    """Decoder parameters with the chosen submodules quantised, and R_NN.
    choice[sub] = (weight step index, bias step index); -1 = no biases."""
    g = groups(cfg)
    out = np.array(params, dtype=np.float64, copy=True)
    bits = 0
    kap = {}
    for sub, (iw, ib) in choice.items():
        w, b = g[sub]
        ks = []
        for idx, ist in ((w, iw), (b, ib)):
            if idx.size == 0 or ist < 0:
                ks.append(-1)
                continue
            q = quantise(out[idx], STEPS[ist])
            out[idx] = STEPS[ist] * q
            nb, k = group_bits(q)
            bits += nb
            ks.append(k)
        kap[sub] = tuple(ks)
    return out, bits, kap


def rd(cfg: Dict, H: int, W: int, latents: np.ndarray, params: np.ndarray, img, lam: float):
    """(mse, latent bits) of the decoder with hard-quantised latents."""
    theta = torch.from_numpy(np.concatenate([np.asarray(latents, np.float64),
                                             np.asarray(params, np.float64)]))
    with torch.no_grad():
        o = forward(cfg, H, W, theta, torch.as_tensor(np.asarray(img, np.float64)), lam, "hard")
    return float(o["mse"]), float(o["bits"])


def select(cfg: Dict, H: int, W: int, latents: np.ndarray, params: np.ndarray, img, lam: float):
    """Successive choice of the steps of every submodule; returns (choice,
    orders, quantised parameters, R_NN, mse, latent bits, cost)."""
    g = groups(cfg)
    choice: Dict[str, Tuple[int, int]] = {}
    for sub in SUBMODULES:
        w, b = g[sub]
        if w.size == 0 and b.size == 0:
            continue
        cands = [(iw, ib) for iw in range(len(STEPS)) for ib in (range(len(STEPS)) if b.size else [-1])]
        best = None
        for c in cands:
            trial = dict(choice)
            trial[sub] = c
            pq, nn_bits, _ = apply(cfg, params, trial)
            mse, bits = rd(cfg, H, W, latents, pq, img, lam)
            cost = mse + lam * (bits + nn_bits) / (H * W)
            if best is None or cost < best[0]:
                best = (cost, c)
        choice[sub] = best[1]
    pq, nn_bits, kap = apply(cfg, params, choice)
    mse, bits = rd(cfg, H, W, latents, pq, img, lam)
    return dict(choice=choice, kappa=kap, params=pq, nn_bits=nn_bits, mse=mse, bits=bits,
                cost=mse + lam * (bits + nn_bits) / (H * W))
