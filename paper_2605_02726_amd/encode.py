"""Multi-stage encoding of one image (Section IV-D, Table I).

  warm-up    several randomly initialised candidates are trained for a few
             hundred iterations; the best ones (rate-distortion cost of the
             hard-quantised decoder) are refined, and the best one is kept
             (Table I: 5 candidates, then 2, 400 iterations each round);
  main       the schedules of Table I over the main budget: learning rate
             cosine 1e-2 -> 1e-5, softround temperature 0.35 -> 0.08 and
             noise std 0.22 -> 0.15 linear;
  hard round actual rounding in the forward pass, latents frozen, decoder
             parameters trained (Table I: 500 iterations).

Readings where the paper is silent: the warm-up rounds run at the
schedules' start values (lr 1e-2, T 0.35, sigma 0.22) and every candidate
draws its own noise (its own seed); the hard-round stage uses a constant
learning rate of 1e-4.  The candidates of a round are stepped together in one
batched launch set.

The driver talks to a backend with four calls (create, step_batch, rd_eval,
state); `GpuBackend` runs them on the library, tests may substitute another.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np


@dataclass
class StagePlan:
    candidates: Sequence[int] = (5, 2)   # candidates per warm-up round
    warmup_iters: int = 400              # iterations per warm-up round
    main_iters: int = 96_700
    hard_iters: int = 500
    lr0: float = 1e-2
    lr1: float = 1e-5
    T0: float = 0.35
    T1: float = 0.08
    s0: float = 0.22
    s1: float = 0.15
    hard_lr: float = 1e-4


def main_schedule(i: int, n: int, p: StagePlan):
    """Table I schedules at main-stage iteration i of n (i from 1)."""
    import math
    a = 0.0 if n <= 1 else (i - 1) / (n - 1)
    lr = p.lr1 + 0.5 * (p.lr0 - p.lr1) * (1.0 + math.cos(math.pi * a))
    return lr, p.T0 + (p.T1 - p.T0) * a, p.s0 + (p.s1 - p.s0) * a


class GpuBackend:
    def __init__(self, mc, image, lam, precision="bf16"):
        import torch
        self.mc, self.lam, self.precision = mc, lam, precision
        self.image = torch.as_tensor(image, dtype=torch.float32)

    def create(self, seed, params):
        from .encoder import Encoder
        # latents start at zero (every grid, hyperlatent grids included)
        return Encoder(self.mc, self.image, self.lam, seed, None, params, precision=self.precision)

    def step_batch(self, handles, specs):
        """specs: list of (t, lr, T, sigma, quant, update_latents)."""
        from .encoder import step_batch, step_params
        step_batch(handles, [step_params(*s) for s in specs], sync=False)

    def rd_eval(self, h):
        return h.rd_eval()

    def latents(self, h):
        return h.get_state()["latents"]


@dataclass
class EncodeResult:
    handle: object
    rd: dict
    history: List[dict] = field(default_factory=list)
    seconds: float = 0.0


def encode(backend, init_params: Sequence[np.ndarray], plan: StagePlan = StagePlan(),
           seeds: Sequence[int] = None) -> EncodeResult:
    """Run the three stages.  init_params: one parameter vector per warm-up
    candidate (len >= plan.candidates[0]); seeds: one noise seed each."""
    t0 = time.perf_counter()
    n0 = plan.candidates[0] if plan.candidates else 1
    seeds = list(seeds) if seeds is not None else list(range(1, n0 + 1))
    pool = [(backend.create(seeds[i], init_params[i]), 0) for i in range(n0)]   # (handle, t)
    history = []
    # warm-up rounds: train all survivors, keep the best `keep`
    rounds = list(plan.candidates[1:]) + [1]
    for keep in rounds if plan.candidates else []:
        specs = []
        for it in range(plan.warmup_iters):
            specs = [(t + it + 1, plan.lr0, plan.T0, plan.s0, "soft", True) for _, t in pool]
            backend.step_batch([h for h, _ in pool], specs)
        pool = [(h, t + plan.warmup_iters) for h, t in pool]
        costs = [backend.rd_eval(h)["loss"] for h, _ in pool]
        order = np.argsort(costs, kind="stable")
        history.append({"stage": "warm-up", "costs": [float(c) for c in costs],
                        "kept": [int(i) for i in order[:keep]]})
        pool = [pool[i] for i in order[:keep]]
    h, t = pool[0]
    # main stage
    for i in range(1, plan.main_iters + 1):
        lr, T, s = main_schedule(i, plan.main_iters, plan)
        backend.step_batch([h], [(t + i, lr, T, s, "soft", True)])
    t += plan.main_iters
    history.append({"stage": "main", "rd": backend.rd_eval(h)})
    # hard-round stage: latents frozen
    for i in range(1, plan.hard_iters + 1):
        backend.step_batch([h], [(t + i, plan.hard_lr, plan.T1, 0.0, "hard", False)])
    rd = backend.rd_eval(h)
    history.append({"stage": "hard", "rd": rd})
    return EncodeResult(h, rd, history, time.perf_counter() - t0)
