"""Launch-shape autotuner for the encode step.

The tunable kernels take their launch shape from the state (see
cc_set_launch_shape): the fused ARM's workgroups per image, the synthesis
backward's 64-pixel chunks per workgroup and the residual adjoint's tiles
per workgroup.  ``tune`` times whole encode steps on the device (HIP events
on the launch stream, around several steps) for candidate shapes, one knob
at a time from the library's defaults (coordinate descent), and keeps the
fastest.  ``ShapeCache`` stores the choices in a JSON file keyed by the
device name, the decoder shape, the precision and an image-size bucket
(sides rounded up to multiples of 256), so a server tunes each bucket once.
Only the order of the weight-gradient partial sums depends on the shape.
"""
from __future__ import annotations

import ctypes as C
import json
import math
import os
from typing import Dict, Optional

import numpy as np
import torch

from . import workloads as wl
from . import _lib
from .encoder import Encoder, schedule

SYN_CHUNKS = (6, 8, 12, 16, 24)
RES_TILES = (1, 2, 4)
ARM_FRACTIONS = (1.0, 0.85, 0.7, 0.6, 0.5)   # of the library's packed default; one band per workgroup too


def size_bucket(H: int, W: int) -> str:
    return f"{256 * math.ceil(H / 256)}x{256 * math.ceil(W / 256)}"


def cache_key(mc, precision: str, H: int, W: int, device: Optional[str] = None) -> str:
    dev = device if device is not None else torch.cuda.get_device_name(torch.cuda.current_device())
    shape = json.dumps(mc.as_dict(), sort_keys=True)
    return f"{dev}|{precision}|{shape}|{size_bucket(H, W)}"


class ShapeCache:
    """Tuned launch shapes in a JSON file (path None: in memory only)."""

    def __init__(self, path: Optional[str] = None):
        self.path = path
        self.entries: Dict[str, dict] = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.entries = json.load(f)

    def get(self, mc, precision: str, H: int, W: int, device: Optional[str] = None):
        e = self.entries.get(cache_key(mc, precision, H, W, device))
        return None if e is None else dict(e["shape"])

    def put(self, mc, precision: str, H: int, W: int, shape: dict, ms: float,
            device: Optional[str] = None):
        self.entries[cache_key(mc, precision, H, W, device)] = {"shape": dict(shape), "ms_per_step": ms}
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(self.entries, f, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def _time_steps(enc: Encoder, t0: int, n: int, warmup: int = 2) -> float:
    """Milliseconds per step over n steps after warmup steps (the schedules
    of a 1,000-iteration encode, repeated if the tuner runs longer)."""
    t = t0
    for _ in range(warmup):
        t += 1
        enc.step(t, *schedule(1 + (t - 1) % 1000, 1000), sync=False)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(n):
        t += 1
        enc.step(t, *schedule(1 + (t - 1) % 1000, 1000), sync=False)
    stop.record()
    stop.synchronize()
    return start.elapsed_time(stop) / n


def search(start: dict, knobs, measure, min_gain: float = 0.01, rounds: int = 1):
    """Coordinate descent: for each (knob, candidates) in turn, time every
    candidate with the other knobs at the best values so far (``measure``:
    shape -> ms); a candidate replaces the best only when faster by more than
    ``min_gain``.  With ``rounds`` > 1 the sweep over the knobs repeats from
    the best shape (knobs interact: the best synthesis chunking depends on how
    many compute units the ARM leaves free) until a round changes nothing;
    a shape already timed is not timed again.  Returns (best shape, its ms,
    the start's ms, trials)."""
    seen = {}

    def timed(shape):
        key = tuple(sorted(shape.items()))
        if key not in seen:
            seen[key] = measure(shape)
            trials.append((dict(shape), seen[key]))
        return seen[key]

    trials = []
    best = dict(start)
    best_ms = timed(best)
    start_ms = best_ms
    for _ in range(rounds):
        changed = False
        for knob, cands in knobs:
            for c in cands:
                if c == best[knob]:
                    continue
                trial = dict(best)
                trial[knob] = c
                ms = timed(trial)
                if ms < best_ms * (1.0 - min_gain):
                    best, best_ms, changed = trial, ms, True
        if not changed:
            break
    return best, best_ms, start_ms, trials


def tune(mc, H: int, W: int, precision: str = "bf16", steps: int = 8, seed: int = 0,
         cache: Optional[ShapeCache] = None, min_gain: float = 0.01, repeats: int = 3,
         rounds: int = 2) -> dict:
    """Fastest launch shape found for this decoder, precision and image size;
    returns {"shape": {...}, "ms_per_step": ..., "default_ms_per_step": ...,
    "trials": [...]} and records it in ``cache``.  A candidate replaces the
    current best only when it is faster by more than ``min_gain``; each
    candidate's time is the smallest of ``repeats`` runs of ``steps`` steps
    (a single short run is noisy enough to reorder candidates a few percent
    apart), and up to ``rounds`` sweeps over the knobs run (one sweep with a
    1.5% threshold stopped at the default ARM workgroups when the next knob
    would have made a smaller count 6% faster)."""
    enc = Encoder(mc, torch.from_numpy(wl.synth_image(H, W, seed)), 1e-3, seed,
                  np.zeros(wl.n_latents(mc, H, W), np.float32), wl.init_params(mc, seed),
                  precision=precision)
    info = enc.launch_shape()
    bands = info.pop("arm_bands")
    knobs = [("syn_chunks_per_wg", SYN_CHUNKS), ("res_tiles_per_wg", RES_TILES)]
    if precision == "bf16" and _lib.lib().cc_arm_fused_available(C.byref(enc.cfg)):
        # the plain ARM runs one workgroup per chunk; only the fused form has this knob
        arm = {max(1, min(bands, int(round(f * info["arm_wgs"])))) for f in ARM_FRACTIONS}
        arm.add(min(bands, 512))
        knobs.insert(0, ("arm_wgs", sorted(arm, reverse=True)))
    clock = {"t": 0}

    def measure(shape):
        enc.set_launch_shape(**shape)
        ms = float("inf")
        for _ in range(repeats):
            ms = min(ms, _time_steps(enc, clock["t"], steps))
            clock["t"] += steps + 2
        return ms

    best, best_ms, default_ms, trials = search(info, knobs, measure, min_gain, rounds)
    del enc
    if cache is not None:
        cache.put(mc, precision, H, W, best, best_ms)
    return {"shape": best, "ms_per_step": best_ms, "default_ms_per_step": default_ms,
            "trials": trials}
