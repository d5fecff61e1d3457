"""Continuous-batching encode server on one GPU.

Requests (an image, a rate-distortion lambda, an iteration budget) arrive over
time.  The server keeps every admitted request's state (latents, decoder
parameters, Adam moments, scratch) resident in HBM, admits queued requests
whenever a slot is free and the HBM budget allows, and at every step runs one
batched encode iteration (one set of launches) over all active requests, each
at its own iteration index of its own schedule.  A request retires after its
budget with a hard-quantised rate/distortion evaluation; a request whose loss
becomes non-finite is cancelled alone.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np
import torch

from . import _lib
from .encoder import Encoder, schedule, state_bytes, step_batch, step_params


@dataclass
class Job:
    rid: int
    image: np.ndarray          # [3, H, W] float32
    lam: float
    seed: int
    n_iter: int
    arrival: float = 0.0       # seconds on the server clock
    params: Optional[np.ndarray] = None
    # filled by the server
    admitted: float = -1.0
    finished: float = -1.0
    status: str = "queued"
    result: Dict = field(default_factory=dict)


class Server:
    def __init__(self, mc, precision: str = "bf16", hbm_budget: int = 64 << 30,
                 max_slots: int = _lib.CC_MAX_BATCH, check_every: int = 50,
                 clock: Callable[[], float] = time.perf_counter, shapes=None):
        self.mc = mc
        # autotune.ShapeCache (or None): tuned launch shapes applied at admission
        self.shapes = shapes
        self.precision = precision
        self.budget = int(hbm_budget)
        self.max_slots = min(int(max_slots), _lib.CC_MAX_BATCH)
        self.check_every = int(check_every)
        self.clock = clock
        self.queue: List[Job] = []
        self.active: List[tuple] = []      # (job, encoder, t)
        self.done: List[Job] = []
        self.used = 0
        self.peak_used = 0
        self.steps = 0
        self.work_px_it = 0.0
        self.t0 = None

    def now(self):
        return self.clock() - self.t0

    def submit(self, job: Job):
        self.queue.append(job)

    def _bytes(self, job):
        _, H, W = job.image.shape
        return state_bytes(self.mc, H, W, self.precision)

    def _admit(self):
        still = []
        for job in self.queue:
            if job.arrival > self.now():
                still.append(job)
                continue
            need = self._bytes(job)
            if need > self.budget:
                job.status = "rejected: larger than the HBM budget"
                job.finished = self.now()
                self.done.append(job)
                continue
            if len(self.active) >= self.max_slots or self.used + need > self.budget:
                still.append(job)
                continue
            _, H, W = job.image.shape
            # latents start at zero (latents=None); the decoder from job.params
            enc = Encoder(self.mc, torch.from_numpy(job.image), job.lam, job.seed, None,
                          job.params, precision=self.precision)
            if self.shapes is not None:
                shape = self.shapes.get(self.mc, self.precision, H, W)
                if shape is not None:
                    # a bucket spans sizes: a smaller image may have fewer ARM bands
                    bands = enc.launch_shape()["arm_bands"]
                    shape["arm_wgs"] = min(int(shape.get("arm_wgs", 0)), bands)
                    enc.set_launch_shape(**shape)
            self.used += enc.nbytes
            self.peak_used = max(self.peak_used, self.used)
            job.admitted = self.now()
            job.status = "running"
            self.active.append([job, enc, 0])
        self.queue = still

    def _retire(self, idx: int, status: str):
        job, enc, _ = self.active[idx]
        if status == "done":
            job.result = enc.rd_eval()
        job.status = status
        job.finished = self.now()
        self.used -= enc.nbytes
        self.done.append(job)
        self.active[idx] = None

    def step(self):
        """One batched iteration over every active request (chunks of
        CC_MAX_BATCH).  Returns the number of requests stepped."""
        if not self.active:
            return 0
        check = self.check_every and (self.steps + 1) % self.check_every == 0
        encs, ps = [], []
        for slot in self.active:
            job, enc, t = slot
            t += 1
            slot[2] = t
            lr, T, s = schedule(t, job.n_iter)
            encs.append(enc)
            ps.append(step_params(t, lr, T, s))
        out = []
        for i in range(0, len(encs), _lib.CC_MAX_BATCH):
            out.append(step_batch(encs[i:i + _lib.CC_MAX_BATCH], ps[i:i + _lib.CC_MAX_BATCH],
                                  sync=check))
        self.steps += 1
        for job, enc, _ in self.active:
            self.work_px_it += enc.H * enc.W
        # cancel non-finite requests (checked every check_every steps), retire finished ones
        if check:
            flat = [x for r in out for x in r]
            for i, (loss, _, _) in enumerate(flat):
                if not np.isfinite(loss):
                    self._retire(i, "cancelled: non-finite loss")
        for i, slot in enumerate(self.active):
            if slot is not None and slot[2] >= slot[0].n_iter:
                self._retire(i, "done")
        n = len(encs)
        self.active = [s for s in self.active if s is not None]
        return n

    def run(self, jobs: List[Job], idle_sleep: float = 1e-3):
        """Serve a finite trace to completion; returns the finished jobs."""
        for j in sorted(jobs, key=lambda j: j.arrival):
            self.submit(j)
        self.t0 = self.clock()
        while self.queue or self.active:
            self._admit()
            if not self.active:
                if self.queue:
                    time.sleep(idle_sleep)
                continue
            self.step()
        torch.cuda.synchronize()
        return self.done

    def stats(self):
        lat = np.array([j.finished - j.arrival for j in self.done if j.status == "done"])
        wall = max((j.finished for j in self.done), default=0.0)
        return dict(completed=int(len(lat)), p50_s=float(np.percentile(lat, 50)) if len(lat) else None,
                    p99_s=float(np.percentile(lat, 99)) if len(lat) else None,
                    wall_s=wall, steps=self.steps,
                    throughput_mpx_it_s=self.work_px_it / max(wall, 1e-9) / 1e6)


def trace_jobs(n=24, rate_hz=8.0, seed=7, lo=256, hi=2048, n_iter=2000, mc=None, param_seed=0):
    """Jobs of a Poisson request trace with synthetic images."""
    from . import workloads as wl
    jobs = []
    for r in wl.request_trace(n, rate_hz, seed, lo, hi):
        img = wl.synth_image(r.H, r.W, r.seed, n_rects=8)
        jobs.append(Job(r.rid, img, r.lam, r.seed, n_iter, r.arrival_s,
                        params=wl.init_params(mc, r.seed) if mc is not None else None))
    return jobs
