"""Serving loop: continuous batching of phase-field requests on one GPU.

A request asks for `steps` adaptive time steps of one problem (grid, seed, mean
composition).  Requests wait in arrival order; one is admitted when a slot is free and the
sum of the resident problems' workspaces (pfnks_workspace_bytes, exact: the library
allocates nothing else on the device) stays within the HBM budget.  Every tick steps all
resident requests once together (pfnks_batch_step, one stream per request, each request
with its own step-size history), so requests join and leave between ticks.  A request's
result depends only on its own inputs: it is bitwise the result of running it alone.

Latency: each request's own step time, from the start of the tick to the completion of its
step on its stream (HIP events on that stream), so a small request that finishes early in a
tick is not charged the tick's slowest member.
"""

import time

import numpy as np

from . import pfnks
from . import workloads as W
from .driver import _Clock


class Request:
    def __init__(self, rid, n, seed, cbar, steps, arrival=0.0):
        self.rid, self.n, self.seed, self.cbar, self.steps, self.arrival = rid, tuple(n), seed, cbar, steps, arrival
        self.problem = None
        self.clock = None
        self.done = 0
        self.admitted_at = None
        self.finished_at = None
        self.step_ms = []
        self.dts = []
        self.retries = 0
        self.stream = None
        self.state = None
        self.t = None


def poisson_requests(rate, window, seed, sides2d, sides3d, frac3d, steps):
    """Seeded Poisson arrivals (exponential gaps of mean 1/rate) over `window` seconds; each
    request 2D with probability 1 - frac3d (side uniform over sides2d) or 3D (sides3d),
    mean composition uniform in [0.13, 0.21], noise seed 5000 + index."""
    rng = np.random.default_rng(seed)
    out, t = [], 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > window:
            break
        k = len(out)
        if rng.uniform() < frac3d:
            s = int(rng.choice(np.array(sides3d)))
            n = (s, s, s)
        else:
            s = int(rng.choice(np.array(sides2d)))
            n = (s, s)
        out.append(Request(k, n, 5000 + k, float(rng.uniform(0.13, 0.21)), steps, arrival=t))
    return out


class Server:
    def __init__(self, solver, wl, hbm_budget, max_resident=64, threads=16, device="cuda:0", keep_state=False):
        self.solver, self.wl, self.budget = solver, wl, hbm_budget
        self.max_resident, self.threads, self.device = max_resident, threads, device
        self.keep_state = keep_state

    def _solver_for(self, n):
        sv = dict(self.solver)
        mixed = sv.get("precision", pfnks.FP64) == pfnks.MIXED
        sv["sweeps"] = W.default_sweeps(len(n), mixed)
        sv["sor_omega"] = W.default_omega(len(n), mixed)
        if len(n) == 3:
            sv["overlap"] = 1
            sv["tile"] = tuple(W.tile_side(s, 8, 1) for s in n)
        else:
            sv["tile"] = (W.tile_side(n[0], 32, sv["overlap"]), W.tile_side(n[1], 32, sv["overlap"]), 1)
        return sv

    def bytes_for(self, r):
        return pfnks.workspace_bytes(r.n, W.H, W.DEFAULT_MODEL, self._solver_for(r.n))

    def run(self, requests, realtime=True):
        """Serve the requests (arrival times in seconds from the start); returns them with
        their records filled (queue wait, per-step latency, final state if keep_state)."""
        import torch

        pending = sorted(requests, key=lambda r: r.arrival)
        need = {r.rid: self.bytes_for(r) for r in pending}
        for r in pending:
            if need[r.rid] > self.budget:
                raise ValueError(f"request {r.rid} needs {need[r.rid]} B, more than the HBM budget")
        resident, used = [], 0
        t_start = time.perf_counter()
        now = lambda: (time.perf_counter() - t_start) if realtime else float("inf")
        while pending or resident:
            # admit, in arrival order, what has arrived and fits
            while pending and pending[0].arrival <= now() and len(resident) < self.max_resident \
                    and used + need[pending[0].rid] <= self.budget:
                r = pending.pop(0)
                c0, e0 = W.init_fields(r.n, r.seed, cbar=r.cbar)
                r.stream = torch.cuda.Stream(device=self.device)
                r.problem = pfnks.Problem(r.n, W.H, W.DEFAULT_MODEL, self._solver_for(r.n), c0, e0,
                                          device=self.device, stream=r.stream)
                r.clock = _Clock(self.wl)
                r.admitted_at = now() if realtime else 0.0
                used += need[r.rid]
                resident.append(r)
            if not resident:
                time.sleep(max(0.0, min(0.05, pending[0].arrival - now())))
                continue
            # one tick: every resident request takes one accepted step; its latency runs from
            # an event recorded on its stream at the start of the tick to one recorded after
            # its accepted step
            todo = list(resident)
            ev0, ev1 = {}, {}
            for r in todo:
                ev0[r.rid] = torch.cuda.Event(enable_timing=True)
                ev0[r.rid].record(r.stream)
            dts = {r.rid: r.clock.next_dt() for r in todo}
            while todo:
                status, st = pfnks.batch_step([r.problem for r in todo], [dts[r.rid] for r in todo], self.threads)
                again = []
                for r, s_, x in zip(todo, status, st):
                    if s_ == pfnks.PFNKS_OK:
                        ev1[r.rid] = torch.cuda.Event(enable_timing=True)
                        ev1[r.rid].record(r.stream)
                        r.clock.accepted(x, dts[r.rid])
                        r.dts.append(dts[r.rid])
                        r.done += 1
                    else:
                        dts[r.rid] = r.clock.failed(dts[r.rid])
                        r.retries += 1
                        again.append(r)
                todo = again
            for r in resident:
                ev1[r.rid].synchronize()
                r.step_ms.append(ev0[r.rid].elapsed_time(ev1[r.rid]))
            # retire finished requests
            still = []
            for r in resident:
                if r.done >= r.steps:
                    r.finished_at = now() if realtime else 0.0
                    if self.keep_state:
                        r.state, r.t = r.problem.get_state()
                    r.problem.close()
                    r.problem = None
                    used -= need[r.rid]
                else:
                    still.append(r)
            resident = still
        return requests


def run_alone(r, solver_for, wl, device="cuda:0"):
    """The same request stepped by itself (reference for the alone-versus-mix check); returns
    its final state and time."""
    c0, e0 = W.init_fields(r.n, r.seed, cbar=r.cbar)
    p = pfnks.Problem(r.n, W.H, W.DEFAULT_MODEL, solver_for(r.n), c0, e0, device=device)
    clk = _Clock(wl)
    for _ in range(r.steps):
        dt = clk.next_dt()
        while True:
            status, st = p.try_step(dt)
            if status == pfnks.PFNKS_OK:
                break
            dt = clk.failed(dt)
        clk.accepted(st, dt)
    X, t = p.get_state()
    p.close()
    return X, t
