"""Serving loop: continuous batching of phase-field requests on one GPU.

A request asks for `steps` adaptive time steps of one problem (grid, seed, mean
composition).  Requests wait in arrival order; one is admitted when a slot is free and the
resident workspaces (pfnks_workspace_bytes, exact: the library allocates nothing else on the
device) stay within the HBM budget.  Every tick steps all resident requests once, each with
its own step-size history, so requests join and leave between ticks.  Two ways to step them:

* mode "groups" (default): requests of one grid shape share a lockstep group
  (pfnks_group_*) of `group_capacity` slots: one launch per kernel and phase for all of
  them; a freed slot takes the next request of that shape (pfnks_group_set_instance), empty
  slots sit the step out, and a group is released when its last request leaves.  Each group
  steps on a host thread and stream of its own.  A shape's group takes at most group_share of
  the HBM budget (an eighth by default: fewer slots for large grids), and a new group is created only when the device
  also has the memory free.  A request's result is bitwise its result in a group of one
  (run_alone).
* mode "threads": every request is a problem of its own (pfnks_batch_step, one stream per
  request, host threads); a request's result is bitwise its pfnks_step result alone.

Latency: each request's own step time from events on the stream that steps it: from the
start of the tick to the completion of its accepted step (in a group, of the group's step,
whose launches the members share).
"""

import time
from concurrent.futures import ThreadPoolExecutor

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
        self.slot = None
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


class _SlotGroup:
    """A lockstep group of one grid shape whose slots requests occupy and leave."""

    def __init__(self, n, solver, capacity, c0, e0, device, nbytes):
        import torch

        self.n = tuple(n)
        self.nbytes = nbytes  # the group's workspace
        self.stream = torch.cuda.Stream(device=device)
        # every slot starts as a copy of the first request's fields; set_instance gives each
        # slot its own request when it is taken
        self.group = pfnks.Group(self.n, W.H, W.DEFAULT_MODEL, solver, [c0] * capacity, [e0] * capacity,
                                 device=device, stream=self.stream)
        self.slots = [None] * capacity

    def free_slot(self):
        for i, r in enumerate(self.slots):
            if r is None:
                return i
        return -1

    def occupied(self):
        return [r for r in self.slots if r is not None]


class Server:
    def __init__(self, solver, wl, hbm_budget, max_resident=64, threads=16, device="cuda:0", keep_state=False,
                 mode="groups", group_capacity=8, group_share=0.125):
        self.solver, self.wl, self.budget = solver, wl, hbm_budget
        self.max_resident, self.threads, self.device = max_resident, threads, device
        self.keep_state = keep_state
        if mode not in ("groups", "threads"):
            raise ValueError("mode is 'groups' or 'threads'")
        self.mode = mode
        self.group_capacity = max(1, min(int(group_capacity), pfnks.MAX_GROUP))
        self.group_share = group_share  # largest fraction of the budget one group may take

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
        if self.mode == "groups":
            return self._run_groups(requests, realtime)
        return self._run_threads(requests, realtime)

    def capacity_for(self, nbytes_one):
        """Slots of a new group: group_capacity, fewer for large grids (a group takes at most
        group_share of the budget), at least one."""
        return max(1, min(self.group_capacity, int(self.budget * self.group_share // max(nbytes_one, 1))))

    def _run_groups(self, requests, realtime):
        import gc

        import torch

        pending = sorted(requests, key=lambda r: r.arrival)
        one = {r.rid: self.bytes_for(r) for r in pending}
        for r in pending:
            if one[r.rid] > self.budget:
                raise ValueError(f"request {r.rid} needs {one[r.rid]} B, more than the HBM budget")
        groups, used, nres = [], 0, 0
        t_start = time.perf_counter()
        now = lambda: (time.perf_counter() - t_start) if realtime else float("inf")
        pool = ThreadPoolExecutor(max_workers=max(1, self.threads))

        def admit(r):
            nonlocal used, nres
            g = next((g for g in groups if g.n == r.n and g.free_slot() >= 0), None)
            cap = self.capacity_for(one[r.rid])
            need = one[r.rid] * cap
            if g is None:
                if used + need > self.budget:
                    return False
                # the device must hold it too (released workspaces are collected first)
                if torch.cuda.mem_get_info(self.device)[0] < need + (1 << 30):
                    gc.collect()
                    torch.cuda.empty_cache()
                    if torch.cuda.mem_get_info(self.device)[0] < need + (1 << 30):
                        if nres:
                            return False
                        raise RuntimeError(f"request {r.rid}: {need} B of workspace do not fit on the device")
            c0, e0 = W.init_fields(r.n, r.seed, cbar=r.cbar)
            if g is None:
                g = _SlotGroup(r.n, self._solver_for(r.n), cap, c0, e0, self.device, need)
                groups.append(g)
                used += need
            i = g.free_slot()
            g.group.set_instance(i, c0, e0)
            g.slots[i] = r
            r.slot = (g, i)
            r.clock = _Clock(self.wl)
            r.admitted_at = now() if realtime else 0.0
            nres += 1
            return True

        def tick(g):
            # one accepted step of every request in the group: the others sit out (dt = 0)
            # while failed ones retry with their smaller dt
            members = {i: r for i, r in enumerate(g.slots) if r is not None}
            ev0 = torch.cuda.Event(enable_timing=True)
            ev0.record(g.stream)
            dts = {i: r.clock.next_dt() for i, r in members.items()}
            todo = set(members)
            while todo:
                status, st = g.group.step([dts[i] if i in todo else 0.0 for i in range(len(g.slots))])
                for i in sorted(todo):
                    r = members[i]
                    if status[i] == pfnks.PFNKS_OK:
                        r.clock.accepted(st[i], dts[i])
                        r.dts.append(dts[i])
                        r.done += 1
                        todo.discard(i)
                    else:
                        dts[i] = r.clock.failed(dts[i])
                        r.retries += 1
            ev1 = torch.cuda.Event(enable_timing=True)
            ev1.record(g.stream)
            ev1.synchronize()
            ms = ev0.elapsed_time(ev1)
            for r in members.values():
                r.step_ms.append(ms)

        try:
            while pending or nres:
                while pending and pending[0].arrival <= now() and nres < self.max_resident and admit(pending[0]):
                    pending.pop(0)
                if not nres:
                    time.sleep(max(0.0, min(0.05, pending[0].arrival - now())))
                    continue
                live = [g for g in groups if g.occupied()]
                for f in [pool.submit(tick, g) for g in live]:
                    f.result()
                # retire finished requests; release groups that have emptied
                for g in live:
                    for i, r in enumerate(g.slots):
                        if r is not None and r.done >= r.steps:
                            r.finished_at = now() if realtime else 0.0
                            if self.keep_state:
                                r.state, r.t = g.group.get_state(i)
                            g.slots[i] = None
                            r.slot = None
                            nres -= 1
                    if not g.occupied():
                        g.group.close()
                        groups.remove(g)
                        used -= g.nbytes
        finally:
            pool.shutdown()
        return requests

    def _run_threads(self, requests, realtime):
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


def run_alone(r, solver_for, wl, device="cuda:0", mode="threads"):
    """The same request stepped by itself (reference for the alone-versus-mix check): a single
    problem (mode "threads") or a group of one (mode "groups"); returns its final state and
    time."""
    c0, e0 = W.init_fields(r.n, r.seed, cbar=r.cbar)
    if mode == "groups":
        g = pfnks.Group(r.n, W.H, W.DEFAULT_MODEL, solver_for(r.n), [c0], [e0], device=device)
        clk = _Clock(wl)
        for _ in range(r.steps):
            dt = clk.next_dt()
            while True:
                status, st = g.step([dt])
                if status[0] == pfnks.PFNKS_OK:
                    break
                dt = clk.failed(dt)
            clk.accepted(st[0], dt)
        X, t = g.get_state(0)
        g.close()
        return X, t
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
