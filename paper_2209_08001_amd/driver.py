"""Adaptive time stepping above the C ABI (Section 4): the step size of eq. (sencondt),
    dt_{n+1} = max(dt_min, dt_max / sqrt(1 + zeta |X'_d|^2)),
with X'_d the RMS change of (c, eta) over the last step divided by its dt, dt_1 = dt_min, and
the divergence retry (dt <- dt / sqrt(2), zeta <- 2 zeta, the doubled zeta kept).  A retry
below dt_min / 2^6 gives up.  One problem (`adaptive_run`), an ensemble stepped together
through pfnks_batch_step (`adaptive_batch_run`, each instance with its own dt history), or
lockstep groups of one grid shape each (`adaptive_group_run`).
"""

import math
import time

from . import pfnks


class _Clock:
    """Per-instance state of the step-size rule."""

    def __init__(self, wl):
        self.dt_min, self.dt_max, self.zeta = wl["dt_min"], wl["dt_max"], wl["zeta"]
        self.rate = None
        self.retries = 0

    def next_dt(self):
        if self.rate is None:
            return self.dt_min
        return max(self.dt_min, self.dt_max / math.sqrt(1.0 + self.zeta * self.rate * self.rate))

    def failed(self, dt):
        self.zeta *= 2.0
        self.retries += 1
        dt /= math.sqrt(2.0)
        if dt < self.dt_min * 2.0 ** -6:
            raise RuntimeError("adaptive driver: step failed down to the dt floor")
        return dt

    def accepted(self, st, dt):
        self.rate = st["dx_rms"] / dt


def adaptive_run(p, nsteps, wl, rate0=None):
    """nsteps accepted steps of one problem; returns (per-step wall latencies, stats).
    rate0: the change rate of the step before (None: the first step takes dt_min)."""
    clk = _Clock(wl)
    clk.rate = rate0
    lat, stats = [], []
    for _ in range(nsteps):
        dt = clk.next_dt()
        t0 = time.perf_counter()
        retries = 0
        while True:
            status, st = p.try_step(dt)
            if status == pfnks.PFNKS_OK:
                break
            dt = clk.failed(dt)
            retries += 1
        lat.append(time.perf_counter() - t0)
        st["dt"], st["retries"] = dt, retries
        stats.append(st)
        clk.accepted(st, dt)
    return lat, stats


def adaptive_batch_run(problems, nsteps, wl, threads=0):
    """nsteps accepted steps of every problem; each round steps all instances together
    (pfnks_batch_step) and re-runs only the instances that must retry.  Returns (per-round
    wall latencies, stats[instance][step])."""
    clocks = [_Clock(wl) for _ in problems]
    lat = []
    stats = [[] for _ in problems]
    for _ in range(nsteps):
        t0 = time.perf_counter()
        todo = list(range(len(problems)))
        dts = {i: clocks[i].next_dt() for i in todo}
        retries = {i: 0 for i in todo}
        while todo:
            status, st = pfnks.batch_step([problems[i] for i in todo], [dts[i] for i in todo], threads)
            again = []
            for j, i in enumerate(todo):
                if status[j] == pfnks.PFNKS_OK:
                    st[j]["dt"], st[j]["retries"] = dts[i], retries[i]
                    stats[i].append(st[j])
                    clocks[i].accepted(st[j], dts[i])
                else:
                    dts[i] = clocks[i].failed(dts[i])
                    retries[i] += 1
                    again.append(i)
            todo = again
        lat.append(time.perf_counter() - t0)
    return lat, stats


def adaptive_group_run(groups, nsteps, wl):
    """nsteps accepted steps of every instance of every lockstep group (pfnks.Group).  Each
    group runs on a host thread of its own (and its own stream); in a round a group steps all
    its instances together, then re-steps only those that must retry while the others sit out
    (dt = 0).  Returns (per-round wall latencies, stats[group][instance][step])."""
    from concurrent.futures import ThreadPoolExecutor

    clocks = [[_Clock(wl) for _ in range(g.count)] for g in groups]
    stats = [[[] for _ in range(g.count)] for g in groups]

    def one_round(gi):
        g, cl = groups[gi], clocks[gi]
        dts = [c.next_dt() for c in cl]
        retries = [0] * g.count
        todo = set(range(g.count))
        while todo:
            status, st = g.step([dts[i] if i in todo else 0.0 for i in range(g.count)])
            for i in sorted(todo):
                if status[i] == pfnks.PFNKS_OK:
                    st[i]["dt"], st[i]["retries"] = dts[i], retries[i]
                    stats[gi][i].append(st[i])
                    cl[i].accepted(st[i], dts[i])
                    todo.discard(i)
                else:
                    dts[i] = cl[i].failed(dts[i])
                    retries[i] += 1

    lat = []
    with ThreadPoolExecutor(max_workers=max(1, len(groups))) as pool:
        for _ in range(nsteps):
            t0 = time.perf_counter()
            for f in [pool.submit(one_round, gi) for gi in range(len(groups))]:
                f.result()
            lat.append(time.perf_counter() - t0)
    return lat, stats
