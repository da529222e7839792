"""Benchmark: Newton time steps per second of the NSOA-1 Newton-Krylov-Schwarz step on one MI355X.

Default workload: 2D 512 x 512 periodic grid, c + eta_1..3 + displacement (6 unknowns per
node), seeded noise around c = 0.17, adaptive dt in [1e-3, 1] (eq. (sencondt) with zeta = 100
and the divergence retry), Schwarz tiles 32 x 32 with overlap 2, FP64 throughout.

  python bench.py [--gpus 1] [--steps K] [--warmup W]

Warm-up: W steps on a scratch problem (same input).  Timed: K steps of the adaptive
trajectory from t = 0 on a fresh problem whose inputs are already resident in HBM.
Prints one JSON line.  Only one GPU is supported: --gpus N > 1 exits with a message.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton time steps/s + HBM GB/s % peak at 1e-8 rel err; p50/p99 step latency"
HBM_PEAK_GBS = 8000.0


# source file of each kernel kind; a stored traffic figure is used only while that file is
# byte-identical to the one it was measured with
KERNEL_SOURCE = {"residual": "kernels_phase.hip", "linearise": "kernels_phase.hip", "jv": "kernels_phase.hip",
                 "ras": "kernels_ras.hip", "spectral": "kernels_fft.hip", "multidot": "kernels_blas.hip",
                 "update": "kernels_blas.hip"}


def pc_names():
    from paper_2209_08001_amd import pfnks

    return {"ras_spectral": pfnks.PC_RAS_SPECTRAL, "ras": pfnks.PC_RAS, "as": pfnks.PC_AS, "rras": pfnks.PC_RRAS}


def kernel_source_sha256(kind):
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2209_08001_amd", "csrc")
    with open(os.path.join(csrc, KERNEL_SOURCE[kind]), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kind, workload, precision, tile, overlap):
    """HBM bytes per launch of one kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the reading of a plain copy of known size), or
    None when there is none for this kernel and workload or the kernel source has changed."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as fh:
        shape = "x".join(str(t) for t in tile)
        rec = json.load(fh).get(f"{kind}/{workload}/{precision}/tile{shape}/ov{overlap}")
    if not rec or rec.get("source_sha256") != kernel_source_sha256(kind):
        return None, None
    return rec["traffic_bytes_per_launch"], rec["summary"]


def model_bytes(kind, n, tile, overlap, krylov_bytes):
    """Algorithmic bytes per launch of the byte model (per node, times the nodes of a launch)
    for the kernel kinds it prices, else None.  RAS apply: rho (n_f b + 136) + n_f b per node,
    rho = ((T + 2 delta) / T)^d the overlap factor, n_f = 4 + d, b the Krylov element bytes:
    the extended read of the right-hand side over all fields plus the node's 16 block values
    and c^n (136 B), and the owned write.  The spectral preconditioner's tile kernel touches
    only the four (c, eta) fields (its own count is kernel_bytes_per_launch); the displacement
    part of the same apply is the Fourier solve's."""
    if kind != "ras":
        return None
    d = len(n)
    rho = 1.0
    for k in range(d):
        rho *= (tile[k] + 2 * overlap) / tile[k]
    nf = 4 + d
    return math.prod(n) * (rho * (nf * krylov_bytes + 136) + nf * krylov_bytes)


def roofline_entry(p, n, tile, overlap, precision):
    """Roofline of the dominant kernel: live HIP-event average per launch, bytes of the byte
    model per launch (the kernel's own count beside it)."""
    roof = p.roofline(HBM_PEAK_GBS)
    mb = model_bytes(roof["kernel"], n, tile, overlap, 4 if precision == "mixed" else 8)
    if mb is not None:
        roof["kernel_bytes_per_launch"] = roof["bytes_per_launch"]
        roof["bytes_per_launch"] = mb
        roof["achieved"] = mb / (roof["avg_launch_us"] * 1e-6) / 1e9
        roof["frac"] = roof["achieved"] / HBM_PEAK_GBS
        roof["bytes_model"] = "rho (n_f b + 136) + n_f b per node"
    return roof


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return float("nan")
    k = (len(s) - 1) * q / 100.0
    f = math.floor(k)
    c = min(f + 1, len(s) - 1)
    return s[f] + (s[c] - s[f]) * (k - f)


def host_info():
    """The host the CPU oracle runs on: CPU model, logical CPUs, CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = None
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "usable_cpus": usable}


def _timed_oracle_step(o, dt):
    """(wall s, process CPU s) of one oracle step."""
    t0, c0 = time.perf_counter(), time.process_time()
    o.step(dt)
    return time.perf_counter() - t0, time.process_time() - c0


def cpu_baseline(wl_name):
    """The CPU oracle (sparse-LU Newton, one process) on a bounded sample of the workload: the
    first step (dt = dt_min) of the seeded trajectory on 32^2, 48^2 and 64^2, and on 64^2 one more
    step at dt_max (the step size of the late trajectory, where most of the workload's steps
    are taken).  The per-step time at the workload's size is extrapolated by the power law
    fitted to the three first-step times, applied to the late step."""
    import numpy as np

    from oracle import Oracle
    from paper_2209_08001_amd import workloads as W

    wl = W.WORKLOADS[wl_name]
    sizes = [32, 48, 64]
    times = []
    wall = cpu = 0.0
    o = None
    for s in sizes:
        n = (s, s)
        c0, e0 = W.init_fields(n, wl["seed"], cbar=wl["cbar"])
        o = Oracle(n, W.H, W.DEFAULT_MODEL, c0, e0)
        w_, c_ = _timed_oracle_step(o, wl["dt_min"])
        times.append(w_)
        wall += w_
        cpu += c_
    t_late, c_ = _timed_oracle_step(o, wl["dt_max"])  # from the 64^2 state after its first step
    wall += t_late
    cpu += c_
    lx = np.log(np.array([s * s for s in sizes], float))
    b, a = np.polyfit(lx, np.log(np.array(times)), 1)
    scale = (float(np.prod(wl["n"])) / (64.0 * 64.0)) ** b
    t_w = t_late * scale
    threads = max(1, round(cpu / wall)) if wall > 0 else 1
    out = {
        "value": 1.0 / t_w,
        "unit": "steps/s",
        "cores": threads,
        "cpu_time_over_wall": cpu / wall if wall > 0 else None,
        "kind": "oracle",
        "extrapolated": True,
        "sample": (f"first step (dt = {wl['dt_min']}) of the seeded trajectory on 32x32, 48x48, 64x64 "
                   f"(measured {', '.join(f'{t:.2f}' for t in times)} s) and one 64x64 step at dt = {wl['dt_max']} "
                   f"({t_late:.2f} s); the late step scaled to {wl['n'][0]}x{wl['n'][1]} by the fitted "
                   f"N^{b:.2f} law of the sparse-LU Newton solve"),
    }
    out.update(host_info())
    return out


def _solver_for(W, pfnks, n, precision, pc, sweeps=None):
    mixed = precision == "mixed"
    sv = dict(W.DEFAULT_SOLVER, sweeps=sweeps or W.default_sweeps(len(n), mixed),
              sor_omega=W.default_omega(len(n), mixed), pc=pc,
              precision=pfnks.MIXED if mixed else pfnks.FP64)
    if len(n) == 3:
        sv.update(tile=tuple(W.tile_side(s, 8, 1) for s in n), overlap=1)
    else:
        sv["tile"] = (W.tile_side(n[0], 32, sv["overlap"]), W.tile_side(n[1], 32, sv["overlap"]), 1)
    return sv


def run_c1(dev):
    """2D 64 x 64, 10 fixed steps of dt = 1e-2, FP64: per-step latency, the error of every step
    against the oracle's root, and the oracle's own 10 steps timed on the host."""
    import numpy as np
    import torch

    from oracle import Oracle
    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W

    wl = W.WORKLOADS["pf2d_64"]
    n, dt, steps = wl["n"], wl["dt"], wl["steps"]
    c0, e0 = W.init_fields(n, wl["seed"], cbar=wl["cbar"])
    sv = _solver_for(W, pfnks, n, "fp64", pfnks.PC_RAS_SPECTRAL)
    pw = pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c0, e0, device=dev)
    for _ in range(3):
        pw.step(dt)
    pw.close()
    p = pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c0, e0, device=dev)
    lat, stats = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        stats.append(p.step(dt))
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    p.close()
    # the same steps again (the path is deterministic) with the state read after each step
    q = pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c0, e0, device=dev)
    states = []
    for _ in range(steps):
        q.step(dt)
        states.append(q.get_state()[0])
    q.close()
    o = Oracle(n, W.H, W.DEFAULT_MODEL, c0, e0)
    wall = cpu = 0.0
    errs = []
    for k in range(steps):
        w_, c_ = _timed_oracle_step(o, dt)
        wall += w_
        cpu += c_
        errs.append(max(float(np.max(np.abs(states[k][f] - o.X[f])) / np.max(np.abs(o.X[f])))
                        for f in range(o.X.shape[0])))
    return {
        "workload": "pf2d_64", "grid": list(n), "precision": "fp64", "dt": dt, "steps": steps,
        "steps_per_s": steps / elapsed,
        "p50_step_ms": 1e3 * percentile(lat, 50), "p99_step_ms": 1e3 * percentile(lat, 99),
        "newton_per_step": sum(s["newton_its"] for s in stats) / steps,
        "gmres_per_newton": sum(s["gmres_its"] for s in stats) / max(1, sum(s["newton_its"] for s in stats)),
        "max_rel_err_vs_oracle": max(errs),
        "rel_err_vs_oracle_per_step": [float("%.3g" % e) for e in errs],
        "oracle": {"value": steps / wall, "unit": "steps/s", "cores": max(1, round(cpu / wall)),
                   "cpu_time_over_wall": cpu / wall, "kind": "oracle",
                   "sample": f"the full {steps} steps, sparse-LU Newton", **host_info()},
        "note": "cache-resident (197 KB per vector): launch- and latency-bound, reported by latency",
    }


def make_groups(W, pfnks, members, prec, dev, tile=None):
    """Lockstep groups of an ensemble: the instances of each side together (at most
    pfnks.MAX_GROUP per group), each group on a stream of its own.  tile (2D): the largest tile
    sides, by default 32 x 16 (a group's launch holds several instances' tiles, and half-size
    tiles let two workgroups share a compute unit: 6-7 % more instance steps/s than 32 x 32 over
    10 steps of the 64-instance ensemble, in FP64 and mixed precision)."""
    tile = tile or (32, 16)
    import torch

    by_side = {}
    for m in members:
        by_side.setdefault(tuple(m["n"]), []).append(m)
    groups = []
    for n, ms in sorted(by_side.items()):
        for k in range(0, len(ms), pfnks.MAX_GROUP):
            part = ms[k:k + pfnks.MAX_GROUP]
            fields = [W.init_fields(n, m["seed"], cbar=m["cbar"]) for m in part]
            sv = _solver_for(W, pfnks, n, prec, pfnks.PC_RAS_SPECTRAL)
            if len(n) == 2:
                sv["tile"] = (W.tile_side(n[0], tile[0], sv["overlap"]), W.tile_side(n[1], tile[1], sv["overlap"]), 1)
            groups.append(pfnks.Group(n, W.H, W.DEFAULT_MODEL, sv, [f[0] for f in fields], [f[1] for f in fields],
                                      device=dev, stream=torch.cuda.Stream(device=dev)))
    return groups


def run_c4_lockstep(dev, steps=3, prec="mixed"):
    """The ens2d_64 ensemble as lockstep groups (one per side, pfnks_group_step: one launch per
    kernel and phase for all instances of a side, the GMRES rotations on the device), the
    groups on concurrent host threads and streams, over the first steps of every instance's
    adaptive trajectory: instance steps/s and node steps/s."""
    import torch

    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W
    from paper_2209_08001_amd.driver import adaptive_group_run

    wl = W.WORKLOADS["ens2d_64"]
    members = W.ensemble_members(wl)
    scratch = make_groups(W, pfnks, members[:8], prec, dev)
    adaptive_group_run(scratch, 1, wl)
    for g in scratch:
        g.close()
    del scratch
    groups = make_groups(W, pfnks, members, prec, dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, stats = adaptive_group_run(groups, steps, wl)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    count = sum(g.count for g in groups)
    nodes = sum(g.N * g.count for g in groups)
    flat = [s for gs in stats for ss in gs for s in ss]
    newton = sum(s["newton_its"] for s in flat)
    out = {
        "workload": "ens2d_64", "mode": "lockstep groups", "instances": count, "groups": len(groups),
        "group_sizes": [g.count for g in groups], "total_nodes": nodes, "precision": prec, "steps": steps,
        "instance_steps_per_s": count * steps / elapsed,
        "node_steps_per_s": nodes * steps / elapsed,
        "p50_round_ms": 1e3 * percentile(lat, 50), "p99_round_ms": 1e3 * percentile(lat, 99),
        "newton_per_step": newton / (count * steps),
        "gmres_per_newton": sum(s["gmres_its"] for s in flat) / max(newton, 1),
    }
    for g in groups:
        g.close()
    return out


def run_c3(dev, steps=10, warmup=2):
    """3D 128^3, the adaptive trajectory from t = 0: plain FP64 and mixed precision (float
    Krylov basis and preconditioner) over the same step sizes (the mixed run replays the FP64
    run's dt sequence), each with its dominant kernel's roofline, and the largest relative
    difference between the two final states."""
    import numpy as np
    import torch

    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W
    from paper_2209_08001_amd.driver import adaptive_run

    wl = W.WORKLOADS["pf3d_128"]
    n = wl["n"]
    c0, e0 = W.init_fields(n, wl["seed"], cbar=wl["cbar"])
    out = {"workload": "pf3d_128", "grid": list(n), "steps": steps}
    dts = None
    final = {}
    for prec in ("fp64", "mixed"):
        sv = _solver_for(W, pfnks, n, prec, pfnks.PC_RAS_SPECTRAL)
        pw = pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c0, e0, device=dev)
        adaptive_run(pw, 1, wl)
        pw.profile(True)
        adaptive_run(pw, warmup, wl)
        table = pw.kernel_table()
        dominant = max(table, key=lambda k: table[k]["total_ms"])
        pw.close()
        del pw
        p = pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c0, e0, device=dev)
        p.profile([dominant])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if dts is None:
            lat, stats = adaptive_run(p, steps, wl)
            dts = [s["dt"] for s in stats]
        else:
            lat, stats = [], []
            for dt in dts:
                t1 = time.perf_counter()
                stats.append(p.step(dt))
                lat.append(time.perf_counter() - t1)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        roof = roofline_entry(p, n, sv["tile"], sv["overlap"], prec)
        traffic, summary = measured_traffic(roof["kernel"], "pf3d_128", prec, sv["tile"], sv["overlap"])
        roof["traffic"] = traffic
        if traffic is not None:
            roof["traffic_over_algorithmic"] = traffic / roof["bytes_per_launch"]
            roof["traffic_source"] = summary
        final[prec] = p.get_state()[0]
        p.close()
        newton = sum(s["newton_its"] for s in stats)
        out[prec] = {
            "steps_per_s": steps / elapsed, "ms_per_step": 1e3 * elapsed / steps,
            "p50_step_ms": 1e3 * percentile(lat, 50), "p99_step_ms": 1e3 * percentile(lat, 99),
            "newton_per_step": newton / steps, "gmres_per_newton": sum(s["gmres_its"] for s in stats) / max(newton, 1),
            "tile": list(sv["tile"]), "overlap": sv["overlap"], "gs_sweeps": sv["sweeps"], "roofline": roof,
        }
    out["dts"] = [float("%.4g" % d) for d in dts]
    out["mixed_vs_fp64_max_rel_diff"] = max(
        float(np.max(np.abs(final["mixed"][f] - final["fp64"][f])) / np.max(np.abs(final["fp64"][f])))
        for f in range(final["fp64"].shape[0]))
    out["mixed_speedup"] = out["mixed"]["steps_per_s"] / out["fp64"]["steps_per_s"]
    return out


def run_ensemble(args, wl):
    """Ensemble workload: every instance takes K adaptive steps; the instances are stepped
    together, either as lockstep groups of one side each (--ensemble-mode lockstep,
    pfnks_group_step) or by host threads over one stream per instance (threads,
    pfnks_batch_step).  value = instance steps per second over the whole ensemble."""
    import torch

    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W
    from paper_2209_08001_amd.driver import adaptive_batch_run, adaptive_group_run

    members = W.ensemble_members(wl)
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    if args.ensemble_mode == "lockstep":
        dev = "cuda:0"
        if args.warmup > 0:
            scratch = make_groups(W, pfnks, members[:8], args.precision, dev, tile)
            adaptive_group_run(scratch, args.warmup, wl)
            for g in scratch:
                g.close()
            del scratch
        groups = make_groups(W, pfnks, members, args.precision, dev, tile)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat, gstats = adaptive_group_run(groups, args.steps, wl)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        stats = [ss for gs in gstats for ss in gs]
        k = sum(g.count for g in groups)
        nodes = sum(g.N * g.count for g in groups)
        sides = sorted({g.n[0] for g in groups})
        mode_cfg = {"mode": "lockstep groups", "groups": [g.count for g in groups],
                    "tiles": sorted({tuple(g._s.tile[:2]) for g in groups})}
        for g in groups:
            g.close()
    else:
        lat = stats = None
    solver = dict(W.DEFAULT_SOLVER, sweeps=args.sweeps or W.default_sweeps(2, args.precision == "mixed"),
                  sor_omega=W.default_omega(2, args.precision == "mixed"),
                  pc=pc_names()[args.pc],
                  precision=pfnks.MIXED if args.precision == "mixed" else pfnks.FP64)
    dev = "cuda:0"

    def make(ms):
        out = []
        for m in ms:
            c0, e0 = W.init_fields(m["n"], m["seed"], cbar=m["cbar"])
            out.append(pfnks.Problem(m["n"], W.H, W.DEFAULT_MODEL, solver, c0, e0, device=dev,
                                     stream=torch.cuda.Stream(device=dev)))
        return out

    if stats is None:
        if args.warmup > 0:
            scratch = make(members[:8])
            adaptive_batch_run(scratch, args.warmup, wl, args.threads)
            for p in scratch:
                p.close()
            del scratch
        probs = make(members)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lat, stats = adaptive_batch_run(probs, args.steps, wl, args.threads)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        k = len(probs)
        nodes = sum(p.N for p in probs)
        sides = sorted({p.n[0] for p in probs})
        mode_cfg = {"mode": "threads", "host_threads": args.threads}
        for p in probs:
            p.close()
    newton = sum(s["newton_its"] for ss in stats for s in ss)
    gmres = sum(s["gmres_its"] for ss in stats for s in ss)
    out = {
        "metric": "ensemble Newton time steps/s (instance steps, all instances)",
        "value": k * args.steps / elapsed,
        "unit": "instance steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": dict({"workload": args.workload, "instances": k, "total_nodes": nodes,
                        "sides": sides, "precision": args.precision, "preconditioner": args.pc}, **mode_cfg),
        "node_steps_per_s": nodes * args.steps / elapsed,
        "p50_round_ms": 1e3 * percentile(lat, 50),
        "p99_round_ms": 1e3 * percentile(lat, 99),
        "newton_per_step": newton / (k * args.steps),
        "gmres_per_newton": gmres / max(newton, 1),
        "retries": sum(s["retries"] for ss in stats for s in ss),
        "roofline": None,
    }
    print(json.dumps(out))


def run_serving(args, wl):
    """Serving workload: seeded Poisson arrivals served with continuous batching; value =
    accepted steps per second over the makespan; per-step latency while resident and queue
    wait reported separately."""
    import torch

    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W
    from paper_2209_08001_amd.serve import Server, poisson_requests

    solver = dict(W.DEFAULT_SOLVER, sweeps=args.sweeps or W.default_sweeps(2, args.precision == "mixed"),
                  sor_omega=W.default_omega(2, args.precision == "mixed"),
                  pc=pc_names()[args.pc],
                  precision=pfnks.MIXED if args.precision == "mixed" else pfnks.FP64)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    window = args.window if args.window is not None else wl["window"]
    mk = lambda seed: poisson_requests(wl["rate"], window, seed, wl["sides2d"], wl["sides3d"],
                                       wl["frac3d"], args.steps if args.steps_given else wl["steps"])
    if args.warmup > 0:
        Server(solver, wl, budget, threads=args.threads, mode=args.serve_mode,
               group_capacity=args.group_capacity).run(mk(wl["seed"] + 1000)[:4], realtime=False)
    reqs = mk(wl["seed"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Server(solver, wl, budget, threads=args.threads, mode=args.serve_mode,
           group_capacity=args.group_capacity).run(reqs, realtime=True)
    torch.cuda.synchronize()
    makespan = time.perf_counter() - t0
    steps = sum(r.done for r in reqs)
    lat = [x for r in reqs for x in r.step_ms]
    waits = [r.admitted_at - r.arrival for r in reqs]
    out = {
        "metric": "served Newton time steps/s (continuous batching); per-step latency p50/p99",
        "value": steps / makespan,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * makespan / max(steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "requests": len(reqs), "rate_per_s": wl["rate"],
                   "window_s": window, "steps_per_request": reqs[0].steps if reqs else 0,
                   "hbm_budget_bytes": budget, "precision": args.precision, "host_threads": args.threads,
                   "mode": args.serve_mode, "group_capacity": args.group_capacity if args.serve_mode == "groups" else None},
        "makespan_s": makespan,
        "p50_step_ms": percentile(lat, 50),
        "p99_step_ms": percentile(lat, 99),
        "p50_queue_wait_s": percentile(waits, 50),
        "p99_queue_wait_s": percentile(waits, 99),
        "roofline": None,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="pf2d_512")
    ap.add_argument("--pc", default="ras_spectral", choices=sorted(pc_names()))
    ap.add_argument("--sweeps", type=int, default=None,
                    help="Gauss-Seidel sweeps of the tile solve (default: workloads.default_sweeps)")
    ap.add_argument("--tile", default=None, help="Schwarz tile, e.g. 32,32 (2D) or 8,8,8 (3D)")
    ap.add_argument("--overlap", type=int, default=None)
    ap.add_argument("--sor", type=float, default=None,
                    help="over-relaxation of the tile sweeps (default: workloads.default_omega)")
    ap.add_argument("--pc-refresh", action="store_true",
                    help="rebuild the preconditioner at every Newton iteration (default: once per step)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick tile / overlap / sweeps by timing candidates first (reported in config)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="mixed: float Krylov basis and Schwarz/Fourier preconditioner, double "
                         "residual, J v arithmetic, Newton update, energy and mass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c1", action="store_true", help="default workload: skip the 64 x 64 fixed-step object")
    ap.add_argument("--no-c3", action="store_true", help="default workload: skip the 128^3 FP64 / mixed object")
    ap.add_argument("--c3-steps", type=int, default=10)
    ap.add_argument("--no-c4", action="store_true", help="default workload: skip the 64-instance ensemble object")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--threads", type=int, default=16,
                    help="ensemble workloads: host threads driving the instances (pfnks_batch_step)")
    ap.add_argument("--serve-mode", default="groups", choices=["groups", "threads"],
                    help="serving workload: lockstep slot groups per grid shape or one problem per request")
    ap.add_argument("--group-capacity", type=int, default=8, help="serving workload: slots of a shape's group")
    ap.add_argument("--ensemble-mode", default="lockstep", choices=["lockstep", "threads"],
                    help="ensemble workloads: lockstep groups of one side each (pfnks_group_step) or "
                         "host threads over one stream per instance (pfnks_batch_step)")
    ap.add_argument("--window", type=float, default=None,
                    help="serving workload: arrival window in seconds (default: the workload's)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="before the run, copy a device buffer of this many MiB once (a plain copy "
                         "kernel of known size, to scale the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    args.steps_given = any(a == "--steps" or a.startswith("--steps=") for a in sys.argv[1:])
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU (asked for --gpus {args.gpus}); the spatial "
              "decomposition over several GPUs is described, not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W
    from paper_2209_08001_amd.driver import adaptive_run

    wl = W.WORKLOADS[args.workload]
    if wl.get("ensemble"):
        return run_ensemble(args, wl)
    if wl.get("serve"):
        return run_serving(args, wl)
    n = wl["n"]
    model = W.DEFAULT_MODEL
    if "particle" in wl:
        c0, e0 = W.particle_fields(n, W.H, wl["particle"])
        model = W.P1_MODEL
        args.no_cpu_baseline = True
    else:
        c0, e0 = W.init_fields(n, wl["seed"], cbar=wl["cbar"])
    solver = dict(W.DEFAULT_SOLVER, sweeps=args.sweeps or W.default_sweeps(2, args.precision == "mixed"),
                  sor_omega=W.default_omega(2, args.precision == "mixed"),
                  pc=pc_names()[args.pc],
                  precision=pfnks.MIXED if args.precision == "mixed" else pfnks.FP64)
    if len(n) == 3:
        solver.update(tile=(8, 8, 8), overlap=1, sweeps=args.sweeps or W.default_sweeps(3, args.precision == "mixed"),
                      sor_omega=W.default_omega(3, args.precision == "mixed"))
    if args.tile:
        t = tuple(int(v) for v in args.tile.split(","))
        solver["tile"] = t if len(t) == 3 else (t[0], t[1], 1)
    if args.overlap is not None:
        solver["overlap"] = args.overlap
    solver["pc_refresh"] = 1 if args.pc_refresh else 0
    if args.sor is not None:
        solver["sor_omega"] = args.sor
    dev = "cuda:0"
    tuned = None
    if args.autotune:
        from paper_2209_08001_amd.autotune import autotune

        best, table = autotune(n, W.H, model, solver, c0, e0, wl, device=dev)
        solver.update(tile=best["tile"], overlap=best["overlap"], sweeps=best["sweeps"])
        tuned = {"best": best, "candidates": len(table)}
    if args.copy_calibration_mb > 0:
        src = torch.ones(args.copy_calibration_mb * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # warm-up on a scratch problem; it also times every kernel kind to find the dominant one
    dominant = "ras"
    table = {}
    if args.warmup > 0:
        pw = pfnks.Problem(n, W.H, model, solver, c0, e0, device=dev)
        if args.warmup > 1:
            # the first step loads every kernel's code; the table covers the steps after it
            adaptive_run(pw, 1, wl)
        pw.profile(True)
        adaptive_run(pw, max(args.warmup - 1, 1), wl)
        table = pw.kernel_table()
        if table:
            dominant = max(table, key=lambda k: table[k]["total_ms"])
        pw.close()
        del pw

    p = pfnks.Problem(n, W.H, model, solver, c0, e0, device=dev)
    if not args.no_roofline:
        p.profile([dominant])  # only the dominant kernel is bracketed in the timed region
    m0 = p.mass()
    E0 = p.energy()[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lat, stats = adaptive_run(p, args.steps, wl)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    newton = sum(s["newton_its"] for s in stats)
    gmres = sum(s["gmres_its"] for s in stats)
    mass_drift = max(abs(s["mass"] - m0) / abs(m0) for s in stats)
    energies = [E0] + [s["energy"] for s in stats]
    energy_up = max(0.0, max(energies[k + 1] - energies[k] for k in range(len(stats))))
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "grid": list(n),
            "unknowns_per_node": 4 + len(n),
            "dt_range": [wl["dt_min"], wl["dt_max"]],
            "preconditioner": args.pc,
            "precision": args.precision,
            "tile": list(solver["tile"][:len(n)]),
            "overlap": solver["overlap"],
            "gs_sweeps": solver["sweeps"],
            "sor_omega": solver.get("sor_omega", 1.0),
            "pc_refresh": solver["pc_refresh"],
            "autotuned": tuned,
            "gmres_restart": solver["gmres_restart"],
            "newton_rtol": solver["newton_rtol"],
            "newton_stol": solver["newton_stol"],
            "gmres_rtol": solver["gmres_rtol"],
        },
        "p50_step_ms": 1e3 * percentile(lat, 50),
        "p99_step_ms": 1e3 * percentile(lat, 99),
        "newton_per_step": newton / args.steps,
        "gmres_per_newton": gmres / max(newton, 1),
        "t_final": p.get_state()[1],
        "dt_last": stats[-1]["dt"],
        "retries": sum(s["retries"] for s in stats),
        "mass_rel_drift_max": mass_drift,
        "energy_increase_max": energy_up,
    }
    if table:
        # every kernel kind timed with events during the warm-up steps (algorithmic bytes)
        out["warmup_kernels"] = {k: {"launches": v["launches"], "avg_us": round(v["avg_us"], 2),
                                     "GB_s": round(v["GB_s"], 1) if v["GB_s"] else None}
                                 for k, v in table.items()}
    if not args.no_roofline:
        roof = roofline_entry(p, n, solver["tile"][:len(n)], solver["overlap"], args.precision)
        traffic, summary = measured_traffic(roof["kernel"], args.workload, args.precision,
                                            solver["tile"][:len(n)], solver["overlap"])
        roof["traffic"] = traffic
        if traffic is not None:
            roof["traffic_over_algorithmic"] = traffic / roof["bytes_per_launch"]
            roof["traffic_source"] = summary
        out["roofline"] = roof
    p.close()
    default_line = args.workload == "pf2d_512" and args.precision == "fp64" and args.pc == "ras_spectral"
    if default_line and not args.no_c3:
        out["c3"] = run_c3(dev, steps=args.c3_steps)
    if default_line and not args.no_c4:
        out["c4"] = run_c4_lockstep(dev)
        # the mixed-precision batched form against this line's plain FP64 form, per node step
        out["c4"]["vs_fp64_single_node_steps"] = out["c4"]["node_steps_per_s"] / (out["value"] * float(math.prod(n)))
    if default_line and not args.no_c1:
        out["c1"] = run_c1(dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
