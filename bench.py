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


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return float("nan")
    k = (len(s) - 1) * q / 100.0
    f = math.floor(k)
    c = min(f + 1, len(s) - 1)
    return s[f] + (s[c] - s[f]) * (k - f)


def cpu_baseline(wl_name, budget_s=30.0):
    """The CPU oracle (sparse LU Newton, one process) on a bounded sample of the workload."""
    import numpy as np

    from oracle import Oracle
    from paper_2209_08001_amd import workloads as W

    wl = W.WORKLOADS[wl_name]
    sizes = [32, 48, 64]
    times = []
    used = []
    t_all = time.perf_counter()
    wall = cpu = 0.0
    for s in sizes:
        n = (s, s)
        c0, e0 = W.init_fields(n, wl["seed"], cbar=wl["cbar"])
        o = Oracle(n, W.H, W.DEFAULT_MODEL, c0, e0)
        t0, c0_cpu = time.perf_counter(), time.process_time()
        o.step(wl.get("dt_min", wl.get("dt")))
        times.append(time.perf_counter() - t0)
        wall += times[-1]
        cpu += time.process_time() - c0_cpu
        used.append(s * s)
        if time.perf_counter() - t_all > budget_s:
            break
    # power-law fit t = a N^b over the sampled sizes, evaluated at the workload's size
    lx = np.log(np.array(used, float))
    ly = np.log(np.array(times))
    b, a = np.polyfit(lx, ly, 1) if len(used) > 1 else (1.0, ly[0] - lx[0])
    Nw = float(np.prod(wl["n"]))
    t_w = math.exp(a) * Nw ** b
    # threads actually used: process CPU time over wall time of the timed solves
    threads = max(1, round(cpu / wall)) if wall > 0 else 1
    return {
        "value": 1.0 / t_w,
        "unit": "steps/s",
        "cores": threads,
        "cpu_time_over_wall": cpu / wall if wall > 0 else None,
        "kind": "oracle",
        "sample": (f"first step (dt = dt_min) of the seeded trajectory on {', '.join(f'{s}x{s}' for s in sizes[:len(used)])} "
                   f"(measured {', '.join(f'{t:.2f}' for t in times)} s), extrapolated to {wl['n'][0]}x{wl['n'][1]} "
                   f"by the fitted N^{b:.2f} law of the sparse-LU Newton solve"),
    }


def run_ensemble(args, wl):
    """Ensemble workload: every instance takes K adaptive steps; the instances are stepped
    together (pfnks_batch_step, one stream per instance).  value = instance steps per second
    over the whole ensemble."""
    import torch

    from paper_2209_08001_amd import pfnks
    from paper_2209_08001_amd import workloads as W
    from paper_2209_08001_amd.driver import adaptive_batch_run

    members = W.ensemble_members(wl)
    solver = dict(W.DEFAULT_SOLVER, sweeps=args.sweeps or W.default_sweeps(2, args.precision == "mixed"),
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
        "config": {"workload": args.workload, "instances": k, "total_nodes": nodes,
                   "sides": sorted({p.n[0] for p in probs}), "precision": args.precision,
                   "preconditioner": args.pc, "host_threads": args.threads},
        "node_steps_per_s": nodes * args.steps / elapsed,
        "p50_round_ms": 1e3 * percentile(lat, 50),
        "p99_round_ms": 1e3 * percentile(lat, 99),
        "newton_per_step": newton / (k * args.steps),
        "gmres_per_newton": gmres / max(newton, 1),
        "retries": sum(s["retries"] for ss in stats for s in ss),
        "roofline": None,
    }
    for p in probs:
        p.close()
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
                  pc=pc_names()[args.pc],
                  precision=pfnks.MIXED if args.precision == "mixed" else pfnks.FP64)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    mk = lambda seed: poisson_requests(wl["rate"], wl["window"], seed, wl["sides2d"], wl["sides3d"],
                                       wl["frac3d"], args.steps if args.steps_given else wl["steps"])
    if args.warmup > 0:
        Server(solver, wl, budget, threads=args.threads).run(mk(wl["seed"] + 1000)[:4], realtime=False)
    reqs = mk(wl["seed"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Server(solver, wl, budget, threads=args.threads).run(reqs, realtime=True)
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
                   "window_s": wl["window"], "steps_per_request": reqs[0].steps if reqs else 0,
                   "hbm_budget_bytes": budget, "precision": args.precision, "host_threads": args.threads},
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
    ap.add_argument("--autotune", action="store_true",
                    help="pick tile / overlap / sweeps by timing candidates first (reported in config)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="mixed: float Krylov basis and Schwarz/Fourier preconditioner, double "
                         "residual, J v arithmetic, Newton update, energy and mass")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-roofline", action="store_true")
    ap.add_argument("--threads", type=int, default=16,
                    help="ensemble workloads: host threads driving the instances (pfnks_batch_step)")
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
                  pc=pc_names()[args.pc],
                  precision=pfnks.MIXED if args.precision == "mixed" else pfnks.FP64)
    if len(n) == 3:
        solver.update(tile=(8, 8, 8), overlap=1, sweeps=args.sweeps or W.default_sweeps(3, args.precision == "mixed"))
    if args.tile:
        t = tuple(int(v) for v in args.tile.split(","))
        solver["tile"] = t if len(t) == 3 else (t[0], t[1], 1)
    if args.overlap is not None:
        solver["overlap"] = args.overlap
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
            "autotuned": tuned,
            "gmres_restart": solver["gmres_restart"],
            "newton_rtol": solver["newton_rtol"],
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
        roof = p.roofline(HBM_PEAK_GBS)
        traffic, summary = measured_traffic(roof["kernel"], args.workload, args.precision,
                                            solver["tile"][:len(n)], solver["overlap"])
        roof["traffic"] = traffic
        if traffic is not None:
            roof["traffic_over_algorithmic"] = traffic / roof["bytes_per_launch"]
            roof["traffic_source"] = summary
        out["roofline"] = roof
    p.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
