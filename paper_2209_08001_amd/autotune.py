"""Autotuner for the Schwarz preconditioner's launch shape: tile, overlap and Gauss-Seidel
sweeps (and the GMRES restart), chosen by timing real steps on the GPU.

The trajectory is first advanced `warm` steps with the default configuration from the
initial state (the early steps have small dt and are not representative); every candidate
then restarts from that state and change rate and takes `steps` adaptive steps, timed with
the stream synchronised on both sides.  Candidates the library rejects (tile shape, LDS)
are skipped.  The result is the fastest candidate and the full table.
"""

import itertools
import time

from . import pfnks
from .driver import adaptive_run


def default_candidates(dim):
    """Tile shapes, overlaps and sweep counts around the measured optima (2D: 32 x 32 tiles,
    overlap 2, 8 sweeps; 3D: 8^3 tiles, overlap 1, 6 sweeps)."""
    if dim == 2:
        tiles = [(32, 32, 1), (32, 16, 1), (16, 32, 1), (64, 16, 1), (16, 16, 1)]
        overlaps = [1, 2, 3]
        sweeps = (6, 8, 10)
    else:
        tiles = [(8, 8, 8), (8, 8, 4), (16, 8, 4)]
        overlaps = [1, 2]
        sweeps = (4, 6, 8)
    return [{"tile": t, "overlap": o, "sweeps": s}
            for t, o, s in itertools.product(tiles, overlaps, sweeps)]


def autotune(n, h, model, solver, c0, eta0, wl, candidates=None, warm=10, steps=3, device="cuda:0"):
    import torch

    candidates = candidates or default_candidates(len(n))
    p = pfnks.Problem(n, h, model, solver, c0, eta0, device=device)
    _, st = adaptive_run(p, warm, wl)
    X, t = p.get_state()
    rate = st[-1]["dx_rms"] / st[-1]["dt"]
    p.close()
    del p
    table = []
    for cand in candidates:
        sv = dict(solver, **cand)
        try:
            q = pfnks.Problem(n, h, model, sv, c0, eta0, device=device)
        except pfnks.PfnksError:
            continue  # shape the tile kernel or the LDS does not hold
        q.set_state(X, t)
        torch.cuda.synchronize(device)
        t0 = time.perf_counter()
        _, sts = adaptive_run(q, steps, wl, rate0=rate)
        torch.cuda.synchronize(device)
        ms = 1e3 * (time.perf_counter() - t0) / steps
        table.append(dict(cand, ms_per_step=ms,
                          gmres_per_newton=sum(s["gmres_its"] for s in sts) / max(1, sum(s["newton_its"] for s in sts))))
        q.close()
        del q
    best = min(table, key=lambda r: r["ms_per_step"])
    return best, table
