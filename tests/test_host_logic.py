"""Host logic of the package that runs without a GPU.

* The adaptive step-size clock of the driver (Section 4, eq. (sencondt) and the retry rule),
  checked against the oracle's prediction of the same rule.
* The seeded Poisson arrivals of the serving workload.
* The autotuner's candidate set against the library's own host-side validation
  (pfnks_workspace_bytes checks tile shapes and the tile kernel's LDS budget).
"""

import math
import os

import numpy as np
import pytest

from oracle import predict_dt
from paper_2209_08001_amd import workloads as W
from paper_2209_08001_amd.autotune import default_candidates
from paper_2209_08001_amd.driver import _Clock
from paper_2209_08001_amd.serve import poisson_requests

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2209_08001_amd", "libpfnks.so")


def test_clock_follows_the_step_size_rule():
    wl = W.WORKLOADS["pf2d_512"]
    c = _Clock(wl)
    assert c.next_dt() == wl["dt_min"]  # the first step takes dt_min
    for rate in (0.0, 0.05, 3.0, 1e6):
        c.rate = rate
        assert abs(c.next_dt() - predict_dt(rate, wl["dt_min"], wl["dt_max"], wl["zeta"])) <= 1e-15
    # a failed attempt: dt / sqrt(2), zeta doubled, and the doubled zeta is kept
    c.rate = 0.05
    dt = c.next_dt()
    dt2 = c.failed(dt)
    assert abs(dt2 - dt / math.sqrt(2.0)) <= 1e-15
    assert c.zeta == 2.0 * wl["zeta"] and c.retries == 1
    assert abs(c.next_dt() - predict_dt(0.05, wl["dt_min"], wl["dt_max"], 2.0 * wl["zeta"])) <= 1e-15
    # an accepted step: the change rate is the RMS change divided by dt
    c.accepted({"dx_rms": 0.3}, 0.5)
    assert c.rate == 0.6
    # retries give up below dt_min / 2^6: the 13th halving by sqrt(2) from dt_min crosses it
    d = wl["dt_min"]
    for _ in range(12):
        d = c.failed(d)
    with pytest.raises(RuntimeError):
        c.failed(d)


def test_poisson_requests_are_seeded_and_shaped():
    wl = W.WORKLOADS["serve_mix"]
    args = (wl["rate"], wl["window"], wl["seed"], wl["sides2d"], wl["sides3d"], wl["frac3d"], wl["steps"])
    a = poisson_requests(*args)
    b = poisson_requests(*args)
    assert [(r.n, r.seed, r.cbar, r.arrival) for r in a] == [(r.n, r.seed, r.cbar, r.arrival) for r in b]
    assert len(a) == 1289  # the serving workload: 60 s at 20 requests/s (1200 expected, sd 35)
    t = [r.arrival for r in a]
    assert all(0.0 < x <= wl["window"] for x in t) and t == sorted(t)
    for k, r in enumerate(a):
        assert r.rid == k and r.seed == 5000 + k and r.steps == wl["steps"]
        assert 0.13 <= r.cbar <= 0.21
        assert (len(r.n) == 2 and r.n[0] in wl["sides2d"]) or (len(r.n) == 3 and r.n[0] in wl["sides3d"])
    # a long window: the count, the mean gap and the 3D share follow rate and frac3d (4 sigma)
    many = poisson_requests(50.0, 200.0, 1, (64,), (32,), 0.3, 1)
    m = len(many)
    assert abs(m - 10000) < 4 * math.sqrt(10000)
    f3 = sum(len(r.n) == 3 for r in many) / m
    assert abs(f3 - 0.3) < 4 * math.sqrt(0.3 * 0.7 / m)
    gaps = np.diff([0.0] + [r.arrival for r in many])
    assert abs(gaps.mean() - 1 / 50.0) < 4 * (1 / 50.0) / math.sqrt(m)


@pytest.mark.parametrize("name,default", [
    ("pf2d_512", {"tile": (32, 32, 1), "overlap": 2, "sweeps": 8}),
    ("pf3d_128", {"tile": (8, 8, 8), "overlap": 1, "sweeps": 6}),
])
def test_autotune_candidates_against_host_validation(name, default):
    """Every default candidate is either accepted or rejected as an invalid argument (a tile
    beyond the LDS budget) by pfnks_workspace_bytes, which the autotuner calls before it
    allocates anything; the workload's own configuration is a candidate and is accepted."""
    if not os.path.exists(LIB):
        pytest.skip("libpfnks.so not built")
    from paper_2209_08001_amd import pfnks

    n = W.WORKLOADS[name]["n"]
    cands = default_candidates(len(n))
    assert default in cands
    for precision in (pfnks.FP64, pfnks.MIXED):
        accepted = []
        for cand in cands:
            sv = dict(W.DEFAULT_SOLVER, precision=precision, **cand)
            try:
                assert pfnks.workspace_bytes(n, W.H, W.DEFAULT_MODEL, sv) > 0
                accepted.append(cand)
            except pfnks.PfnksError as e:
                assert e.status == pfnks.PFNKS_EINVAL, (cand, e)
        assert default in accepted
        assert len(accepted) >= (2 * len(cands)) // 3, (precision, len(accepted), len(cands))


@pytest.mark.parametrize("dim,ncol", [(2, 5), (3, 7)])
def test_tile_colourings_separate_every_diamond(dim, ncol):
    """The multicolour orders of the Schwarz tile solve: colour (a + 2b) mod 5 in 2D,
    (a + 2b + 3c) mod 7 in 3D.  Two nodes coupled by the Jacobian (|da| + |db| (+ |dc|) <= 2,
    the 13- and 25-point diamonds) never share a colour, so a colour's nodes update at once
    exactly as sequential Gauss-Seidel would."""
    w = (1, 2, 3)[:dim]
    offsets = [o for o in np.ndindex(*(5,) * dim)]
    for o in offsets:
        d = [x - 2 for x in o]
        if 0 < sum(abs(x) for x in d) <= 2:
            assert sum(wi * di for wi, di in zip(w, d)) % ncol != 0, d
