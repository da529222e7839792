"""Lockstep problem groups (pfnks_group_*) against the single-problem path and the oracle.

A group steps `count` instances of one grid shape with one launch per kernel kind and phase;
each instance must follow the iteration pfnks_step takes on it alone.  The two differ only in
where the GMRES rotations and the cycle's triangular solve are computed (device instead of
host), i.e. by rounding, so a group member is compared with the same instance stepped alone
at 1e-9 relative to each field's max-norm (both stop within 1e-8 of the same root, and their
iterations differ by rounding only), and with the oracle's root at 1e-8 (the bound of every
step-parity test).
"""

import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2209_08001_amd import workloads as W

pytestmark = pytest.mark.gpu

_TRAJ = {}


def _cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _relmax(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _solver(n, prec, **kw):
    from paper_2209_08001_amd import pfnks

    sv = dict(W.DEFAULT_SOLVER, precision=pfnks.MIXED if prec == "mixed" else pfnks.FP64)
    if len(n) == 3:
        sv["tile"] = tuple(W.tile_side(k, 4, 1) for k in n)
        sv["overlap"] = 1
    else:
        sv["tile"] = (W.tile_side(n[0], 16, 2), W.tile_side(n[1], 16, 2), 1)
        sv["overlap"] = 2
    sv.update(kw)
    return sv


def _oracle_traj(n, seed, dts):
    key = (tuple(n), seed, tuple(dts))
    if key not in _TRAJ:
        c0, e0 = W.init_fields(n, seed)
        o = Oracle(n, W.H, W.DEFAULT_MODEL, c0, e0)
        traj = []
        for dt in dts:
            o.step(dt)
            traj.append(o.X.copy())
        _TRAJ[key] = traj
    return _TRAJ[key]


# (shape, precision, seeds, per-step dts of each instance): instances of one group take
# different step sizes, so their Newton and GMRES counts differ and the per-instance masks of
# every phase are exercised
CASES = [
    ((32, 32), "fp64", (5, 9, 13), [(0.01, 0.05, 0.002), (0.05, 0.01, 0.002)]),
    ((32, 32), "mixed", (5, 9, 13), [(0.01, 0.05, 0.002), (0.05, 0.01, 0.002)]),
    ((24, 40), "fp64", (21, 22), [(0.01, 0.04), (0.02, 0.01)]),
    ((8, 8, 8), "mixed", (7, 17), [(0.01, 0.03), (0.03, 0.01)]),
    # 3D with sides that are not powers of two: the general Fourier path (mixed-radix lines)
    ((6, 10, 14), "fp64", (3, 4), [(0.01, 0.02)]),
]


@pytest.mark.parametrize("n,prec,seeds,dts", CASES)
def test_group_equals_single_and_oracle(n, prec, seeds, dts):
    from paper_2209_08001_amd import pfnks

    _cuda()
    _note(f"group n={n} {prec} instances={len(seeds)}")
    fields = [W.init_fields(n, s) for s in seeds]
    sv = _solver(n, prec)
    g = pfnks.Group(n, W.H, W.DEFAULT_MODEL, sv, [f[0] for f in fields], [f[1] for f in fields])
    alone = [pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c, e) for c, e in fields]
    for k, step_dts in enumerate(dts):
        status, stats = g.step(step_dts)
        assert all(s == pfnks.PFNKS_OK for s in status), status
        launches, syncs = g.counters()
        for i, p in enumerate(alone):
            sa = p.step(step_dts[i])
            assert stats[i]["newton_its"] == sa["newton_its"], (k, i, stats[i], sa)
            assert abs(stats[i]["mass"] - sa["mass"]) <= 1e-13 * abs(sa["mass"]), (k, i)
        _note(f"  step {k}: newton {[s['newton_its'] for s in stats]} gmres {[s['gmres_its'] for s in stats]} "
              f"launches {launches} syncs {syncs}")
    for i, p in enumerate(alone):
        Xg, tg = g.get_state(i)
        Xa, ta = p.get_state()
        assert tg == pytest.approx(ta, rel=1e-15)
        d = max(_relmax(Xg[f], Xa[f]) for f in range(Xg.shape[0]))
        ref = _oracle_traj(n, seeds[i], tuple(dt[i] for dt in dts))[-1]
        e = max(_relmax(Xg[f], ref[f]) for f in range(Xg.shape[0]))
        _note(f"  instance {i}: vs alone {d:.2e}, vs oracle {e:.2e}")
        assert d <= 1e-9, (i, d)
        assert e <= 1e-8, (i, e)
    g.close()
    for p in alone:
        p.close()


def test_group_of_one_equals_single():
    """A group of one instance (the count-1 launch descriptor of every kernel) steps as the
    single problem does."""
    from paper_2209_08001_amd import pfnks

    _cuda()
    n = (64, 64)
    c0, e0 = W.init_fields(n, 3)
    sv = _solver(n, "fp64")
    g = pfnks.Group(n, W.H, W.DEFAULT_MODEL, sv, [c0], [e0])
    p = pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c0, e0)
    for dt in (0.01, 0.1, 1.0):
        status, st = g.step([dt])
        sa = p.step(dt)
        assert status == [pfnks.PFNKS_OK]
        assert st[0]["newton_its"] == sa["newton_its"] and st[0]["gmres_its"] == sa["gmres_its"]
        assert st[0]["energy"] == pytest.approx(sa["energy"], rel=1e-12)
    Xg, _ = g.get_state(0)
    Xa, _ = p.get_state()
    assert max(_relmax(Xg[f], Xa[f]) for f in range(Xg.shape[0])) <= 1e-9
    g.close()
    p.close()


def test_group_failures_match_single():
    """Instances of one group that do not converge within the Newton limit report ENOCONV and
    keep their state while the others advance, exactly as each instance does alone (statuses
    and states compared with single problems at the same settings)."""
    from paper_2209_08001_amd import pfnks

    _cuda()
    n = (32, 32)
    seeds = (31, 32, 33, 34)
    dts = (1e-3, 1.0, 0.02, 2.0)
    fields = [W.init_fields(n, s) for s in seeds]
    sv = _solver(n, "fp64", newton_maxit=2)
    g = pfnks.Group(n, W.H, W.DEFAULT_MODEL, sv, [f[0] for f in fields], [f[1] for f in fields])
    status, st = g.step(dts)
    for i, (c, e) in enumerate(fields):
        p = pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c, e)
        sa_status, sa = p.try_step(dts[i])
        assert status[i] == sa_status, (i, status[i], sa_status)
        Xg, tg = g.get_state(i)
        Xa, ta = p.get_state()
        assert tg == ta
        assert max(_relmax(Xg[f], Xa[f]) for f in range(Xg.shape[0])) <= 1e-9, i
        if sa_status != pfnks.PFNKS_OK:
            X0 = np.concatenate([c[None], e.reshape((3,) + c.shape)], axis=0)
            assert np.array_equal(Xg[:4], X0), i
        p.close()
    _note(f"  statuses {status}")
    g.close()


@pytest.mark.parametrize("pc", ["ras", "as", "rras"])
def test_group_schwarz_variants(pc):
    """The Schwarz variants of Section 4 that solve every field in the tiles (left-RAS,
    classical AS and right-RAS, the last two through the per-node gather of the tiles'
    extended solutions) in a group: every member within 1e-9 of the instance stepped alone and
    within 1e-8 of the oracle's root."""
    from paper_2209_08001_amd import pfnks

    _cuda()
    n = (32, 32)
    seeds = (51, 52)
    dts = (0.01, 0.03)
    code = {"ras": pfnks.PC_RAS, "as": pfnks.PC_AS, "rras": pfnks.PC_RRAS}[pc]
    sv = _solver(n, "fp64", pc=code)
    fields = [W.init_fields(n, s) for s in seeds]
    g = pfnks.Group(n, W.H, W.DEFAULT_MODEL, sv, [f[0] for f in fields], [f[1] for f in fields])
    status, st = g.step(dts)
    assert all(x == pfnks.PFNKS_OK for x in status), status
    for i, (c, e) in enumerate(fields):
        p = pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c, e)
        p.step(dts[i])
        Xg, _ = g.get_state(i)
        Xa, _ = p.get_state()
        d = max(_relmax(Xg[f], Xa[f]) for f in range(Xg.shape[0]))
        ref = _oracle_traj(n, seeds[i], (dts[i],))[-1]
        err = max(_relmax(Xg[f], ref[f]) for f in range(Xg.shape[0]))
        _note(f"  {pc} instance {i}: vs alone {d:.2e}, vs oracle {err:.2e}")
        assert d <= 1e-9 and err <= 1e-8, (i, d, err)
        p.close()
    g.close()


@pytest.mark.parametrize("case", ["pc_refresh", "spectral", "none", "3d_fp64"])
def test_group_solver_options(case):
    """Solver options in a group: the preconditioner rebuilt at every Newton iteration, the
    Fourier displacement block alone and no preconditioner (the copies of the unsolved blocks
    go through the per-instance launch), and 3D in FP64: every member within 1e-9 of the
    instance stepped alone and within 1e-8 of the oracle's root."""
    from paper_2209_08001_amd import pfnks

    _cuda()
    n = (8, 8, 8) if case == "3d_fp64" else (24, 24)
    kw = {"pc_refresh": dict(pc_refresh=1), "spectral": dict(pc=pfnks.PC_SPECTRAL),
          "none": dict(pc=pfnks.PC_NONE), "3d_fp64": {}}[case]
    sv = _solver(n, "fp64", **kw)
    seeds = (61, 62)
    dts = (0.002, 0.004) if case == "none" else (0.01, 0.004)
    fields = [W.init_fields(n, s) for s in seeds]
    g = pfnks.Group(n, W.H, W.DEFAULT_MODEL, sv, [f[0] for f in fields], [f[1] for f in fields])
    status, st = g.step(dts)
    assert all(x == pfnks.PFNKS_OK for x in status), status
    for i, (c, e) in enumerate(fields):
        p = pfnks.Problem(n, W.H, W.DEFAULT_MODEL, sv, c, e)
        sa = p.step(dts[i])
        assert st[i]["newton_its"] == sa["newton_its"], (i, st[i], sa)
        Xg, _ = g.get_state(i)
        Xa, _ = p.get_state()
        d = max(_relmax(Xg[f], Xa[f]) for f in range(Xg.shape[0]))
        ref = _oracle_traj(n, seeds[i], (dts[i],))[-1]
        err = max(_relmax(Xg[f], ref[f]) for f in range(Xg.shape[0]))
        _note(f"  {case} instance {i}: gmres {st[i]['gmres_its']} vs alone {d:.2e}, vs oracle {err:.2e}")
        assert d <= 1e-9 and err <= 1e-8, (i, d, err)
        p.close()
    g.close()
