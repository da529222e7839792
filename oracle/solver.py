"""Root of the NSOA-1 system by plain Newton with exact sparse LU, plus the time driver.

Test infrastructure only (see the package docstring).

Section 4 solves F(X) = 0 each step by inexact Newton (Krylov + Schwarz) from
the previous state.  The oracle reaches the same root plainly: X_0 = X^n,
J S = -F solved exactly (scipy SuperLU), full steps, halving only when the
trial leaves the log domain or increases ||F||, stop once the update is below
1e-12 in max-norm (quadratic convergence then leaves an error at rounding).

Gauge.  The central difference D-hat annihilates functions constant on each
parity class (i_k mod 2 per even direction), so u is fixed only up to one
constant per component and class.  The class sums of the u-rows of F vanish
identically, so the first u-equation of each class is redundant; the oracle
replaces it by "update = 0" and afterwards moves u to zero mean on every class.
The strain, the energy and c, eta do not depend on this choice.
"""

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .grid import Grid
from .jacobian import jacobian, _stress_derivs
from .model import Model
from .scheme import residual, energy, mass, strain_el, stress


class NoConvergence(RuntimeError):
    pass


class DomainError(ValueError):
    pass


def in_domain(X):
    """0 < c < 1 and 0 < c eta_i < 1 for i = 1..4 (eta_4 = 4 - sum eta_p): the
    arguments of every Psi term (Section 2 / Appendix A) lie in (0, 1)."""
    c = X[0]
    e4 = 4.0 - X[1] - X[2] - X[3]
    args = [c, c * X[1], c * X[2], c * X[3], c * e4]
    return all(np.all(a > 0.0) and np.all(a < 1.0) for a in args) and np.all(np.isfinite(X))


def _gauge_rows(grid):
    cls, ncls = grid.parity_class()
    flat = cls.ravel()
    first = [int(np.argmax(flat == k)) for k in range(ncls)]
    return flat, ncls, first


def project_gauge(X, grid):
    """Zero mean of every displacement component on every parity class."""
    flat, ncls, _ = _gauge_rows(grid)
    d = grid.d
    for I in range(d):
        u = X[4 + I].ravel()
        for k in range(ncls):
            sel = flat == k
            u[sel] -= u[sel].mean()
        X[4 + I] = u.reshape(grid.shape)
    return X


def _pin(J, rhs, grid, field_offset, nfields, everywhere=False):
    """Replace the first equation of each (component, class) by 'unknown = 0'.

    With no elasticity (Lscale = 0) every displacement equation is void and
    every displacement unknown is pinned (``everywhere``)."""
    _, ncls, first = _gauge_rows(grid)
    nodes = range(grid.N) if everywhere else first
    J = J.tolil()
    for I in range(nfields):
        for k in nodes:
            r = (field_offset + I) * grid.N + k
            J.rows[r] = [r]
            J.data[r] = [1.0]
            rhs[r] = 0.0
    return J.tocsc(), rhs


def elastic_init(c0, grid, m, cbar0):
    """u^0 solving the discrete equilibrium sum_J D-hat_J sigma_IJ(u, c^0) = 0
    (eq. (mechanicalequilibrium-dis)); the energy identity of Theorem 3.1
    uses equilibrium at both time levels, so the initial u is solved for."""
    d = grid.d
    if m.Lscale == 0.0:
        return np.zeros((d,) + grid.shape)
    Dh, dsu, _ = _stress_derivs(grid, m)
    K = sp.bmat([[sum(Dh[J] @ dsu[I][J][Kc] for J in range(d)) for Kc in range(d)] for I in range(d)],
                format="csr")
    zero = [np.zeros(grid.shape) for _ in range(d)]
    sig = stress(strain_el(zero, c0, cbar0, grid, m), m)
    rhs = -np.concatenate([sum(grid.Dhat(sig[I][J], J) for J in range(d)).ravel() for I in range(d)])
    Kp, rhs = _pin(K, rhs, grid, 0, d)
    u = spla.spsolve(Kp, rhs)
    X = np.zeros((4 + d,) + grid.shape)
    X[4:] = u.reshape((d,) + grid.shape)
    project_gauge(X, grid)
    return X[4:]


def newton_solve(Xn, dt, grid, m, cbar0, maxit=30, step_tol=1e-12, max_halvings=30):
    """Root of F(X; X^n, dt) = 0 from X_0 = X^n.  Returns (X, info)."""
    d = grid.d
    X = Xn.copy()
    F = residual(X, Xn, dt, grid, m, cbar0)
    r0 = float(np.linalg.norm(F))
    hist = [r0]
    its = 0
    if r0 == 0.0:
        return X, {"newton_its": 0, "res0": r0, "res_final": r0, "hist": hist}
    for its in range(1, maxit + 1):
        J = jacobian(X, Xn, dt, grid, m)
        Jp, rhs = _pin(J, -F.ravel(), grid, 4, d, everywhere=(m.Lscale == 0.0))
        S = spla.splu(Jp).solve(rhs).reshape(X.shape)
        lam = 1.0
        rF = float(np.linalg.norm(F))
        for _ in range(max_halvings):
            Xt = X + lam * S
            if in_domain(Xt):
                Ft = residual(Xt, Xn, dt, grid, m, cbar0)
                rt = float(np.linalg.norm(Ft))
                if np.isfinite(rt) and (rt < rF or lam * np.max(np.abs(S)) <= step_tol):
                    break
            lam *= 0.5
        else:
            raise NoConvergence("line search exhausted")
        X, F = Xt, Ft
        hist.append(rt)
        if lam * np.max(np.abs(S)) <= step_tol:
            break
    else:
        raise NoConvergence("Newton iteration limit")
    project_gauge(X, grid)
    F = residual(X, Xn, dt, grid, m, cbar0)
    return X, {"newton_its": its, "res0": r0, "res_final": float(np.linalg.norm(F)), "hist": hist}


def predict_dt(dx_rate, dt_min, dt_max, zeta):
    """Eq. (sencondt): dt~ = max(dt_min, dt_max / sqrt(1 + zeta X_d'^2)),
    X_d' = ||X^n - X^{n-1}|| / dt_{n-1} (the caller passes X_d')."""
    return max(dt_min, dt_max / math.sqrt(1.0 + zeta * dx_rate ** 2))


class Oracle:
    """Same semantics as the C ABI: create from (c^0, eta^0), step(dt), energy(), mass(), state()."""

    def __init__(self, n, h, model, c0, eta0):
        self.grid = Grid(n, h)
        self.m = model if isinstance(model, Model) else Model.from_dict(model)
        g = self.grid
        d = g.d
        c0 = np.asarray(c0, dtype=np.float64).reshape(g.shape)
        eta0 = np.asarray(eta0, dtype=np.float64).reshape((3,) + g.shape)
        X = np.zeros((4 + d,) + g.shape)
        X[0] = c0
        X[1:4] = eta0
        if not in_domain(X):
            raise DomainError("initial state outside the log domain")
        self.cbar0 = float(np.mean(c0))
        X[4:] = elastic_init(c0, g, self.m, self.cbar0)
        self.X = X
        self.t = 0.0
        self.n = 0

    def step(self, dt):
        """One NSOA-1 step; on failure the state is left unchanged and NoConvergence raised."""
        Xn = self.X
        X, info = newton_solve(Xn, dt, self.grid, self.m, self.cbar0)
        diff = X[:4] - Xn[:4]
        info["dx_rms"] = float(np.sqrt(np.mean(diff ** 2)))
        self.X = X
        self.t += dt
        self.n += 1
        info["energy"] = self.energy()[0]
        info["mass"] = self.mass()
        return info

    def energy(self):
        return energy(self.X, self.grid, self.m, self.cbar0)

    def mass(self):
        return mass(self.X, self.grid)

    def state(self):
        d = self.grid.d
        return self.X[0].copy(), self.X[1:4].copy(), self.X[4:4 + d].copy(), self.t

    def advance(self, n_steps, dt_min, dt_max, zeta, retry_floor=2 ** -6, fail_hook=None):
        """Adaptive stepping of Section 4: predict dt by eq. (sencondt); when the
        solve fails, dt~ := dt~/sqrt(2) and zeta := 2 zeta, and retry (readings:
        the first step uses dt_min, the rate X_d' is the RMS change of c and eta
        per unit time, the doubled zeta persists, retries stop below
        dt_min * retry_floor).  Returns the list of per-step records."""
        log = []
        rate = None
        for _ in range(n_steps):
            dt = dt_min if rate is None else predict_dt(rate, dt_min, dt_max, zeta)
            retries = 0
            while True:
                try:
                    if fail_hook is not None and fail_hook(self.n, dt):
                        raise NoConvergence("forced")
                    info = self.step(dt)
                    break
                except NoConvergence:
                    dt = dt / math.sqrt(2.0)
                    zeta = 2.0 * zeta
                    retries += 1
                    if dt < dt_min * retry_floor:
                        raise
            rate = info["dx_rms"] / dt
            info.update(dt=dt, retries=retries, zeta=zeta, t=self.t)
            log.append(info)
        return log
