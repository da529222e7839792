"""Seeded synthetic inputs and the model-parameter set shared by the HIP path and the oracle.

This module holds inputs only: no arithmetic of the method.  Tests, bench.py
and smoke() draw initial fields and parameters here and hand the same arrays
to both the C-ABI library and the CPU oracle.

Model parameters (dimensionless, Appendix A of Huang & Yang; hats dropped):
  theta     = R T / (V_m Delta E), T = 1037 K, V_m = 1.48e-5 m^3/mol, Delta E = 3.3e7 J/m^3
  gamma_c   = 2.5e-9 J/m / (Delta E L^2), gamma_eta = 6.0e-12 J/m / (Delta E L^2), L = 1.5 nm
  kappa     = 0.008 (c-mobility prefactor), eps0 = 0.049 (lattice misfit per unit c)
  L_eta     = 1 (eta-mobility, absorbed in the time unit)
The CALPHAD coefficients (e0, L0..L3, U1, U4) and the elastic constants are not
printed in the paper.  The synthetic set below keeps e0 = L1 = L2 = L3 = 0 and
fits (L0, U1, U4) so that the reduced energy has a common tangent between the
wells (c, eta) = (0.137, 1) and (0.229, 0.02) with d f / d eta = 0 at the
ordered well (the equilibria the paper quotes at 1037 K); oracle/fit_coefficients.py
reproduces the fit.  C11, C12, C44 are round positive-definite cubic values
of the magnitude of a Ni-base alloy's stiffness divided by Delta E.
"""

import numpy as np

R_GAS = 8.314462618
T_K = 1037.0
V_M = 1.48e-5
DELTA_E = 3.3e7
LENGTH = 1.5e-9

DEFAULT_MODEL = {
    "theta": R_GAS * T_K / (V_M * DELTA_E),
    "w_c": 1.0,
    "e0": 0.0,
    "L": (-173.2737, 0.0, 0.0, 0.0),
    "U1": -19.77085,
    "U4": 3.857830,
    "gamma_c": 2.5e-9 / (DELTA_E * LENGTH ** 2),
    "gamma_eta": 6.0e-12 / (DELTA_E * LENGTH ** 2),
    "kappa": 0.008,
    "L_eta": 1.0,
    "eps0": 0.049,
    "C11": 6000.0,
    "C12": 4000.0,
    "C44": 3000.0,
    "Lscale": 1.0,
    "S": 10,
    "n_eta": 3,
}

H = 0.25  # grid spacing of every experiment in Section 5

# Solver settings: Newton rtol 1e-8, GMRES rtol 1e-6 (Section 5), restart 30,
# Schwarz tiles 32 x 32 with overlap 2 for the 2D workloads.
DEFAULT_SOLVER = {
    "newton_rtol": 1e-8,
    # update test of the Newton stop: the last accepted correction below 1e-8 of every field's
    # max-norm (with the residual test alone the iterate can stop ~1e-8 from the root)
    "newton_stol": 1e-8,
    "newton_atol_rms": 1e-12,
    "newton_maxit": 20,
    "gmres_rtol": 1e-6,
    "gmres_atol_rms": 1e-14,
    "gmres_restart": 30,
    "gmres_maxit": 600,
    "tile": (32, 32, 1),
    "overlap": 2,
    # symmetric Gauss-Seidel sweeps of the tile solve (see default_sweeps), over-relaxed (SSOR):
    # measured on MI355X, 512^2 FP64 30-step runs (sweeps / omega -> steps/s): 8 / 1.0 148,
    # 8 / 1.2 162, 8 / 1.4 174, 8 / 1.6 165, 6 / 1.4 160, 10 / 1.4 176, 12 / 1.4 175;
    # 128^3 mixed 10-step runs: 6 / 1.0 13.1, 6 / 1.2 14.3, 6 / 1.4 14.6, 8 / 1.2 14.2, 4 / 1.2 13.3
    "sweeps": 8,
    "sor_omega": 1.4,
    "ls_alpha": 1e-4,
    "ls_max_halvings": 10,
}

def default_omega(dim, mixed):
    """Over-relaxation of the tile sweeps, as measured fastest per step on MI355X: 1.4, except
    2D in mixed precision, where 1.2 is (512^2 mixed 30-step runs, 8 sweeps: omega 1.0 180
    steps/s, 1.2 194, 1.4 185)."""
    return 1.2 if (dim == 2 and mixed) else 1.4


def default_sweeps(dim, mixed):
    """Gauss-Seidel sweeps of the tile solve, as measured fastest per step on MI355X: each
    sweep costs ~6 us per apply at 512^2 FP64 (~4 us mixed) and saves GMRES iterations
    (512^2 FP64: 6 sweeps 13.7 iterations per Newton step and 178 steps/s, 8 sweeps 11.7 and
    195, 10 and 12 sweeps the same speed as 8; mixed: 8 sweeps 244 steps/s; 128^3 mixed: 6
    sweeps, 4 and 8 slower)."""
    if dim == 3:
        return 6
    return 8


WORKLOADS = {
    # 2D 64 x 64, 10 fixed steps dt = 1e-2
    "pf2d_64": {"n": (64, 64), "seed": 1, "cbar": 0.17, "steps": 10, "dt": 1e-2},
    # 2D 512 x 512, adaptive dt in [1e-3, 1], 200 steps
    "pf2d_512": {"n": (512, 512), "seed": 2, "cbar": 0.17, "steps": 200,
                 "dt_min": 1e-3, "dt_max": 1.0, "zeta": 100.0},
    # 3D 128^3, adaptive dt in [1e-3, 1], 100 steps
    "pf3d_128": {"n": (128, 128, 128), "seed": 3, "cbar": 0.17, "steps": 100,
                 "dt_min": 1e-3, "dt_max": 1.0, "zeta": 100.0},
    # ensemble of 64 independent 2D instances (sides and mean compositions drawn from seed 4,
    # instance k's noise from seed 4000 + k), 50 adaptive steps each
    "ens2d_64": {"ensemble": True, "count": 64, "seed": 4, "sides": (128, 192, 256, 384, 512),
                 "cbar_range": (0.13, 0.21), "steps": 50, "dt_min": 1e-3, "dt_max": 1.0, "zeta": 100.0},
    # Section 5.1 single particle (one order parameter via the symmetric subspace): radius 7.5
    # at the centre, dt_1 = dt_min = 0.01, dt_max = 2, zeta = 100, on the paper's 80^3 grid
    "particle3d_80": {"n": (80, 80, 80), "particle": 7.5, "steps": 50,
                       "dt_min": 1e-2, "dt_max": 2.0, "zeta": 100.0},
    # the Section 5.4 (Table 2) preconditioner comparison in kind: the first 10 steps with a fixed
    # dt = 0.01 on the paper's 80^3 grid (the paper: 256 cores; here one GPU)
    "table2_3d": {"n": (80, 80, 80), "seed": 3, "cbar": 0.17, "steps": 10,
                  "dt_min": 1e-2, "dt_max": 1e-2, "zeta": 100.0},
    # serving: Poisson arrivals (20 requests/s over a 60 s window, seed 5), 70 % 2D (sides the
    # multiples of 64 up to 1024) and 30 % 3D (sides 64, 80, 96, 112, 128), 50 adaptive steps per
    # request, continuous batching (bench.py --window shortens the arrival window)
    "serve_mix": {"serve": True, "rate": 20.0, "window": 60.0, "seed": 5,
                  "sides2d": tuple(64 * k for k in range(1, 17)), "sides3d": (64, 80, 96, 112, 128),
                  "frac3d": 0.3, "steps": 50, "dt_min": 1e-3, "dt_max": 1.0, "zeta": 100.0},
}


def tile_side(side, largest, overlap):
    """Schwarz tile side for a grid side: the largest divisor of the side not above `largest`
    whose extended block (tile + 2 overlap) still fits in the side."""
    t = largest
    while side % t or t + 2 * overlap > side:
        t -= 1
    return t


def ensemble_members(wl):
    """Instances of an ensemble workload: list of {"n", "seed", "cbar"}.  Side and mean
    composition of instance k are the k-th draws of numpy.random.default_rng(wl["seed"])
    (side uniform over wl["sides"], then cbar uniform in wl["cbar_range"])."""
    rng = np.random.default_rng(wl["seed"])
    out = []
    for k in range(wl["count"]):
        side = int(rng.choice(np.array(wl["sides"])))
        cbar = float(rng.uniform(*wl["cbar_range"]))
        out.append({"n": (side, side), "seed": wl["seed"] * 1000 + k, "cbar": cbar})
    return out


def init_fields(n, seed, cbar=0.17, amp_c=0.01, eta_base=1.0, amp_eta=0.01):
    """Seeded initial state on a periodic grid of sizes n (x first).

    c = cbar + U(-amp_c, amp_c); eta_p = eta_base + U(-amp_eta, amp_eta), p = 1..3
    (eta_p = 1 is the disordered gamma matrix; the noise is the perturbation).
    Draw order: c, eta_1, eta_2, eta_3, each in C order with x fastest, from
    numpy.random.default_rng(seed) (PCG64).  Returns (c0, eta0) with shapes
    (*reversed(n)) and (3, *reversed(n)), float64.
    """
    shape = tuple(reversed(tuple(n)))
    rng = np.random.default_rng(seed)
    c0 = cbar + rng.uniform(-amp_c, amp_c, size=shape)
    eta0 = np.empty((3,) + shape)
    for p in range(3):
        eta0[p] = eta_base + rng.uniform(-amp_eta, amp_eta, size=shape)
    return c0, eta0


def particle_fields(n, h, radius, c_in=0.238, eta_in=0.01, c_out=0.1375, eta_out=0.99):
    """One spherical (circular in 2D) gamma' particle of the given radius (length units) at the
    centre of the periodic box, as in the single-particle runs of Section 5.1: c = c_in,
    eta = eta_in inside, c = c_out, eta = eta_out outside; all three order parameters equal
    (the one-order-parameter model is the symmetric subspace eta_1 = eta_2 = eta_3 of the
    three-parameter one, with L_eta = 3).  Returns (c0, eta0) like init_fields."""
    shape = tuple(reversed(tuple(n)))
    axes = [(np.arange(m) + 0.5) * h - 0.5 * m * h for m in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    inside = sum(g * g for g in grids) <= radius * radius
    c0 = np.where(inside, c_in, c_out).astype(np.float64)
    e = np.where(inside, eta_in, eta_out).astype(np.float64)
    eta0 = np.stack([e, e, e])
    return c0, eta0


# the one-order-parameter model of Sections 2-3 as the symmetric subspace of the three-parameter
# model: identical eta_p and L_eta = 3 (the three equal eta-rows then carry the 1/3 weights)
P1_MODEL = dict(DEFAULT_MODEL, L_eta=3.0)


def random_state(n, seed, cbar=0.17, amp=0.02, u_amp=1e-3):
    """A random valid full state X (c, eta_1..3, u_1..d) for kernel-level tests:
    shape (4 + d, *reversed(n)).  The displacement is random, not in equilibrium."""
    d = len(n)
    shape = tuple(reversed(tuple(n)))
    rng = np.random.default_rng(seed)
    X = np.empty((4 + d,) + shape)
    X[0] = cbar + rng.uniform(-amp, amp, size=shape)
    for p in range(3):
        X[1 + p] = 1.0 + rng.uniform(-5 * amp, 5 * amp, size=shape)
    for I in range(d):
        X[4 + I] = rng.uniform(-u_amp, u_amp, size=shape)
    return X
