"""Fit of the synthetic chemical coefficients (L0, U1, U4) used by the workloads.

Test infrastructure only (see the package docstring).  Run as
``python -m oracle.fit_coefficients``; it prints the fitted values.

The paper does not print the CALPHAD coefficients (Appendix A cites a
database).  It does print the two equilibria at 1037 K: the disordered gamma
phase at (c, eta) = (0.137, 1) and the ordered gamma' phase at (0.229, 0.02).
With e0 = L1 = L2 = L3 = 0 the reduced density (eta_1 = eta_2 = eta_3 = eta) is
linear in (L0, U1, U4), so three conditions fix them:
  d f/d eta (0.229, 0.02) = 0,
  d f/d c (0.137, 1) = d f/d c (0.229, 0.02)          (equal chemical potentials),
  f(0.229, 0.02) - f(0.137, 1) = mu (0.229 - 0.137)    (common tangent).
Derivatives are taken by complex step of the oracle's density.
"""

import numpy as np

from .model import Model, chem_density


def _f(m, c, e):
    return chem_density(c, [e, e, e], m)


def _d(m, c, e, which, h=1e-30):
    if which == "c":
        return np.imag(_f(m, complex(c, h), e)) / h
    return np.imag(_f(m, c, complex(e, h))) / h


def conditions(base, L0, U1, U4):
    m = Model.from_dict(dict(base, L=(L0, 0.0, 0.0, 0.0), U1=U1, U4=U4, e0=0.0))
    ca, ea, cb, eb = 0.137, 1.0, 0.229, 0.02
    mu_a = _d(m, ca, ea, "c")
    mu_b = _d(m, cb, eb, "c")
    return np.array([
        _d(m, cb, eb, "e"),
        mu_a - mu_b,
        np.real(_f(m, cb, eb) - _f(m, ca, ea)) - mu_a * (cb - ca),
    ])


def fit(base):
    r0 = conditions(base, 0.0, 0.0, 0.0)
    A = np.zeros((3, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = 1.0
        A[:, k] = conditions(base, *e) - r0
    return np.linalg.solve(A, -r0)


if __name__ == "__main__":
    base = {
        "theta": 8.314462618 * 1037.0 / (1.48e-5 * 3.3e7), "w_c": 1.0, "e0": 0.0, "L": (0, 0, 0, 0),
        "U1": 0.0, "U4": 0.0, "gamma_c": 0.0, "gamma_eta": 0.0, "kappa": 0.008, "L_eta": 1.0,
        "eps0": 0.049, "C11": 0.0, "C12": 0.0, "C44": 0.0,
    }
    for wc in (1.0, 0.0):
        L0, U1, U4 = fit(dict(base, w_c=wc))
        print(f"w_c={wc}: L0={L0:.6f} U1={U1:.6f} U4={U4:.6f}")
