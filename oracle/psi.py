"""The logarithmic term Psi and its Taylor-stabilised first-order quotient.

Test infrastructure only (see the package docstring).

Section 2: Psi(z) = z ln z + (1 - z) ln(1 - z).
Section 3, the construction above eq. (D2-1): Psi_S(y, delta) is Psi plus its
Taylor terms delta^s Psi^(s)(y) / s! for s = 1 .. 2S, and the quotient
Psi_S[y1, y2] = (Psi_S(ybar, delta) - Psi_S(ybar, -delta)) / (2 delta) with
ybar = (y1 + y2)/2 and delta = (y2 - y1)/2.  The paper stresses that this is a
polynomial in delta; the even-order terms of the two expansions cancel, so the
polynomial is the sum over odd s of delta^(s-1) Psi^(s)(ybar) / s!, which is what
``psi_S_quotient`` evaluates (no subtraction, no division by delta).

All functions accept real or complex numpy arrays (the complex case serves the
complex-step Jacobian of ``model.dg_chem_jac``).
"""

import math

import numpy as np


def psi(z):
    """Psi(z) = z ln z + (1 - z) ln(1 - z)  (Section 2, definition of E_G)."""
    return z * np.log(z) + (1.0 - z) * np.log(1.0 - z)


def dpsi(z, s):
    """The s-th derivative of Psi.

    Psi' = ln z - ln(1 - z); for s >= 2 the derivatives of 1/z and 1/(1-z) give
    Psi^(s)(z) = (s-2)! [ (-1)^s z^(1-s) + (1-z)^(1-s) ].
    """
    if s == 0:
        return psi(z)
    if s == 1:
        return np.log(z) - np.log(1.0 - z)
    k = math.factorial(s - 2)
    return k * ((-1.0) ** s * z ** (1 - s) + (1.0 - z) ** (1 - s))


def psi_S_quotient(y1, y2, S):
    """Psi_S[y1, y2]: the Taylor-stabilised quotient of Section 3 (eq. (D2-1)).

    Psi_S(ybar, +d) - Psi_S(ybar, -d) keeps twice the odd-order terms
    d^s Psi^(s)(ybar)/s! (s = 1, 3, ..., 2S-1); dividing by 2d leaves
    sum_{s odd <= 2S} d^(s-1) Psi^(s)(ybar)/s!.
    """
    ybar = 0.5 * (y1 + y2)
    d = 0.5 * (y2 - y1)
    total = dpsi(ybar, 1)
    for s in range(3, 2 * S + 1, 2):
        total = total + d ** (s - 1) * dpsi(ybar, s) / math.factorial(s)
    return total


def psi_exact_quotient(y1, y2):
    """The exact quotient Psi[y1, y2] = (Psi(y1) - Psi(y2)) / (y1 - y2) of eq. (D2).

    Used only by tests as the quantity Psi_S approximates (unstable when
    y1 -> y2, which is why the paper replaces it)."""
    return (psi(y1) - psi(y2)) / (y1 - y2)
