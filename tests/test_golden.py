"""Pins against values the paper prints (tests/golden/, Appendix A): the dimensionless model
parameters of the workloads follow from the printed physical ones, and the synthetic chemical
coefficients put the two printed phases on a common tangent of the free energy with the
ordered phase at an extremum in eta (the conditions the coefficients were fitted to)."""

import os

import pytest

from oracle.fit_coefficients import conditions
from paper_2209_08001_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "appendix_a_parameters.txt")
R_GAS = 8.314462618  # J/(mol K), CODATA (not a value of the paper)


def golden():
    """name -> the numbers on its line (a trailing unit is skipped)."""
    def num(tok):
        try:
            return float(tok)
        except ValueError:
            return None

    vals = {}
    for line in open(GOLDEN):
        tok = line.split("#")[0].split()
        if tok:
            vals[tok[0]] = [x for x in map(num, tok[1:]) if x is not None]
    return vals


def test_dimensionless_parameters_follow_from_appendix_a():
    g = golden()
    V_m, gc, ge = g["V_m"][0], g["gamma_c"][0], g["gamma_eta"][0]
    dE, L, kappa, T = g["Delta_E"][0], g["L"][0], g["kappa"][0], g["T"][0]
    m = W.DEFAULT_MODEL
    assert m["theta"] == pytest.approx(R_GAS * T / (V_m * dE), rel=1e-12)
    assert m["gamma_c"] == pytest.approx(gc / (dE * L * L), rel=1e-12)
    assert m["gamma_eta"] == pytest.approx(ge / (dE * L * L), rel=1e-12)
    assert m["kappa"] == kappa
    # the magnitudes the design quotes (theta = 17.654, gamma_c = 33.67, gamma_eta = 0.0808)
    assert m["theta"] == pytest.approx(17.654, abs=5e-4)
    assert m["gamma_c"] == pytest.approx(33.67, abs=5e-3)
    assert m["gamma_eta"] == pytest.approx(0.0808, abs=5e-5)


def test_printed_phases_on_a_common_tangent():
    g = golden()
    (ea, ca), (eb, cb) = g["eq_gamma"], g["eq_gamma_prime"]
    assert (ca, ea, cb, eb) == (0.137, 1.0, 0.229, 0.02)  # the points the fit uses
    m = dict(W.DEFAULT_MODEL, C11=0.0, C12=0.0, C44=0.0)
    r = conditions(m, m["L"][0], m["U1"], m["U4"])
    # d f/d eta at gamma' = 0; equal chemical potentials; common tangent.  The coefficients are
    # stored to 7 significant digits, so the conditions hold to about 1e-5 of |mu| ~ 190.
    assert max(abs(x) for x in r) <= 1e-6 * 190.0
