"""Chemical free energy and its discrete variational derivative (three order parameters).

Test infrastructure only (see the package docstring).

Appendix A writes the Gibbs energy of the gamma/gamma' sublattice model as
E^dis(c) + E^ord(c, eta_1, eta_2, eta_3) - E^ord(c, 1, 1, 1) with
  E^ord_0 = 6 U1 c^2 sum phi_k^2,  ideal part (RT/4) sum_{i=1..4} Psi(c eta_i),
  excess  = -2 U1 c^2 sum phi_k^2 + 12 U4 (1 - 2c) c^2 sum phi_k^2 - 48 U4 c^3 phi_1 phi_2 phi_3,
  phi_1 = 1 - (eta_1 + eta_2)/2, phi_2 = 1 - (eta_1 + eta_3)/2, phi_3 = 1 - (eta_2 + eta_3)/2,
  eta_4 = 4 - eta_1 - eta_2 - eta_3,
and E^dis = E0^Al c + E0^Ni (1 - c) + RT Psi(c) + c(1 - c) sum_k L_k (2c - 1)^k.
After dividing by V_m Delta E (hats dropped here) the density is

  f = p(c) + A(c) S2(phi) + B(c) P3(phi) + theta [ w_c Psi(c) + 1/4 sum_{i=1..4} Psi(c eta_i) ],
  p(c) = e0 c + c(1-c) sum_k L_k (2c-1)^k,  A(c) = 4 U1 c^2 + 12 U4 (1-2c) c^2,  B(c) = -48 U4 c^3,
  S2 = sum_k phi_k^2,  P3 = phi_1 phi_2 phi_3.

The RT Psi(c) of E^dis cancels against -E^ord(c,1,1,1) in Appendix A, while the
main text's E_G (Section 2) and the quotient (D2)/(D2-1) keep theta Psi(c): the
weight w_c selects between the two (reading: default 1, the scheme's form).
With eta_1 = eta_2 = eta_3 = eta this is the reduced energy of Section 2
(3 A phi^2 + B phi^3, Psi(c eta) three times and Psi(c(4 - 3 eta)) once).
"""

from dataclasses import dataclass, field

import numpy as np
from numpy.polynomial import polynomial as npoly

from .psi import psi, psi_S_quotient


@dataclass
class Model:
    """Dimensionless model parameters (Appendix A; hats dropped)."""

    theta: float
    e0: float
    L: tuple
    U1: float
    U4: float
    gamma_c: float
    gamma_eta: float
    kappa: float
    L_eta: float
    eps0: float
    C11: float
    C12: float
    C44: float
    Lscale: float = 1.0
    w_c: float = 1.0
    S: int = 10
    n_eta: int = 3
    extra: dict = field(default_factory=dict)

    @classmethod
    def from_dict(cls, d):
        keys = set(cls.__dataclass_fields__) - {"extra"}
        kw = {k: d[k] for k in d if k in keys}
        kw["L"] = tuple(float(x) for x in d["L"])
        return cls(**kw)


# --- polynomial pieces -----------------------------------------------------------

def _coeffs_p(m):
    """Monomial coefficients (ascending) of p(c) = e0 c + c(1-c) sum_k L_k (2c-1)^k."""
    coef = np.array([0.0, m.e0])
    base = np.array([0.0, 1.0, -1.0])  # c (1 - c)
    for k, Lk in enumerate(m.L):
        term = npoly.polymul(base, npoly.polypow([-1.0, 2.0], k)) * Lk
        coef = npoly.polyadd(coef, term)
    return coef


def _coeffs_A(m):
    """A(c) = 4 U1 c^2 + 12 U4 (1 - 2c) c^2: the sum-phi^2 coefficient (E^ord_0 + excess)."""
    return np.array([0.0, 0.0, 4.0 * m.U1 + 12.0 * m.U4, -24.0 * m.U4])


def _coeffs_B(m):
    """B(c) = -48 U4 c^3: the phi_1 phi_2 phi_3 coefficient of the excess energy."""
    return np.array([0.0, 0.0, 0.0, -48.0 * m.U4])


def _polyval(coef, x):
    out = np.zeros_like(x) if isinstance(x, np.ndarray) else 0.0 * x
    for k in range(len(coef) - 1, -1, -1):
        out = out * x + coef[k]
    return out


def _divdiff(coef, a, b):
    """Divided difference g[a, b] of a polynomial g written in expanded form.

    (a^m - b^m)/(a - b) = sum_{j<m} a^j b^(m-1-j); this is the form the paper
    writes in Appendix B and stays finite at a = b (no division)."""
    out = 0.0 * (a + b)
    for mpow in range(1, len(coef)):
        q = 0.0 * (a + b)
        for j in range(mpow):
            q = q + a ** j * b ** (mpow - 1 - j)
        out = out + coef[mpow] * q
    return out


def _phis(eta):
    e1, e2, e3 = eta
    return (1.0 - 0.5 * (e1 + e2), 1.0 - 0.5 * (e1 + e3), 1.0 - 0.5 * (e2 + e3))


# which phi_k contain eta_p (phi_1: eta_1, eta_2; phi_2: eta_1, eta_3; phi_3: eta_2, eta_3)
_PHI_OF_ETA = ((0, 1), (0, 2), (1, 2))


def chem_density(c, eta, m):
    """Dimensionless chemical free energy density f(c, eta_1..3) (Appendix A)."""
    e4 = 4.0 - eta[0] - eta[1] - eta[2]
    ph = _phis(eta)
    S2 = ph[0] ** 2 + ph[1] ** 2 + ph[2] ** 2
    P3 = ph[0] * ph[1] * ph[2]
    f = _polyval(_coeffs_p(m), c) + _polyval(_coeffs_A(m), c) * S2 + _polyval(_coeffs_B(m), c) * P3
    ideal = m.w_c * psi(c)
    for ei in (eta[0], eta[1], eta[2], e4):
        ideal = ideal + 0.25 * psi(c * ei)
    return f + m.theta * ideal


def dg_chem(c1, eta1, c0, eta0, m, S=None):
    """Chemical part of the discrete variational derivative, G^1 + G^{2,S}.

    Superscript 1 is t_{n+1}, 0 is t_n.  Returns (G_c, [G_eta_1, G_eta_2, G_eta_3]).

    G^1 (Appendix B, generalised): product-rule quotients of the polynomial
    part -- the c-direction takes time-averaged phi-factors times the expanded
    divided differences p[c1,c0], A[c1,c0], B[c1,c0]; the phi-direction takes
    time-averaged A, B times the exact quotient of phi_k^2 (2 phi_bar_k) and the
    averaged-vector-field quotient of phi_1 phi_2 phi_3, then the chain rule
    d phi_k / d eta_p = -1/2.
    G^{2,S} (eq. (D2-1), generalised): with y_i = c eta_i and the product rule
    Delta y_i = eta_bar_i Delta c + c_bar Delta eta_i (eta_4 = 4 - sum eta_p),
      G_c   += theta ( w_c Psi_S[c1,c0] + 1/4 sum_i eta_bar_i Psi_S[y_i^1, y_i^0] ),
      G_eta_p += theta/4 c_bar ( Psi_S[y_p^1, y_p^0] - Psi_S[y_4^1, y_4^0] ).
    With eta_1 = eta_2 = eta_3 the c-row equals Appendix B + (D2-1) and the sum
    of the three eta-rows equals the single eta-row there.
    """
    S = m.S if S is None else S
    e1 = list(eta1)
    e0 = list(eta0)
    e1.append(4.0 - e1[0] - e1[1] - e1[2])
    e0.append(4.0 - e0[0] - e0[1] - e0[2])
    f1 = _phis(eta1)
    f0 = _phis(eta0)
    S2_1 = f1[0] ** 2 + f1[1] ** 2 + f1[2] ** 2
    S2_0 = f0[0] ** 2 + f0[1] ** 2 + f0[2] ** 2
    P3_1 = f1[0] * f1[1] * f1[2]
    P3_0 = f0[0] * f0[1] * f0[2]
    cp, cA, cB = _coeffs_p(m), _coeffs_A(m), _coeffs_B(m)
    Abar = 0.5 * (_polyval(cA, c1) + _polyval(cA, c0))
    Bbar = 0.5 * (_polyval(cB, c1) + _polyval(cB, c0))

    # G^1, c-direction
    Gc = (_divdiff(cp, c1, c0) + 0.5 * (S2_1 + S2_0) * _divdiff(cA, c1, c0)
          + 0.5 * (P3_1 + P3_0) * _divdiff(cB, c1, c0))

    # G^1, phi-direction: d(phi_k^2) quotient and AVF quotient of the triple product
    T = []
    for k in range(3):
        a, b = [j for j in range(3) if j != k]
        T.append((f0[a] * f0[b] + f1[a] * f1[b]) / 3.0 + (f0[a] * f1[b] + f1[a] * f0[b]) / 6.0)
    Gphi = [Abar * (f1[k] + f0[k]) + Bbar * T[k] for k in range(3)]
    Ge = [-0.5 * (Gphi[_PHI_OF_ETA[p][0]] + Gphi[_PHI_OF_ETA[p][1]]) for p in range(3)]

    # G^{2,S}
    Q = [psi_S_quotient(c1 * e1[i], c0 * e0[i], S) for i in range(4)]
    logc = m.w_c * psi_S_quotient(c1, c0, S)
    for i in range(4):
        logc = logc + 0.25 * 0.5 * (e1[i] + e0[i]) * Q[i]
    Gc = Gc + m.theta * logc
    cbar = 0.5 * (c1 + c0)
    Ge = [Ge[p] + 0.25 * m.theta * cbar * (Q[p] - Q[3]) for p in range(3)]
    return Gc, Ge


def dg_chem_jac(c1, eta1, c0, eta0, m, h=1e-30):
    """Local block d(G_c, G_eta_1..3)/d(c1, eta1_1..3), a (4, 4, ...) array.

    Complex-step differentiation of ``dg_chem``: every piece of G_chem is an
    analytic function of the t_{n+1} values, so Im G(V + i h e_b)/h is the exact
    derivative up to rounding (no subtractive cancellation)."""
    V = [np.asarray(c1, dtype=np.complex128)] + [np.asarray(e, dtype=np.complex128) for e in eta1]
    shape = np.shape(V[0])
    out = np.zeros((4, 4) + shape)
    for b in range(4):
        Vb = [v.copy() for v in V]
        Vb[b] = Vb[b] + 1j * h
        Gc, Ge = dg_chem(Vb[0], Vb[1:], c0, eta0, m)
        out[0, b] = np.imag(Gc) / h
        for p in range(3):
            out[1 + p, b] = np.imag(Ge[p]) / h
    return out
