"""Residual of scheme (NSOA-1), the discrete energy and the discrete mass.

Test infrastructure only (see the package docstring).

State layout: X has shape (n_f, *grid.shape) with fields
  X[0] = c,  X[1:4] = eta_1..eta_3,  X[4:4+d] = u_1..u_d   (n_f = 4 + d).
"""

import numpy as np

from .model import chem_density, dg_chem


def strain_el(u, c, cbar0, grid, m):
    """Discrete elastic strain (Section 3, below eq. (freeenergy)):
    eps_IJ = (D-hat_J u_I + D-hat_I u_J)/2 - delta_IJ eps0 (c - cbar0)."""
    d = grid.d
    eps = [[None] * d for _ in range(d)]
    for I in range(d):
        for J in range(d):
            e = 0.5 * (grid.Dhat(u[I], J) + grid.Dhat(u[J], I))
            if I == J:
                e = e - m.eps0 * (c - cbar0)
            eps[I][J] = e
    return eps


def stress(eps, m):
    """sigma = Lscale C : eps for the three-constant cubic C of Appendix A,
    eq. (elastic-energy): sigma_II = C11 eps_II + C12 sum_{K != I} eps_KK,
    sigma_IJ = 2 C44 eps_IJ (I != J); Section 5.1 scales C by Lscale."""
    d = len(eps)
    tr = sum(eps[K][K] for K in range(d))
    sig = [[None] * d for _ in range(d)]
    for I in range(d):
        for J in range(d):
            if I == J:
                sig[I][J] = m.Lscale * (m.C11 * eps[I][I] + m.C12 * (tr - eps[I][I]))
            else:
                sig[I][J] = m.Lscale * 2.0 * m.C44 * eps[I][J]
    return sig


def residual(X, Xn, dt, grid, m, cbar0):
    """F(X; X^n, dt) of scheme (NSOA-1) with the equilibrium (mechanicalequilibrium-dis).

      G_c   = G_chem,c  - eps0 sum_I sigma_bar_II  - gamma_c Delta_h c_bar      (G^1+G^{2,S}+G^3+G^4)
      G_eta = G_chem,eta_p                         - gamma_eta Delta_h eta_bar_p
      F_c   = (c^{n+1} - c^n)/dt - nabla_h.(M nabla_h G_c)      [A~ = diag(-D M D, 1)]
      F_eta = (eta^{n+1} - eta^n)/dt + L_eta G_eta
      F_u_I = sum_J D-hat_J sigma_IJ(u^{n+1}, c^{n+1})
    where bar is the t_{n+1/2} average, sigma the elastic stress of the
    t_{n+1} and t_n states (G^3 = -eps0 C eps^el_{n+1/2}), and M is the face
    mobility built from c^n (semi-implicit).  L_eta = 1 is the model as written
    (the eta-mobility is absorbed in the time unit, Appendix A).
    """
    d = grid.d
    c1, e1, u1 = X[0], X[1:4], X[4:4 + d]
    c0, e0, u0 = Xn[0], Xn[1:4], Xn[4:4 + d]
    sig1 = stress(strain_el(u1, c1, cbar0, grid, m), m)
    sig0 = stress(strain_el(u0, c0, cbar0, grid, m), m)
    Gc_chem, Ge_chem = dg_chem(c1, e1, c0, e0, m)
    trbar = sum(0.5 * (sig1[I][I] + sig0[I][I]) for I in range(d))
    Gc = Gc_chem - m.eps0 * trbar - m.gamma_c * grid.lap(0.5 * (c1 + c0))
    F = np.empty_like(X)
    F[0] = (c1 - c0) / dt - grid.div_M_grad(Gc, c0, m.kappa)
    for p in range(3):
        Gp = Ge_chem[p] - m.gamma_eta * grid.lap(0.5 * (e1[p] + e0[p]))
        F[1 + p] = (e1[p] - e0[p]) / dt + m.L_eta * Gp
    for I in range(d):
        F[4 + I] = sum(grid.Dhat(sig1[I][J], J) for J in range(d))
    return F


def energy(X, grid, m, cbar0):
    """Discrete free energy E~ of eqs. (relations)/(freeenergy), split into
    (chemical E1+E2, elastic E3, interfacial E4):

      E1+E2 = f(c, eta),  E3 = eps^el : sigma / 2,
      E4 = gamma_c/2 sum_k [(D_k^+- c)^2] + gamma_eta/2 sum_p sum_k [(D_k^+- eta_p)^2]
    with [(D^+- w)^2] = ((D^+ w)^2 + (D^- w)^2)/2 and <.> = h^d sum_i.
    The gradient term per order parameter is gamma_eta/2 |grad eta_i|^2
    (Appendix A, eq. (free energy)); with three equal order parameters it is
    the 3 gamma_eta/2 |grad eta|^2 of Section 2.
    """
    d = grid.d
    c, eta, u = X[0], X[1:4], X[4:4 + d]
    chem = grid.integral(chem_density(c, eta, m))
    eps = strain_el(u, c, cbar0, grid, m)
    sig = stress(eps, m)
    el = 0.0
    for I in range(d):
        for J in range(d):
            el = el + 0.5 * eps[I][J] * sig[I][J]
    elastic = grid.integral(el)

    def grad2(w):
        return sum(0.5 * (grid.Dp(w, k) ** 2 + grid.Dm(w, k) ** 2) for k in range(d))

    inter = 0.5 * m.gamma_c * grad2(c)
    for p in range(3):
        inter = inter + 0.5 * m.gamma_eta * grad2(eta[p])
    interfacial = grid.integral(inter)
    return chem + elastic + interfacial, (chem, elastic, interfacial)


def mass(X, grid):
    """Discrete mass <c> = h^d sum_i c_i (Theorem 3.2, item 1)."""
    return grid.integral(X[0])
