"""Analytic sparse Jacobian J = dF/dX of the NSOA-1 residual (Section 4, eq. (eq:line-system)).

Test infrastructure only (see the package docstring).

The residual is linear in everything except the local chemical gradient
G_chem(V^{n+1}, V^n); that part enters through the per-node 4x4 block
B = dG_chem/dV^{n+1} (``model.dg_chem_jac``).  All stencil parts are assembled
from the scipy.sparse operators of ``grid``; the t_{n+1/2} averages contribute
a factor 1/2 to every t_{n+1} derivative.
"""

import scipy.sparse as sp

from .model import dg_chem_jac


def _stress_derivs(grid, m):
    """d sigma_IJ / d u_K (sparse) and d sigma_IJ / d c (scalar) for sigma = Lscale C : eps^el."""
    d = grid.d
    Dh = [grid.sDhat(k) for k in range(d)]
    dsu = [[[None] * d for _ in range(d)] for _ in range(d)]
    dsc = [[0.0] * d for _ in range(d)]
    for I in range(d):
        for J in range(d):
            for K in range(d):
                if I == J:
                    coef = m.C11 if K == I else m.C12
                    dsu[I][J][K] = m.Lscale * coef * Dh[K]
                else:
                    op = sp.csr_matrix((grid.N, grid.N))
                    if K == I:
                        op = op + Dh[J]
                    if K == J:
                        op = op + Dh[I]
                    dsu[I][J][K] = m.Lscale * m.C44 * op
            if I == J:
                dsc[I][J] = -m.Lscale * m.eps0 * (m.C11 + (d - 1) * m.C12)
    return Dh, dsu, dsc


def jacobian(X, Xn, dt, grid, m):
    """Sparse CSR Jacobian of ``scheme.residual`` at X (field-major, x fastest)."""
    d = grid.d
    N = grid.N
    nf = 4 + d
    Id = sp.identity(N, format="csr")
    Lap = grid.slap()
    Lm = grid.sdiv_M_grad(Xn[0], m.kappa)
    B = dg_chem_jac(X[0], X[1:4], Xn[0], Xn[1:4], m)  # (4, 4, *shape)
    Bd = [[sp.diags(B[a, b].ravel()) for b in range(4)] for a in range(4)]
    Dh, dsu, dsc = _stress_derivs(grid, m)

    blocks = [[None] * nf for _ in range(nf)]
    # c-row: F_c = (c1 - c0)/dt - Lm G_c
    trc = sum(dsc[I][I] for I in range(d))
    dGc_dc = Bd[0][0] + (-0.5 * m.eps0 * trc) * Id - 0.5 * m.gamma_c * Lap
    blocks[0][0] = Id / dt - Lm @ dGc_dc
    for p in range(3):
        blocks[0][1 + p] = -(Lm @ Bd[0][1 + p])
    for K in range(d):
        tru = sum(dsu[I][I][K] for I in range(d))
        blocks[0][4 + K] = -(Lm @ (-0.5 * m.eps0 * tru))
    # eta-rows: F_eta_p = (eta1 - eta0)/dt + L_eta G_eta_p
    for p in range(3):
        blocks[1 + p][0] = m.L_eta * Bd[1 + p][0]
        for q in range(3):
            blk = m.L_eta * Bd[1 + p][1 + q]
            if p == q:
                blk = blk + Id / dt - 0.5 * m.L_eta * m.gamma_eta * Lap
            blocks[1 + p][1 + q] = blk
    # u-rows: F_u_I = sum_J D-hat_J sigma_IJ(u1, c1)
    for I in range(d):
        blocks[4 + I][0] = Dh[I] * dsc[I][I]
        for K in range(d):
            blocks[4 + I][4 + K] = sum(Dh[J] @ dsu[I][J][K] for J in range(d))
    return sp.bmat(blocks, format="csr")
