"""Plain FP64 CPU oracle for one NSOA-1 time step of the Ni-alloy phase-field model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: it is used by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  It shares no code, header, table or
constant generator with the HIP path; the two meet only through the seeded
input arrays and the model-parameter dictionary that a test hands to both.

What it computes (Huang & Yang, "Parallel energy stable phase field simulations
of Ni-based alloys system"):

* the discrete free energy of Section 3, eqs. (relations)/(freeenergy), with the
  chemical energy of Appendix A (sublattice model, three order parameters) and
  the cubic elastic energy of Appendix A, eq. (elastic-energy);
* the discrete variational derivative G^S of Section 3 (G^1 as in Appendix B,
  G^{2,S} as in eq. (D2-1), G^3 and G^4 as in eq. (dvds-1) and the line above
  it), generalised to three order parameters;
* the residual F of scheme (NSOA-1) with the discrete mechanical equilibrium
  (mechanicalequilibrium-dis);
* its root, reached by plain Newton from X^n with an exact sparse LU solve of
  the analytic Jacobian (Section 4 describes an inexact Newton--Krylov--Schwarz
  route to the same root);
* the discrete mass <c> (Theorem 3.1/3.2) and the adaptive time-step rule of
  Section 4, eq. (sencondt), with its divergence retry.

Every function is in FP64 (numpy/scipy).  Each module's and function's
docstring names the passage it follows and, where the paper leaves that passage
silent or garbled, states the reading taken.

Parity status: every part is pinned by the CPU tests in ``tests/test_oracle_*``
except the adaptive time-step driver, whose sequence of step sizes is pinned
only by the written rule (parity unpinned against the paper: the paper prints
no step-size history).
"""

from .psi import psi, dpsi, psi_S_quotient, psi_exact_quotient  # noqa: F401
from .model import Model, chem_density, dg_chem, dg_chem_jac  # noqa: F401
from .grid import Grid  # noqa: F401
from .scheme import residual, energy, mass, strain_el, stress  # noqa: F401
from .jacobian import jacobian  # noqa: F401
from .solver import Oracle, elastic_init, newton_solve, predict_dt  # noqa: F401
