"""Periodic cell-centred grid and the difference operators of Section 3.

Test infrastructure only (see the package docstring).

Section 3 writes the operators in 1D on x_i = (i - 1/2) dx:
  D^+ w_i = (w_{i+1} - w_i)/dx,  D^- w_i = (w_i - w_{i-1})/dx,
  D-hat w_i = (w_{i+1} - w_{i-1})/(2 dx),
  [(D^+- w)^2]_i = ((D^+ w_i)^2 + (D^- w_i)^2)/2,
  [D M D w]_i = (M_{i+1/2}(w_{i+1} - w_i) - M_{i-1/2}(w_i - w_{i-1}))/dx^2,
  M_{i+1/2} = kappa (c_i(1 - c_i) + c_{i+1}(1 - c_{i+1}))/2 at t_n.
The multi-dimensional operators are their tensor-product sums over directions
k (reading: the paper states the scheme in 1D "without loss of generality").

Arrays are (..., [Nz,] Ny, Nx): direction k = 0 is x (last axis), k = 1 is y,
k = 2 is z.  Both numpy-roll forms (used by the residual) and scipy.sparse forms
(used by the Jacobian) are provided; they are separate code paths on purpose.
"""

import numpy as np
import scipy.sparse as sp


class Grid:
    def __init__(self, n, h):
        """n: sizes per direction (x first), h: spacing (periodic box of side n_k h)."""
        self.n = tuple(int(v) for v in n)
        self.d = len(self.n)
        self.h = float(h)
        self.shape = tuple(reversed(self.n))  # numpy shape, x fastest
        self.N = int(np.prod(self.n))

    # ---- roll-based operators -------------------------------------------------
    def shift(self, w, k, s):
        """w_{i + s e_k} (periodic)."""
        return np.roll(w, -s, axis=w.ndim - 1 - k)

    def Dp(self, w, k):
        return (self.shift(w, k, 1) - w) / self.h

    def Dm(self, w, k):
        return (w - self.shift(w, k, -1)) / self.h

    def Dhat(self, w, k):
        return (self.shift(w, k, 1) - self.shift(w, k, -1)) / (2.0 * self.h)

    def lap(self, w):
        """Delta_h = sum_k D_k^+ D_k^-."""
        return sum(self.Dp(self.Dm(w, k), k) for k in range(self.d))

    def face_mobility(self, cn, kappa, k):
        """M_{i+1/2 e_k} from c at t_n (Section 3, below the definition of D M D)."""
        g = cn * (1.0 - cn)
        return kappa * 0.5 * (g + self.shift(g, k, 1))

    def div_M_grad(self, g, cn, kappa):
        """[nabla_h . M nabla_h g]_i = sum_k D_k (M D_k g) at faces i +- 1/2 e_k."""
        out = np.zeros_like(g)
        for k in range(self.d):
            Mp = self.face_mobility(cn, kappa, k)      # M_{i+1/2}
            Mm = self.shift(Mp, k, -1)                 # M_{i-1/2}
            out = out + (Mp * (self.shift(g, k, 1) - g) - Mm * (g - self.shift(g, k, -1))) / self.h ** 2
        return out

    def mean(self, w):
        return float(np.mean(w))

    def integral(self, w):
        """<w> := h^d sum_i w_i (Section 3, the bracket below eq. (neq:02))."""
        return float(np.sum(w)) * self.h ** self.d

    # ---- sparse operators -------------------------------------------------------
    def _idx(self):
        return np.arange(self.N).reshape(self.shape)

    def Pshift(self, k, s):
        """Sparse P with (P w)_i = w_{i + s e_k}."""
        idx = self._idx()
        tgt = np.roll(idx, -s, axis=self.d - 1 - k)
        return sp.csr_matrix((np.ones(self.N), (idx.ravel(), tgt.ravel())), shape=(self.N, self.N))

    def sDp(self, k):
        return (self.Pshift(k, 1) - sp.identity(self.N)) / self.h

    def sDm(self, k):
        return (sp.identity(self.N) - self.Pshift(k, -1)) / self.h

    def sDhat(self, k):
        return (self.Pshift(k, 1) - self.Pshift(k, -1)) / (2.0 * self.h)

    def slap(self):
        return sum(self.sDp(k) @ self.sDm(k) for k in range(self.d))

    def sdiv_M_grad(self, cn, kappa):
        """Sparse sum_k D_k^- diag(M_{.+1/2 e_k}) D_k^+."""
        out = sp.csr_matrix((self.N, self.N))
        for k in range(self.d):
            Mp = self.face_mobility(cn, kappa, k).ravel()
            out = out + self.sDm(k) @ sp.diags(Mp) @ self.sDp(k)
        return out

    def parity_class(self):
        """Index of each node's parity class: i_k mod 2 in every direction of even size.

        The central difference D-hat annihilates exactly the functions that are
        constant on each class, so these classes label the displacement gauge."""
        cls = np.zeros(self.shape, dtype=np.int64)
        mult = 1
        for k in range(self.d):
            if self.n[k] % 2 == 0:
                ik = np.indices(self.shape)[self.d - 1 - k]
                cls = cls + mult * (ik % 2)
                mult *= 2
        return cls, mult
