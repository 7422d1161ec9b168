"""Constant-potential charge solve (oracle, FP64).

Test infrastructure only (see the package docstring).

Sec. 2, Eqs. (7)-(11): with Psi = A Q - b = psibar e + Delta psi d, where
d_j = -1/2 on the negative and +1/2 on the positive electrode, and total
neutrality e^T Q = 0,

    psibar = -e^T A^-1 (Delta psi d + b) / (e^T A^-1 e)            (Eq. (9))
    Q      = J A^-1 (Delta psi d + b),
    J      = I - A^-1 e e^T / (e^T A^-1 e)                          (Eqs. (10), (11)).

J A^-1 v is formed as x - g (e^T x)/(e^T g) with x = A^-1 v and g = A^-1 e,
which is the product of Eq. (11) with A^-1 v written out; the solves use a
Cholesky factorisation of the symmetric positive-definite A.
"""

import numpy as np
from scipy.linalg import cho_factor, cho_solve


def side_vector(ele_side):
    """d of Eq. (7): -1/2 on the negative electrode (side -1), +1/2 on the positive (side +1)."""
    s = np.asarray(ele_side)
    if not np.all((s == 1) | (s == -1)):
        raise ValueError("electrode side must be -1 or +1")
    return 0.5 * s.astype(np.float64)


class Solver:
    """Factorises A once (A is constant, Sec. 2) and solves Eqs. (9)-(10) for any b."""

    def __init__(self, A):
        self.A = np.asarray(A, dtype=np.float64)
        self.cho = cho_factor(self.A, lower=True)
        n = len(self.A)
        self.g = cho_solve(self.cho, np.ones(n))
        self.eg = float(np.sum(self.g))

    def solve(self, ele_side, dpsi, b):
        """Return (Q, psibar) for one right-hand side b (shape (N_ele,))."""
        v = dpsi * side_vector(ele_side) + np.asarray(b, dtype=np.float64)
        x = cho_solve(self.cho, v)
        psibar = -np.sum(x) / self.eg
        Q = x + psibar * self.g
        return Q, psibar

    def inverse_projected(self):
        """S = J A^-1 as a dense matrix (Eq. (10) without the right-hand side)."""
        Ainv = cho_solve(self.cho, np.eye(len(self.A)))
        return Ainv - np.outer(self.g, self.g) / self.eg
