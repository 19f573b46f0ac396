"""Direct solve of the saddle-point system (eq. ``systemmatrix``).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The pressure is fixed only up to a constant (Sec. 3.2: Q carries the
zero-mean constraint, which a Krylov solver need not impose).  In the
M-spline basis every pressure function has unit integral, so the zero-mean
condition on p_h is sum_i p_i = 0; it is appended as a Lagrange multiplier
row and column and the bordered matrix is factored by sparse LU.
"""
import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla


def bordered_matrix(K, nV, nQ):
    c = np.zeros(nV + nQ)
    c[nV:] = 1.0
    c = sps.csr_matrix(c[:, None])
    return sps.bmat([[K, c], [c.T, None]]).tocsc()


class DirectSolver:
    """Sparse-LU solver for K x = b with a zero-mean pressure."""

    def __init__(self, sysm):
        self.s = sysm
        self.lu = spla.splu(bordered_matrix(sysm.K, sysm.nV, sysm.nQ))

    def solve(self, b):
        rhs = np.concatenate([b, [0.0]])
        return self.lu.solve(rhs)[:-1]


def mean_zero_pressure(x, nV):
    """x with the mean of its pressure block removed (sum p_i = 0)."""
    y = x.copy()
    y[nV:] -= y[nV:].mean()
    return y
