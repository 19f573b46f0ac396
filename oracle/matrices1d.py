"""Univariate matrices (App. B.3 and Sec. 3.3 of the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

With N_i = N_{i,p} and M_i = M_{i,p-1} (``oracle.splines``):

    M_ij  = int N_i N_j        K_ij  = int N_i' N_j'      C_ij  = int N_i M_j'
    M^_ij = int M_i M_j        K^_ij = int M_i' M_j'      C^_ij = int N_i' M_j
    N^_ij = M_i(1) M_j(1) + M_i(0) M_j(0)
    B^_ij = M_i(1) M_j'(1) - M_i(0) M_j'(0)
    T^    = 1/2 (K^ + 2 C_pen/h N^ - B^ - B^^T)          (Sec. 3.3)

All integrals over [0, 1] by element-wise Gauss--Legendre quadrature with
p+1 points, which is exact for these polynomial integrands.

The strong condition v.n = 0 (Sec. 3.1) removes N_1 and N_n in the normal
direction of each velocity component; ``interior`` rows/columns keep
indices 2..n-1.
"""
import numpy as np

from .splines import SplinePair, gauss_points


class Matrices1D:
    """All univariate matrices of one direction for (E, p, C_pen)."""

    def __init__(self, E, p, c_pen, nquad=None):
        sp = SplinePair(E, p)
        self.E, self.p, self.c_pen = E, p, c_pen
        self.n = sp.n
        self.h = 1.0 / E
        x, w = gauss_points(E, p, nquad)
        N, dN = sp.N(x)
        Mf, dMf = sp.M(x)
        W = w[None, :]
        self.M = (N * W) @ N.T
        self.K = (dN * W) @ dN.T
        self.C = (N * W) @ dMf.T
        self.Mc = (Mf * W) @ Mf.T
        self.Kc = (dMf * W) @ dMf.T
        self.Cc = (dN * W) @ Mf.T
        m0, dm0 = sp.M(np.array([0.0]))
        m1, dm1 = sp.M(np.array([1.0]))
        m0, dm0, m1, dm1 = m0[:, 0], dm0[:, 0], m1[:, 0], dm1[:, 0]
        self.Nc = np.outer(m1, m1) + np.outer(m0, m0)
        self.Bc = np.outer(m1, dm1) - np.outer(m0, dm0)
        self.alpha = c_pen / self.h
        self.Tc = 0.5 * (self.Kc + 2.0 * self.alpha * self.Nc - self.Bc - self.Bc.T)
        # interior N functions (v.n = 0 imposed strongly)
        it = slice(1, self.n - 1)
        self.M_int = self.M[it, it]
        self.K_int = self.K[it, it]
        self.C_int = self.C[it, :]        # rows: interior N, cols: all M
        self.Cc_int = self.Cc[it, :]      # rows: interior N, cols: all M
        # 1D load-vector pieces used by the lid right-hand side
        self.int_N = (N * W).sum(axis=1)[it]
        self.int_M = (Mf * W).sum(axis=1)
        self.M_at1 = m1
        self.dM_at1 = dm1
        self.sp = sp

    @property
    def nN(self):
        """Number of interior degree-p functions, n - 2."""
        return self.n - 2

    @property
    def nM(self):
        """Number of degree p-1 functions, n - 1."""
        return self.n - 1


def difference_matrix(n):
    """D_n of App. B.1: (n-1) x n with rows (-1, 1)."""
    D = np.zeros((n - 1, n))
    for i in range(n - 1):
        D[i, i] = -1.0
        D[i, i + 1] = 1.0
    return D
