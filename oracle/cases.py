"""Benchmark problems: the 3D lid-driven cavity (Sec. 5, Fig. ``liddrivencavity``)
and its loss gradient for the differentiable solve.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Cavity: Omega = [0, 1]^3, viscosity nu, lid velocity (U, 0, 0) on x3 = 1,
no-slip on the other walls (tangential velocity weakly by Nitsche, normal
velocity strongly), optional separable body force.

Gradient (adjoint of the linear solve): with K x = F(beta, nu),
F = [F_lid(nu) + M_V beta; 0], and L = (u - u_t)^T M_V (u - u_t):

    K lambda = [dL/du; 0],   dL/du = 2 M_V (u - u_t)
    dL/dbeta = M_V lambda_u
    dL/dnu   = lambda^T (dF/dnu - dK/dnu x)
             = lambda_u^T (F_lid / nu - (A / nu) u)

(K is symmetric, A and F_lid are linear in nu, B carries no nu.)
"""
import numpy as np
import scipy.sparse as sps

from .assemble import KronSystem, kron3
from .direct import DirectSolver


def cavity(E, p, nu=1.0, U=1.0, modes=None, c_pen=None):
    """(system, right-hand side) of the cavity."""
    S = KronSystem(E, p, nu, c_pen)
    b = S.lid_rhs(U)
    if modes is not None:
        b = b + S.body_force_rhs(modes)
    return S, b


def velocity_mass(S):
    """Block-diagonal velocity mass matrix M_V (L2 inner product on V_h)."""
    m = S.m
    return sps.block_diag([kron3(m.Mc, m.Mc, m.M_int),
                           kron3(m.Mc, m.M_int, m.Mc),
                           kron3(m.M_int, m.Mc, m.Mc)]).tocsr()


class CavityLoss:
    """L(beta, nu) = ||u_h - u_t||^2_{L2} for the cavity with body force M_V beta."""

    def __init__(self, E, p, U=1.0, u_target=None, c_pen=None):
        self.E, self.p, self.U, self.c_pen = E, p, U, c_pen
        self.u_target = u_target

    def _system(self, nu):
        S = KronSystem(self.E, self.p, nu, self.c_pen)
        return S, S.lid_rhs(self.U)

    def solve(self, beta, nu):
        S, b = self._system(nu)
        MV = velocity_mass(S)
        b = b.copy()
        b[:S.nV] += MV @ beta
        x = DirectSolver(S).solve(b)
        return S, MV, b, x

    def value(self, beta, nu):
        S, MV, b, x = self.solve(beta, nu)
        d = x[:S.nV] - self.u_target
        return d @ (MV @ d)

    def gradient(self, beta, nu):
        """(L, dL/dbeta, dL/dnu) by one forward and one adjoint direct solve."""
        S, MV, b, x = self.solve(beta, nu)
        u = x[:S.nV]
        d = u - self.u_target
        L = d @ (MV @ d)
        rhs = np.zeros(S.N)
        rhs[:S.nV] = 2.0 * (MV @ d)
        lam = DirectSolver(S).solve(rhs)
        lu = lam[:S.nV]
        g_beta = MV @ lu
        F_lid = S.lid_rhs(self.U)[:S.nV]
        g_nu = lu @ (F_lid / nu - (S.A @ u) / nu)
        return L, g_beta, g_nu
