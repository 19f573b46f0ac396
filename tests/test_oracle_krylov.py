"""Pins of the oracle's Krylov solvers and of the solved cavity.

* MINRES iterates equal scipy's preconditioned MINRES (library routine);
* FGMRES iterates equal the least-squares minimiser over the preconditioned
  Krylov space, formed by brute force (tiny size);
* the Krylov solution equals the direct (bordered LU) solution; the direct
  velocity is pointwise divergence-free (App. B.2);
* cavity symmetries under x -> 1-x and y -> 1-y;
* iteration counts reproduce Table 1 at 8^3 elements (soft, +-3).
"""
import os

import numpy as np
import pytest
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from oracle.assemble import KronSystem, kron3
from oracle.cases import cavity
from oracle.direct import DirectSolver, mean_zero_pressure
from oracle.krylov import fgmres, minres
from oracle.matrices1d import difference_matrix
from oracle.precond import BasePreconditioner, HyperPower


def test_minres_matches_scipy():
    S, b = cavity(3, 2)
    P0 = BasePreconditioner(S)
    Kop = lambda x: S.K @ x
    Minv = spla.LinearOperator(S.K.shape, matvec=P0.apply)
    for it in (3, 10, 20):
        ours = minres(Kop, P0.apply, b, tol=0.0, maxit=it)
        ref, _ = spla.minres(S.K, b, M=Minv, rtol=1e-30, maxiter=it)
        assert np.linalg.norm(ours.x - ref) <= 1e-9 * np.linalg.norm(ref)


def test_fgmres_equals_bruteforce_least_squares():
    S, b = cavity(2, 2)
    P0 = BasePreconditioner(S)
    K = S.K.toarray()
    Pm = np.column_stack([P0.apply(e) for e in np.eye(S.N)])
    for j in (2, 5, 9):
        res = fgmres(lambda x: K @ x, lambda v, i: P0.apply(v), b, tol=0.0, restart=50, maxit=j)
        # x_j minimises ||b - K x|| over x in P^{-1} span{b, K P^{-1} b, ...}
        W = [b / np.linalg.norm(b)]
        for _ in range(j - 1):
            w = K @ (Pm @ W[-1])
            for v in W:
                w -= (w @ v) * v
            for v in W:
                w -= (w @ v) * v
            W.append(w / np.linalg.norm(w))
        Z = Pm @ np.column_stack(W)
        y, *_ = np.linalg.lstsq(K @ Z, b, rcond=None)
        assert np.linalg.norm(res.x - Z @ y) <= 1e-8 * np.linalg.norm(Z @ y)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_krylov_solution_equals_direct_and_is_divergence_free(k):
    E, p = 4, 2
    S, b = cavity(E, p)
    H = HyperPower(S, 2, k)
    r = minres(lambda x: S.K @ x, H.apply, b, tol=1e-10, maxit=500)
    xd = DirectSolver(S).solve(b)
    xk = mean_zero_pressure(r.x, S.nV)
    assert np.linalg.norm(xk[:S.nV] - xd[:S.nV]) <= 1e-7 * np.linalg.norm(xd[:S.nV])
    assert np.linalg.norm(xk[S.nV:] - xd[S.nV:]) <= 1e-6 * np.linalg.norm(xd[S.nV:])
    # pointwise divergence: coefficients D u of the direct solution vanish
    n = S.m.n
    Dh = difference_matrix(n)[:, 1:-1]
    I = np.eye(n - 1)
    D = sps.hstack([kron3(I, I, Dh), kron3(I, Dh, I), kron3(Dh, I, I)])
    assert np.abs(D @ xd[:S.nV]).max() <= 1e-11 * np.abs(xd[:S.nV]).max()
    fF = F = fgmres(lambda x: S.K @ x, lambda v, i: H.apply(v), b, tol=1e-10)
    xf = mean_zero_pressure(fF.x, S.nV)
    assert np.linalg.norm(xf[:S.nV] - xd[:S.nV]) <= 1e-7 * np.linalg.norm(xd[:S.nV])


def test_cavity_symmetries():
    """Reflections x1 -> 1-x1 and x2 -> 1-x2 map the discrete cavity to itself
    (uniform symmetric knots): u1 even / u2 odd under x2 -> 1-x2 ... etc."""
    E, p = 4, 3
    S, b = cavity(E, p)
    x = DirectSolver(S).solve(b)
    o = S.offsets
    nN, nM = E + p - 2, E + p - 1
    u1 = x[o[0]:o[1]].reshape(nM, nM, nN)     # [i3, i2, i1]
    u2 = x[o[1]:o[2]].reshape(nM, nN, nM)
    u3 = x[o[2]:o[3]].reshape(nN, nM, nM)
    pr = x[o[3]:].reshape(nM, nM, nM)
    s = np.abs(x).max()
    tol = 1e-10 * s
    # y -> 1 - y (axis 1 of [i3, i2, i1]): u1, u3, p even; u2 odd
    assert np.abs(u1 - u1[:, ::-1, :]).max() < tol
    assert np.abs(u3 - u3[:, ::-1, :]).max() < tol
    assert np.abs(u2 + u2[:, ::-1, :]).max() < tol
    assert np.abs(pr - pr[:, ::-1, :]).max() < tol
    # x -> 1 - x (axis 2): the lid reverses, so u1 is even, u2, u3 odd,
    # and the (zero-mean) pressure is odd
    assert np.abs(u1 - u1[:, :, ::-1]).max() < tol
    assert np.abs(u2 + u2[:, :, ::-1]).max() < tol
    assert np.abs(u3 + u3[:, :, ::-1]).max() < tol
    assert np.abs(pr + pr[:, :, ::-1]).max() < tol


def _golden_table(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            v = [int(t) for t in line.split()]
            rows[v[0]] = v[1:]
    return rows


@pytest.mark.parametrize("k", [0, 1, 2])
def test_iteration_counts_table1_8cube(k):
    """MINRES counts at 8^3, degree 2 reproduce Table 1 within +-3."""
    table = _golden_table("table1_liddriven_8cube.txt")
    S, b = cavity(8, 2)
    H = HyperPower(S, 2, k)
    r = minres(lambda x: S.K @ x, H.apply, b, tol=1e-8, maxit=300)
    assert r.converged
    assert abs(r.iters - table[2][k]) <= 3
    assert r.true_relres < 1e-7


def test_default_penalty_reading():
    """C_pen = max(12.5, 2.5 (p+1)) (the paper is silent): 12.5 up to degree
    4; at degree 8 it keeps T^ positive definite from 6 elements on, where
    12.5 does not, and keeps sigma(P_{V,0}^{-1} A) at 8^3 inside (0, 2)."""
    import scipy.linalg as sla
    from oracle.assemble import default_c_pen
    from oracle.matrices1d import Matrices1D
    assert [default_c_pen(p) for p in (2, 3, 4, 6, 8)] == [12.5, 12.5, 12.5, 17.5, 22.5]
    m = Matrices1D(6, 8, default_c_pen(8))
    assert sla.eigh(m.Tc, m.Mc, eigvals_only=True)[0] > 0
    m = Matrices1D(5, 8, 12.5)
    assert sla.eigh(m.Tc, m.Mc, eigvals_only=True)[0] < 0


@pytest.mark.parametrize("p,k", [(6, 1), (8, 1)])
def test_iteration_counts_table1_high_degree(p, k):
    """MINRES counts at 8^3 for degrees 6 and 8 reproduce Table 1 within +-2
    under the default penalty."""
    table = {}
    path = os.path.join(os.path.dirname(__file__), "golden", "table1_liddriven_all.txt")
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            v = line.split()
            table[(int(v[0]), int(v[1]))] = [int(t) for t in v[2:7]]
    S, b = cavity(8, p)
    r = minres(lambda x: S.K @ x, HyperPower(S, 2, k).apply, b, tol=1e-8, maxit=300)
    assert r.converged and abs(r.iters - table[(8, p)][k]) <= 2
