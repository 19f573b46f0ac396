"""Pins of the oracle's univariate splines and 1D matrices (App. B).

Each check is fixed by mathematics independent of the code under test:
partition of unity, unit integrals, polynomial reproduction (Greville
abscissae), finite-difference derivatives, the derivative identity
eq. ``reduction`` and the integration-by-parts relations between the
univariate matrices.
"""
import numpy as np
import pytest

from oracle.matrices1d import Matrices1D, difference_matrix
from oracle.splines import SplinePair, bspline_values_and_derivs, gauss_points, open_knots

CASES = [(1, 2), (3, 2), (4, 3), (5, 4), (7, 5)]


def _interior_points(E, n=57, seed=0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, n)
    # keep away from breakpoints where derivatives jump
    frac = (x * E) % 1.0
    return x[(frac > 1e-3) & (frac < 1 - 1e-3)]


@pytest.mark.parametrize("E,p", CASES)
def test_partition_of_unity_and_nonnegativity(E, p):
    sp = SplinePair(E, p)
    x = np.concatenate([np.linspace(0, 1, 101), _interior_points(E)])
    N, _ = sp.N(x)
    assert N.shape[0] == E + p
    assert np.allclose(N.sum(axis=0), 1.0, atol=1e-14)
    assert N.min() >= -1e-15


@pytest.mark.parametrize("E,p", CASES)
def test_M_splines_have_unit_integral(E, p):
    sp = SplinePair(E, p)
    x, w = gauss_points(E, p, p + 5)
    M, _ = sp.M(x)
    assert M.shape[0] == E + p - 1
    assert np.allclose(M @ w, 1.0, atol=1e-13)


@pytest.mark.parametrize("E,p", CASES)
def test_polynomial_reproduction_greville(E, p):
    """sum_i xi_i N_{i,p}(x) = x with the Greville abscissae (textbook)."""
    t = open_knots(E, p)
    n = E + p
    xi = np.array([t[i + 1:i + p + 1].mean() for i in range(n)])
    x = np.linspace(0, 1, 203)
    N, _ = bspline_values_and_derivs(t, p, x)
    assert np.allclose(xi @ N, x, atol=1e-14)


@pytest.mark.parametrize("E,p", CASES)
def test_derivatives_match_finite_differences(E, p):
    sp = SplinePair(E, p)
    x = _interior_points(E)
    h = 1e-6
    for fam in (sp.N, sp.M):
        _, d = fam(x)
        fd = (fam(x + h)[0] - fam(x - h)[0]) / (2 * h)
        assert np.allclose(d, fd, atol=1e-6 * max(1.0, np.abs(d).max()))


@pytest.mark.parametrize("E,p", CASES)
def test_derivative_identity_reduction(E, p):
    """(sum a_i N_i)' = sum (a_{i+1} - a_i) M_i  (eq. reduction)."""
    sp = SplinePair(E, p)
    rng = np.random.default_rng(1)
    a = rng.standard_normal(E + p)
    x = _interior_points(E)
    _, dN = sp.N(x)
    M, _ = sp.M(x)
    D = difference_matrix(E + p)
    assert np.allclose(a @ dN, (D @ a) @ M, atol=1e-11 * np.abs(a @ dN).max())


@pytest.mark.parametrize("E,p", CASES)
def test_univariate_matrix_relations(E, p):
    """Relations that follow from eq. reduction and integration by parts:
    C^ = D^T M^, K = D^T M^ D, C = [N M]_0^1 - C^, K 1 = 0, M 1 = int N."""
    m = Matrices1D(E, p, c_pen=12.5)
    n = m.n
    D = difference_matrix(n)
    sc = np.abs(m.K).max()
    assert np.allclose(m.Cc, D.T @ m.Mc, atol=1e-12 * sc)
    assert np.allclose(m.K, D.T @ m.Mc @ D, atol=1e-12 * sc)
    sp = m.sp
    N0, _ = sp.N(np.array([0.0]))
    N1, _ = sp.N(np.array([1.0]))
    M0, _ = sp.M(np.array([0.0]))
    M1, _ = sp.M(np.array([1.0]))
    bnd = np.outer(N1[:, 0], M1[:, 0]) - np.outer(N0[:, 0], M0[:, 0])
    assert np.allclose(m.C, bnd - m.Cc, atol=1e-12 * sc)
    assert np.allclose(m.K @ np.ones(n), 0.0, atol=1e-12 * sc)
    x, w = gauss_points(E, p, p + 4)
    Nv, _ = sp.N(x)
    assert np.allclose(m.M @ np.ones(n), Nv @ w, atol=1e-14)
    # symmetric / skew properties stated in Sec. 3.3
    assert np.allclose(m.M, m.M.T) and np.allclose(m.Mc, m.Mc.T)
    assert np.allclose(m.Tc, m.Tc.T)
    # interior rows of C are -C^ (integration by parts with vanishing ends)
    assert np.allclose(m.C_int, -m.Cc_int, atol=1e-12 * sc)


@pytest.mark.parametrize("E,p", CASES)
def test_quadrature_is_exact(E, p):
    """p+1 Gauss points integrate all products exactly: compare with 2p+3."""
    a = Matrices1D(E, p, 12.5)
    b = Matrices1D(E, p, 12.5, nquad=2 * p + 3)
    for name in ("M", "K", "C", "Mc", "Kc", "Cc", "Tc"):
        A, B = getattr(a, name), getattr(b, name)
        assert np.allclose(A, B, atol=1e-13 * np.abs(B).max()), name


@pytest.mark.parametrize("E,p", [(2, 2), (4, 3), (8, 4), (32, 3)])
def test_T_check_is_spd(E, p):
    """T^ must be positive definite (Sec. 3.3) for the chosen penalty."""
    m = Matrices1D(E, p, 12.5)
    assert np.linalg.eigvalsh(m.Tc).min() > 0
    assert np.linalg.eigvalsh(m.K_int).min() > 0
