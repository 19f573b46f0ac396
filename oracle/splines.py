"""Univariate splines for the oracle (App. B.1 of the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The velocity and pressure spaces are built from two univariate families on
a uniform mesh of E elements of [0, 1] at maximum regularity:

* ``N_i = N_{i,p}``, i = 1..n with n = E + p: the B-splines of degree p,
  smoothness p-1, defined by the Cox--de Boor recursion on the open knot
  vector {0^(p+1), 1/E, ..., (E-1)/E, 1^(p+1)} (App. B.1);
* ``M_i = M_{i,p-1}``, i = 1..n-1: the degree p-1 B-splines on the same
  breakpoints (end multiplicity p), each divided by its integral so that it
  has unit integral (App. B.1, the normalisation after eq. ``reduction``).

Derivatives are obtained by differentiating the Cox--de Boor recursion
itself (product rule), not from the derivative identity eq. ``reduction``;
that identity is then a pin of this module (``tests/test_oracle_splines``).
"""
import numpy as np


def open_knots(E, p):
    """Open uniform knot vector of degree p on E elements of [0, 1]."""
    inner = [i / E for i in range(1, E)]
    return np.array([0.0] * (p + 1) + inner + [1.0] * (p + 1))


def _degree0(knots, x):
    """Indicator functions of the knot spans [t_i, t_{i+1}).

    The right end x == t_last is assigned to the last non-empty span so that
    the basis stays a partition of unity on the closed interval.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(knots) - 1
    N = np.zeros((m, x.size))
    for i in range(m):
        a, b = knots[i], knots[i + 1]
        if b > a:
            N[i] = (x >= a) & (x < b)
    last = max(i for i in range(m) if knots[i + 1] > knots[i])
    N[last, x == knots[-1]] = 1.0
    return N


def bspline_values_and_derivs(knots, p, x):
    """All B-splines of degree p on ``knots`` and their first derivatives.

    Returns (V, dV), each of shape (n, len(x)) with n = len(knots) - p - 1.
    Both follow the Cox--de Boor recursion
        N_{i,d} = (x - t_i)/(t_{i+d} - t_i) N_{i,d-1}
                + (t_{i+d+1} - x)/(t_{i+d+1} - t_{i+1}) N_{i+1,d-1},
    with 0/0 := 0, and its derivative by the product rule.
    """
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    t = knots
    N = _degree0(t, x)
    dN = np.zeros_like(N)
    for d in range(1, p + 1):
        m = len(t) - d - 1
        Nn = np.zeros((m, x.size))
        dNn = np.zeros((m, x.size))
        for i in range(m):
            den1 = t[i + d] - t[i]
            den2 = t[i + d + 1] - t[i + 1]
            if den1 > 0:
                Nn[i] += (x - t[i]) / den1 * N[i]
                dNn[i] += N[i] / den1 + (x - t[i]) / den1 * dN[i]
            if den2 > 0:
                Nn[i] += (t[i + d + 1] - x) / den2 * N[i + 1]
                dNn[i] += -N[i + 1] / den2 + (t[i + d + 1] - x) / den2 * dN[i + 1]
        N, dN = Nn, dNn
    return N, dN


class SplinePair:
    """The pair (N_{i,p}, M_{i,p-1}) on E uniform elements (App. B.1)."""

    def __init__(self, E, p):
        if p < 2:
            raise ValueError("the velocity degree must be at least 2")
        self.E, self.p = E, p
        self.kn = open_knots(E, p)
        self.km = self.kn[1:-1]
        self.n = E + p
        # integrals of the unnormalised degree p-1 B-splines, by Gauss
        # quadrature (exact for polynomials of degree <= 2p-1 per element)
        xg, wg = gauss_points(E, p)
        V, _ = bspline_values_and_derivs(self.km, p - 1, xg)
        self.m_integrals = V @ wg

    def N(self, x):
        """(values, derivatives) of N_1..N_n at x."""
        return bspline_values_and_derivs(self.kn, self.p, x)

    def M(self, x):
        """(values, derivatives) of the unit-integral M_1..M_{n-1} at x."""
        V, dV = bspline_values_and_derivs(self.km, self.p - 1, x)
        s = 1.0 / self.m_integrals[:, None]
        return V * s, dV * s


def gauss_points(E, p, npts=None):
    """Element-wise Gauss--Legendre points and weights on [0, 1].

    ``npts`` defaults to p+1 points per element, which integrates every
    product of two basis functions of degree <= p exactly.
    """
    q = p + 1 if npts is None else npts
    g, w = np.polynomial.legendre.leggauss(q)
    xs, ws = [], []
    for e in range(E):
        a, b = e / E, (e + 1) / E
        xs.append(0.5 * (b - a) * g + 0.5 * (a + b))
        ws.append(0.5 * (b - a) * w)
    return np.concatenate(xs), np.concatenate(ws)
