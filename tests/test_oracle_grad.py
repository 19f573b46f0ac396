"""Pins of the oracle's adjoint gradient of L = ||u_h - u_t||^2 (cavity).

* L is quadratic in beta, so a central difference is exact up to rounding;
* u_h = U u_lid + u_beta / nu exactly (A and the lid data scale with nu, the
  body-force load does not), so with zero body force dL/dnu = 0, and in
  general dL/dnu = <dL/du, -u_beta / nu^2> in closed form.
"""
import numpy as np

from oracle.cases import CavityLoss, cavity, velocity_mass
from oracle.direct import DirectSolver


def _setup(E=3, p=2):
    S, b = cavity(E, p, U=1.5)
    ut = DirectSolver(S).solve(b)[:S.nV]
    return S, ut


def test_beta_gradient_central_difference_is_exact():
    S, ut = _setup()
    loss = CavityLoss(3, 2, U=1.0, u_target=ut)
    rng = np.random.default_rng(11)
    beta = 0.3 * rng.standard_normal(S.nV)
    L, gb, gn = loss.gradient(beta, 1.0)
    for _ in range(3):
        d = rng.standard_normal(S.nV)
        h = 1e-3
        fd = (loss.value(beta + h * d, 1.0) - loss.value(beta - h * d, 1.0)) / (2 * h)
        assert abs(fd - gb @ d) <= 1e-8 * max(1.0, abs(fd))


def test_nu_gradient_zero_without_body_force():
    S, ut = _setup()
    loss = CavityLoss(3, 2, U=1.0, u_target=ut)
    L, gb, gn = loss.gradient(np.zeros(S.nV), 0.8)
    assert abs(gn) <= 1e-10 * max(L, 1.0)


def test_nu_gradient_closed_form_and_difference():
    S, ut = _setup()
    loss = CavityLoss(3, 2, U=1.0, u_target=ut)
    rng = np.random.default_rng(12)
    beta = 0.5 * rng.standard_normal(S.nV)
    nu = 1.3
    L, gb, gn = loss.gradient(beta, nu)
    # closed form: u = u_lid + u_beta(nu=1) / nu
    S1, b1 = cavity(3, 2, nu=1.0, U=0.0)
    MV = velocity_mass(S1)
    fb = np.zeros(S1.N)
    fb[:S1.nV] = MV @ beta
    ub = DirectSolver(S1).solve(fb)[:S1.nV]
    _, _, _, x = loss.solve(beta, nu)
    d = x[:S.nV] - ut
    closed = (2 * MV @ d) @ (-ub / nu ** 2)
    assert abs(gn - closed) <= 1e-9 * abs(closed)
    h = 1e-4
    fd = (loss.value(beta, nu + h) - loss.value(beta, nu - h)) / (2 * h)
    assert abs(fd - gn) <= 1e-6 * abs(gn)
