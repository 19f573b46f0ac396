"""Pins of the oracle's Lanczos spectrum estimates (Secs. 2 and 5.2).

* Run to the dimension of the block, the Lanczos extremes of the pencils
  (A, P_{V,0}) and (S~_0, P_{Q,0}) equal those of the dense generalised
  eigenproblems (brute force; for S~_0 the smallest non-zero eigenvalue,
  the constant pressure being its null vector);
* at 2^3 elements, degree 4, a few dozen steps reproduce the extremes the
  paper prints for P_{V,0}^{-1} A (0.71 and 1.41, within 0.02);
* the hyper-power interval map gives the paper's lambda_min sequence and
  the extremes of the dense spectra of P_{V,k}^{-1} A for q = 2, 3.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.assemble import KronSystem
from oracle.precond import BasePreconditioner, dense_hyperpower
from oracle.spectra import (dense_sequence_spectrum, hyperpower_interval, lanczos,
                            pressure_null_vector, ritz_extremes,
                            schur_block_extremes, velocity_block_extremes)


def _golden():
    path = os.path.join(os.path.dirname(__file__), "golden", "spectrum_2cube_p4.txt")
    rows = {}
    for line in open(path):
        parts = line.split()
        if parts and not parts[0].startswith("#"):
            rows[parts[0]] = [float(v) for v in parts[1:]]
    return rows


def _dense(S):
    A = S.A.toarray()
    o = S.offsets
    Dv = np.zeros_like(A)
    for c in range(3):
        Dv[o[c]:o[c + 1], o[c]:o[c + 1]] = A[o[c]:o[c + 1], o[c]:o[c + 1]]
    return A, Dv


@pytest.mark.parametrize("E,p,nu", [(2, 2, 1.0), (3, 2, 0.4)])
def test_velocity_lanczos_full_run_equals_dense(E, p, nu):
    S = KronSystem(E, p, nu)
    pre = BasePreconditioner(S)
    A, Dv = _dense(S)
    ev = sla.eigh(A, Dv, eigvals_only=True)
    lo, hi = velocity_block_extremes(pre, S.nV, seed=E)
    assert abs(lo - ev[0]) < 1e-8 and abs(hi - ev[-1]) < 1e-8


@pytest.mark.parametrize("E,p,nu", [(2, 2, 1.0), (3, 2, 2.5)])
def test_schur_lanczos_full_run_equals_dense(E, p, nu):
    S = KronSystem(E, p, nu)
    pre = BasePreconditioner(S)
    A, Dv = _dense(S)
    B = S.B.toarray()
    St = B.T @ np.linalg.solve(Dv, B)
    PQinv = np.column_stack([pre.apply_Q0(e) for e in np.eye(S.nQ)])
    PQ = np.linalg.inv(PQinv)
    ev = sla.eigh(St, 0.5 * (PQ + PQ.T), eigvals_only=True)
    assert abs(ev[0]) < 1e-10 * ev[-1]            # the constant-pressure mode
    assert ev[1] > 1e-6 * ev[-1]                  # ... and only that one
    lo, hi = schur_block_extremes(pre, S.nQ, seed=E)
    assert abs(lo - ev[1]) < 1e-8 and abs(hi - ev[-1]) < 1e-8


def test_velocity_lanczos_reproduces_the_worked_example():
    g = _golden()
    S = KronSystem(2, 4, 1.0)
    lo, hi = velocity_block_extremes(BasePreconditioner(S), 60, seed=1)
    assert abs(lo - g["lambda0_min"][0]) < 0.02
    assert abs(hi - g["lambda0_max"][0]) < 0.02


def test_interval_map_gives_the_printed_sequence():
    g = _golden()
    lo, hi = g["lambda0_min"][0], g["lambda0_max"][0]
    seq = [hyperpower_interval(lo, hi, 2, k)[0] for k in range(4)]
    assert np.allclose(seq, g["lambda_min_k"], atol=6e-5)
    assert hyperpower_interval(lo, hi, 2, 1)[1] == 1.0


@pytest.mark.parametrize("q", [2, 3])
def test_interval_map_matches_dense_spectra(q):
    S = KronSystem(2, 3, 1.0)
    A, Dv = _dense(S)
    ev0 = sla.eigh(A, Dv, eigvals_only=True)
    for k, X in enumerate(dense_hyperpower(A, np.linalg.inv(Dv), q, 3)):
        evk = np.sort(np.linalg.eigvals(X @ A).real)
        lo, hi = hyperpower_interval(ev0[0], ev0[-1], q, k)
        assert abs(lo - evk[0]) < 1e-9 and abs(hi - evk[-1]) < 1e-9 + (1e-9 if k else 0)


def test_lanczos_tridiagonal_of_a_diagonal_pencil():
    """Diagonal M and P: the Ritz values after n steps are the ratios."""
    rng = np.random.default_rng(0)
    m = rng.uniform(1, 5, 30)
    d = rng.uniform(0.5, 2, 30)
    al, be = lanczos(lambda v: m * v, lambda r: r / d, rng.standard_normal(30), 30)
    lo, hi = ritz_extremes(al, be)
    assert abs(lo - (m / d).min()) < 1e-10 and abs(hi - (m / d).max()) < 1e-10


@pytest.mark.parametrize("E,p", [(3, 2), (4, 3)])
def test_pressure_null_vector_is_the_constant_pressure(E, p):
    """B n = 0, and n is the only null direction of B (its other singular
    values are bounded away from zero)."""
    S = KronSystem(E, p, 1.0)
    n = pressure_null_vector(S)
    B = S.B.toarray()
    assert np.abs(B @ n).max() < 1e-12 * np.abs(B).max()
    sv = np.linalg.svd(B, compute_uv=False)
    assert sv[-2] > 1e-3 * sv[0]


def test_schur_sequences_at_the_worked_example():
    """2^3 elements, degree 4 (the spectra of Sec. 5.2), the preconditioned
    Schur complement P_{Q,k}^{-1} B^T A^{-1} B for the three sequences:
    * eq. Pcq_exact is a hyper-power sequence on S itself, so its spectrum
      is the image of the k = 0 spectrum under t -> 2t - t^2 (Corollary
      cor:Skform), inside (0, 1] for k >= 1;
    * with inner updates (eq. Pcq1) the spectra are close to those of
      Pcq_exact (within 10 % in the condition number) and decrease with k;
    * without inner updates (eq. Pcq2) the sequence converges to
      S~_0^{-1}, so the condition number tends to that of (S, S~_0), and
      only its first three updates lower it (as the paper observes)."""
    from oracle.precond import HyperPower
    S = KronSystem(2, 4, 1.0)
    P0 = BasePreconditioner(S)
    ev = {}
    for var in ("Pcq_exact", "Pcq1", "Pcq2"):
        H = HyperPower(S, 2, 0, variant=var, base=P0)
        ev[var] = [dense_sequence_spectrum(H, "Q", k) for k in range(7 if var == "Pcq2" else 5)]
    e0 = ev["Pcq_exact"][0]
    assert e0[0] > 0 and e0[-1] <= 1 + 1e-12
    for k in range(1, 5):
        pred = np.sort(e0.copy())
        for _ in range(k):
            pred = 2 * pred - pred * pred
        assert np.allclose(ev["Pcq_exact"][k], np.sort(pred), atol=1e-9)
    kap = {v: [e[-1] / e[0] for e in ev[v]] for v in ev}
    for k in range(1, 4):
        assert kap["Pcq1"][k] < kap["Pcq1"][k - 1]
        assert abs(kap["Pcq1"][k] / kap["Pcq_exact"][k] - 1) < 0.10
    # limit of eq. Pcq2: the pencil (S, S~_0)
    A = S.A.toarray()
    B = S.B.toarray()
    o = S.offsets
    Dv = np.zeros_like(A)
    for c in range(3):
        Dv[o[c]:o[c + 1], o[c]:o[c + 1]] = A[o[c]:o[c + 1], o[c]:o[c + 1]]
    St0 = B.T @ np.linalg.solve(Dv, B)
    Sx = B.T @ np.linalg.solve(A, B)
    lim = np.sort(np.linalg.eigvals(np.linalg.pinv(St0) @ Sx).real)[1:]
    assert abs(kap["Pcq2"][6] / (lim[-1] / lim[0]) - 1) < 1e-3
    # only the first three updates of eq. Pcq2 lower the condition number
    assert kap["Pcq2"][3] < kap["Pcq2"][2] < kap["Pcq2"][1] < kap["Pcq2"][0]
    assert kap["Pcq2"][4] > kap["Pcq2"][3]


@pytest.mark.parametrize("var,k,s_level", [("Pcq1", 1, None), ("Pcq1", 2, 1), ("Pcq2", 2, None)])
def test_schur_lanczos_with_updates_equals_dense(var, k, s_level):
    from oracle.precond import HyperPower
    from oracle.spectra import schur_lanczos
    S = KronSystem(2, 2, 0.8)
    H = HyperPower(S, 2, 0, variant=var, fixed_level=1)
    ev = dense_sequence_spectrum(H, "Q", k, s_level)
    x0 = np.random.default_rng(4).standard_normal(S.nQ)
    lo, hi = ritz_extremes(*schur_lanczos(H, k, s_level, x0, S.nQ))
    assert abs(lo - ev[0]) < 1e-8 * ev[-1] and abs(hi - ev[-1]) < 1e-8 * ev[-1]
