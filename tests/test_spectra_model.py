"""Host-side model of the a-priori depth choice (paper_2311_06926_amd.spectra)
checked on the CPU against the oracle:

* the interval map equals the paper's lambda_min sequence from [0.71, 1.41]
  (Corollary cor:Skform) and, for q = 3, the dense spectra;
* the saddle-point inclusion contains every non-zero eigenvalue of the
  block-diagonally preconditioned K (dense, tiny mesh, with P_{V,k} and the
  exact-Schur sequence P_{Q,k} of eq. Pcq_exact), and touches its extremes
  within a factor of 2;
* the MINRES bound is not below the oracle MINRES iteration count.
"""
import numpy as np
import pytest

from oracle.assemble import KronSystem
from oracle.precond import BasePreconditioner, HyperPower
from oracle.spectra import dense_sequence_spectrum
from paper_2311_06926_amd import spectra as model


def test_map_reproduces_the_printed_sequence():
    seq = [model.hyperpower_interval(0.71, 1.41, 2, k)[0] for k in range(4)]
    assert np.allclose(seq, [0.71, 0.8319, 0.9717, 0.9992], atol=6e-5)


def test_map_matches_dense_spectra_for_q3():
    S = KronSystem(2, 3, 1.0)
    H = HyperPower(S, 3, 0)
    e0 = dense_sequence_spectrum(H, "V", 0)
    for k in (1, 2):
        ek = dense_sequence_spectrum(H, "V", k)
        lo, hi = model.hyperpower_interval(e0[0], e0[-1], 3, k)
        assert abs(lo - ek[0]) < 1e-9 and abs(hi - ek[-1]) < 1e-9


@pytest.mark.parametrize("k", [0, 1, 2])
def test_inclusion_and_minres_bound(k):
    from oracle.krylov import minres
    S = KronSystem(3, 2, 1.0)
    P0 = BasePreconditioner(S)
    H = HyperPower(S, 2, k, variant="Pcq_exact", base=P0)
    ev_v = dense_sequence_spectrum(H, "V", k)
    ev_s = dense_sequence_spectrum(H, "Q", k)
    neg, pos = model.saddle_intervals((ev_v[0], ev_v[-1]), (ev_s[0], ev_s[-1]))
    X = np.column_stack([H.apply(e) for e in np.eye(S.N)])
    lam = np.linalg.eigvals(X @ S.K.toarray()).real
    lam = lam[np.abs(lam) > 1e-9]                     # the constant-pressure zero
    ln, lp = -lam[lam < 0], lam[lam > 0]
    tol = 1e-10
    assert ln.max() <= neg[0] * (1 + tol) and ln.min() >= neg[1] * (1 - tol)
    assert lp.min() >= pos[0] * (1 - tol) and lp.max() <= pos[1] * (1 + tol)
    assert ln.max() > neg[0] / 2 and lp.max() > pos[1] / 2
    b = S.lid_rhs(1.0)
    ref = minres(lambda v: S.K @ v, H.apply, b, tol=1e-8)
    assert model.minres_bound(neg, pos, 1e-8) >= ref.iters


def test_schur_level_and_choice():
    assert model.schur_level_for((0.71, 1.41), 2) == 5        # 0.41^32 < 1e-8
    pred = {"k": [{"k": 0, "minres_bound": 100}, {"k": 1, "minres_bound": 50},
                  {"k": 2, "minres_bound": 40}]}
    assert model.choose_iters(pred, {0: 1.0, 1: 1.5, 2: 3.0}) == 1
    assert model.choose_iters(pred, {0: 1.0, 1: 2.5, 2: 3.0}) == 0
