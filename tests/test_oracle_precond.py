"""Pins of the oracle's preconditioners (Secs. 2, 4, 5.2, App. A.4).

* fast diagonalization (App. A.4) written with numpy's eigh reproduces the
  dense inverse of each diagonal block of A (the oracle's P_{V,0} uses LU);
* trace(P_{V,0}^{-1} A) = n_V;
* the spectrum at 2^3 elements, degree 4 (the paper's worked example);
* Lemma Sk_posdef / Corollary cor:Skform: sigma(P_k^{-1} A) is the image
  of sigma(P_0^{-1} A) under l_q(t) = 1 - (1 - t)^q, condition numbers
  decrease, every P_k is SPD (Theorem positive definite);
* the closed forms I - A P_{V,k}^{-1} = (I - A P_{V,0}^{-1})^{q^k} (and
  the same for eq. Pcq2 and one step of eq. Pcq1), by dense brute force;
* application counts and the cost ratios of Sec. 5.1.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sps

from oracle.assemble import KronSystem
from oracle.precond import BasePreconditioner, HyperPower, dense_hyperpower


def _read_golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        rows[parts[0]] = [float(v) for v in parts[1:]]
    return rows


def _dense_ops(S):
    A = S.A.toarray()
    o = S.offsets
    Dv = np.zeros_like(A)
    for c in range(3):
        Dv[o[c]:o[c + 1], o[c]:o[c + 1]] = A[o[c]:o[c + 1], o[c]:o[c + 1]]
    return A, Dv


@pytest.mark.parametrize("E,p", [(2, 2), (3, 3)])
def test_fast_diagonalization_equals_dense_inverse(E, p):
    """App. A.4: (U3 (x) U2 (x) U1) diag(1/(l1+l2+l3)) (U3 (x) U2 (x) U1)^T
    with U_k the M_k-orthonormal generalised eigenvectors of (A_k, M_k)."""
    nu = 0.7
    S = KronSystem(E, p, nu)
    m = S.m

    def geig(A, M):
        lam, U = sla.eigh(A, M)
        return lam, U

    lK, UK = geig(m.K_int, m.M_int)
    lT, UT = geig(m.Tc, m.Mc)
    fams = [((lK, UK), (lT, UT), (lT, UT)),    # component 1: K in dir 1
            ((lT, UT), (lK, UK), (lT, UT)),
            ((lT, UT), (lT, UT), (lK, UK))]
    A, _ = _dense_ops(S)
    o = S.offsets
    for c in range(3):
        (l1, U1), (l2, U2), (l3, U3) = fams[c]
        U = np.kron(U3, np.kron(U2, U1))
        lam = (l3[:, None, None] + l2[None, :, None] + l1[None, None, :]).reshape(-1)
        Pinv = U @ np.diag(1.0 / (2 * nu * lam)) @ U.T
        blk = A[o[c]:o[c + 1], o[c]:o[c + 1]]
        assert np.abs(Pinv @ blk - np.eye(blk.shape[0])).max() < 1e-10


@pytest.mark.parametrize("E,p,nu", [(2, 2, 0.7), (3, 3, 1.3), (2, 5, 1.0)])
def test_fast_diagonalisation_tier_equals_lu_and_dense_inverse(E, p, nu):
    """The oracle's einsum fast-diagonalisation tier (App. A.4) equals the
    sparse-LU P_{V,0} and the dense inverse of each diagonal block of A."""
    from oracle.precond import FastDiagBase
    S = KronSystem(E, p, nu)
    x = np.random.default_rng(E + p).standard_normal(S.N)
    lu = BasePreconditioner(S)
    fd = FastDiagBase(S)
    yv = fd.apply_V0(x[:S.nV])
    assert np.abs(yv - lu.apply_V0(x[:S.nV])).max() <= 1e-11 * np.abs(yv).max()
    o = S.offsets
    A, _ = _dense_ops(S)
    for c in range(3):
        blk = A[o[c]:o[c + 1], o[c]:o[c + 1]]
        ref = np.linalg.solve(blk, x[o[c]:o[c + 1]])
        assert np.abs(yv[o[c]:o[c + 1]] - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.array_equal(fd.apply_Q0(x[S.nV:]), lu.apply_Q0(x[S.nV:]))


def test_trace_of_preconditioned_A():
    S = KronSystem(3, 2, 1.0)
    A, Dv = _dense_ops(S)
    assert abs(np.trace(np.linalg.solve(Dv, A)) - S.nV) < 1e-9 * S.nV


def test_spectrum_worked_example():
    """2^3 elements, degree 4: sigma(P_{V,0}^{-1} A) within 0.02 of [0.71, 1.41]."""
    g = _read_golden("spectrum_2cube_p4.txt")
    S = KronSystem(2, 4, 1.0)
    A, Dv = _dense_ops(S)
    ev = sla.eigh(A, Dv, eigvals_only=True)
    assert abs(ev.min() - g["lambda0_min"][0]) < 0.02
    assert abs(ev.max() - g["lambda0_max"][0]) < 0.02
    assert ev.min() > 0 and ev.max() < 2


def test_lambda_min_sequence_from_the_paper():
    """Corollary cor:Skform applied to [0.71, 1.41] gives the printed sequence."""
    g = _read_golden("spectrum_2cube_p4.txt")
    l = lambda t: 2 * t - t * t
    lo, hi = g["lambda0_min"][0], g["lambda0_max"][0]
    seq = [lo]
    lo, hi = min(l(lo), l(hi)), max(l(lo), l(hi))
    seq.append(lo)
    for _ in range(2):
        lo = l(lo)
        seq.append(lo)
    assert np.allclose(seq, g["lambda_min_k"], atol=6e-5)


@pytest.mark.parametrize("q", [2, 3])
def test_spectral_map_and_spd(q):
    S = KronSystem(2, 3, 1.0)
    A, Dv = _dense_ops(S)
    X0 = np.linalg.inv(Dv)
    Xs = dense_hyperpower(A, X0, q, 3)
    ev0 = np.sort(np.linalg.eigvals(X0 @ A).real)
    lq = lambda t: 1 - (1 - t) ** q
    kappa = []
    for k, X in enumerate(Xs):
        evk = np.sort(np.linalg.eigvals(X @ A).real)
        pred = np.sort(ev0.copy())
        for _ in range(k):
            pred = lq(pred)
        assert np.allclose(evk, np.sort(pred), atol=1e-9)
        Xs_sym = 0.5 * (X + X.T)
        assert np.abs(X - X.T).max() < 1e-9 * np.abs(X).max()
        assert np.linalg.eigvalsh(Xs_sym).min() > 0
        kappa.append(evk.max() / evk.min())
        if k > 0:
            # (0, 1] for even q (Lemma Sk_posdef, q = 2); odd q keeps (0, 2)
            top = 1 + 1e-12 if q % 2 == 0 else 2.0
            assert evk.max() <= top and evk.min() > 0
    assert all(kappa[i + 1] < kappa[i] for i in range(len(kappa) - 1))


@pytest.mark.parametrize("q,k", [(2, 1), (2, 2), (3, 1), (3, 2)])
def test_operator_recursion_matches_closed_forms(q, k):
    """Literal recursion (operator form) vs dense closed forms (block-wise)."""
    S = KronSystem(2, 2, 1.3)
    A, Dv = _dense_ops(S)
    B = S.B.toarray()
    nV, nQ = S.nV, S.nQ
    P0 = BasePreconditioner(S)
    X0v = np.linalg.inv(Dv)
    X0q = np.column_stack([P0.apply_Q0(e) for e in np.eye(nQ)])
    # V block: I - A P_{V,k}^{-1} = (I - A P_{V,0}^{-1})^{q^k}
    for variant in ("Pcq1", "Pcq2"):
        H = HyperPower(S, q, k, variant=variant, base=P0)
        Xv = np.column_stack([H.apply_V(k, e) for e in np.eye(nV)])
        lhs = np.eye(nV) - A @ Xv
        rhs = np.linalg.matrix_power(np.eye(nV) - A @ X0v, q ** k)
        assert np.abs(lhs - rhs).max() < 1e-10
        Xq = np.column_stack([H.apply_Q(k, e) for e in np.eye(nQ)])
        if variant == "Pcq2":
            St = B.T @ X0v @ B
            rhs = np.linalg.matrix_power(np.eye(nQ) - St @ X0q, q ** k)
            assert np.abs((np.eye(nQ) - St @ Xq) - rhs).max() < 1e-10
        else:
            # one step of eq. Pcq1: I - S_l P_k = (I - S_l P_{k-1})^q
            Xprev = np.column_stack([H.apply_Q(k - 1, e) for e in np.eye(nQ)])
            lv = H.l_of(k)
            Xvl = np.column_stack([H.apply_V(lv, e) for e in np.eye(nV)])
            St = B.T @ Xvl @ B
            rhs = np.linalg.matrix_power(np.eye(nQ) - St @ Xprev, q)
            assert np.abs((np.eye(nQ) - St @ Xq) - rhs).max() < 1e-10
        assert np.abs(Xq - Xq.T).max() < 1e-10 * np.abs(Xq).max()
        assert np.linalg.eigvalsh(0.5 * (Xq + Xq.T)).min() > -1e-12


@pytest.mark.parametrize("q,k,l0", [(2, 1, 1), (2, 2, 2), (3, 1, 1)])
def test_fixed_level_and_exact_schur_closed_forms(q, k, l0):
    """Eq. Pcq2 with a fixed P_{V,l0} (option (2) of Sec. 4.1) and eq.
    Pcq_exact are plain hyper-power sequences on S~_{l0} and on
    S = B^T A^{-1} B: I - S P_k^{-1} = (I - S P_0^{-1})^{q^k}."""
    S = KronSystem(2, 2, 0.9)
    A, Dv = _dense_ops(S)
    B = S.B.toarray()
    nV, nQ = S.nV, S.nQ
    P0 = BasePreconditioner(S)
    X0q = np.column_stack([P0.apply_Q0(e) for e in np.eye(nQ)])
    Xv = np.linalg.inv(Dv)
    for _ in range(l0):                                      # dense eq. Pcv, order q
        Xv = dense_hyperpower(A, Xv, q, 1)[-1]
    for variant, Sd in (("Pcq2", B.T @ Xv @ B), ("Pcq_exact", B.T @ np.linalg.solve(A, B))):
        H = HyperPower(S, q, k, variant=variant, base=P0, fixed_level=l0)
        Xq = np.column_stack([H.apply_Q(k, e) for e in np.eye(nQ)])
        rhs = np.linalg.matrix_power(np.eye(nQ) - Sd @ X0q, q ** k)
        assert np.abs((np.eye(nQ) - Sd @ Xq) - rhs).max() < 1e-10, variant
        assert np.abs(Xq - Xq.T).max() < 1e-10 * np.abs(Xq).max()


@pytest.mark.parametrize("E,p,nu", [(3, 2, 0.8), (2, 3, 1.0)])
def test_schur_spectrum_in_unit_interval(E, p, nu):
    """sigma(P_{Q,0}^{-1} B^T A^{-1} B) lies in [0, 1] and reaches close to 1.

    For v with v.n = 0 on the flat faces of the cube, integration by parts
    gives 2 ||eps(v)||^2 = ||curl v||^2 + 2 ||div v||^2, so the weak form
    a(v, v) >= 2 nu ||div v||^2 (plus the Nitsche terms, positive at the
    penalty used), with near-equality for curl-free fields.  Hence
    (B^T A^{-1} B p, p) <= (2 nu)^{-1} (M_q p, p), i.e. the largest
    eigenvalue is at most 1 and close to it: this pins the factor 2 nu of
    P_{Q,0}^{-1} (a factor nu would put the top of the spectrum near 1/2)."""
    S = KronSystem(E, p, nu)
    A = S.A.toarray()
    B = S.B.toarray()
    Sch = B.T @ np.linalg.solve(A, B)
    P0 = BasePreconditioner(S)
    X0q = np.column_stack([P0.apply_Q0(e) for e in np.eye(S.nQ)])
    ev = np.sort(np.linalg.eigvals(X0q @ Sch).real)
    assert ev[0] > -1e-12 and abs(ev[0]) < 1e-10      # constant pressure
    assert ev[1] > 0.01 and ev[-1] <= 1 + 1e-12
    assert ev[-1] >= 0.9


@pytest.mark.parametrize("E,p,nu", [(2, 2, 0.7), (3, 3, 1.9), (1, 4, 1.0)])
def test_apply_Q0_equals_inverse_of_assembled_pressure_mass(E, p, nu):
    """apply_Q0 (three 1D LU solves along the tensor directions, with the
    axis swaps of the Fortran-ordered pressure tensor) equals
    2 nu inv(M^ (x) M^ (x) M^), the dense inverse of the 3D pressure mass
    matrix assembled as a Kronecker product (sparse kron, then dense solve).
    Closed form: the unit-integral M-splines have moments int M_i = 1, so
    the coefficients t of the constant function 1 solve M_q t = (1, ..., 1)
    and 1' M_q^{-1} 1 = int_Omega 1 = 1; hence 1' P_{Q,0}^{-1} 1 = 2 nu."""
    S = KronSystem(E, p, nu)
    m = S.m
    Mq = sps.kron(sps.kron(sps.csr_matrix(m.Mc), sps.csr_matrix(m.Mc)),
                  sps.csr_matrix(m.Mc)).toarray()
    n = S.nQ
    X = np.random.default_rng(E * 10 + p).standard_normal((n, 3))
    P0 = BasePreconditioner(S)
    got = np.column_stack([P0.apply_Q0(X[:, j]) for j in range(3)])
    ref = 2.0 * nu * np.linalg.solve(Mq, X)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    ones = np.ones(n)
    assert abs(ones @ P0.apply_Q0(ones) - 2.0 * nu) <= 1e-12 * 2.0 * nu


def test_damped_base_leaves_the_convergence_interval():
    """Sec. 2 (Lemma Sk_posdef, Remark rmk:convergence_Pk): the hyper-power
    sequence needs sigma(X_0 A~) in (0, 2).  The plain P_{V,0} satisfies it
    at 4^3, degree 3; damping it by w = 1.5 lifts the top of the spectrum
    above 2, the map t -> 1 - (1 - t)^2 then sends that end below 0, so
    P_1 is indefinite, and the oracle's MINRES with P_1 meets a negative
    r' P^{-1} r (the error path HP_ENOTSPD of the library)."""
    import scipy.linalg as sla
    from oracle.cases import cavity
    from oracle.krylov import minres
    S, b = cavity(4, 3)
    A = S.A.toarray()
    o = S.offsets
    Pv = np.zeros_like(A)
    for c in range(3):
        sl = slice(o[c], o[c + 1])
        Pv[sl, sl] = A[sl, sl]
    ev = sla.eigvalsh(A, Pv)
    assert 0.0 < ev[0] and ev[-1] < 2.0
    w = 1.5
    assert w * ev[-1] > 2.0
    assert 1.0 - (1.0 - w * ev[-1]) ** 2 < 0.0

    class Damped(BasePreconditioner):
        def apply_V0(self, x):
            return w * super().apply_V0(x)

        def apply_Q0(self, x):
            return w * super().apply_Q0(x)

    with pytest.raises(FloatingPointError):
        minres(lambda v: S.K @ v, HyperPower(S, 2, 1, base=Damped(S)).apply, b, tol=1e-8)
    # undamped, the same solve converges
    r = minres(lambda v: S.K @ v, HyperPower(S, 2, 1).apply, b, tol=1e-8)
    assert r.converged


# Appendix of base-operator counts per application of P_k^{-1}
COUNTS = {
    # (q, k): (V: PV0, A), Pcq1 literal: (PQ0, Bpairs, PV0, A), Pcq2: (PV0, Bpairs)
    (2, 0): ((1, 0), (1, 0, 0, 0), (0, 0)),
    (2, 1): ((2, 1), (2, 1, 1, 0), (1, 1)),
    (2, 2): ((4, 3), (4, 3, 6, 3), (3, 3)),
    (2, 3): ((8, 7), (8, 7, 20, 13), (7, 7)),
    (3, 1): ((3, 2), (3, 2, 2, 0), (2, 2)),
    (3, 2): ((9, 8), (9, 8, 24, 16), (8, 8)),
}


@pytest.mark.parametrize("qk", sorted(COUNTS))
def test_application_counts(qk):
    q, k = qk
    S = KronSystem(1, 2, 1.0)
    (v_p, v_a), (q_p, q_b, q_pv, q_a), (c2_pv, c2_b) = COUNTS[qk]
    P0 = BasePreconditioner(S)
    H = HyperPower(S, q, k, variant="Pcq1", base=P0)
    H.apply_V(k, np.ones(S.nV))
    assert (P0.counts["PV0"], P0.counts["A"]) == (v_p, v_a)
    for key in P0.counts:
        P0.counts[key] = 0
    H.apply_Q(k, np.ones(S.nQ))
    c = P0.counts
    assert (c["PQ0"], c["B"], c["Bt"], c["PV0"], c["A"]) == (q_p, q_b, q_b, q_pv, q_a)
    for key in P0.counts:
        P0.counts[key] = 0
    H2 = HyperPower(S, q, k, variant="Pcq2", base=P0)
    H2.apply_Q(k, np.ones(S.nQ))
    assert (c["PQ0"], c["PV0"], c["B"]) == (q ** k, c2_pv, c2_b)


def test_cost_model_ratios():
    g = _read_golden("cost_model.txt")
    cP, cA = g["c_P_numer"][0], g["c_A_numer"][0]
    C = lambda k: 2 ** k * cP + (2 ** k - 1) * cA
    assert C(1) / C(0) == pytest.approx(g["ratio_k1"][0])
    assert C(2) / C(0) == pytest.approx(g["ratio_k2"][0], abs=0.03)
    t0, t1, t2 = g["timing_384"]
    assert t1 / t0 == pytest.approx(C(1) / C(0), rel=0.01)
    assert t2 / t0 == pytest.approx(C(2) / C(0), rel=0.01)


@pytest.mark.parametrize("level,m", [(0, 3), (1, 6)])
def test_inner_pcg_matches_scipy_cg(level, m):
    """Options (3)/(4) of Sec. 4.1: the oracle's PCG iterate after m steps
    from zero equals scipy's preconditioned CG with the same P_{V,l}."""
    import scipy.sparse.linalg as spla
    S = KronSystem(3, 2, 0.7)
    H = HyperPower(S, 2, 0, variant="Pcq_pcg", fixed_level=level, pcg_iters=m)
    b = np.random.default_rng(3).standard_normal(S.nV)
    M = spla.LinearOperator((S.nV, S.nV), matvec=lambda r: H.apply_V(level, r))
    ref, _ = spla.cg(S.A, b, x0=np.zeros(S.nV), rtol=1e-300, atol=0.0, maxiter=m, M=M)
    got = H.pcg(b)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_inner_pcg_limits():
    """Run to convergence the inner PCG makes S_pcg the exact Schur
    complement (so the sequence is eq. Pcq_exact); with a tolerance it stops
    once the preconditioned residual has dropped by that factor."""
    S = KronSystem(2, 2, 1.0)
    P0 = BasePreconditioner(S)
    Hx = HyperPower(S, 2, 2, variant="Pcq_exact", base=P0)
    Hp = HyperPower(S, 2, 2, variant="Pcq_pcg", base=P0, pcg_iters=S.nV, pcg_tol=1e-14)
    x = np.random.default_rng(4).standard_normal(S.nQ)
    ref = Hx.apply_Q(2, x)
    assert np.abs(Hp.apply_Q(2, x) - ref).max() <= 1e-8 * np.abs(ref).max()
    Ht = HyperPower(S, 2, 1, variant="Pcq_pcg", base=P0, pcg_iters=100, pcg_tol=1e-3)
    b = np.random.default_rng(5).standard_normal(S.nV)
    y = Ht.pcg(b)
    r = b - S.A @ y
    z = P0.apply_V0(r)
    assert np.sqrt(r @ z) <= 1e-3 * np.sqrt(b @ P0.apply_V0(b)) * (1 + 1e-12)
