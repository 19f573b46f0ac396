"""Extreme eigenvalues of the preconditioned blocks by Lanczos, and the
spectral map of the hyper-power sequence (Sec. 2, Lemma on the spectrum of
P_k and its Corollary; Sec. 4 and the spectra of Sec. 5).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The preconditioned blocks are the pencils (A, P_{V,0}) and
(S~_0, P_{Q,0}) with S~_0 = B^T P_{V,0}^{-1} B; both are symmetric with an
SPD second matrix, so their eigenvalues are those of the symmetric
tridiagonal matrix that the Lanczos process builds in the inner product of
the second matrix.  With a start residual r_0:

    z_j = P^{-1} r_j,  beta_j = sqrt(r_j . z_j),  v_j = z_j / beta_j,
    u = M v_j,  alpha_j = v_j . u,
    r_{j+1} = u - alpha_j P v_j - beta_j P v_{j-1},   P v_j = r_j / beta_j,

T = tridiag(beta; alpha; beta) (beta_j couples v_{j-1} and v_j); no reorthogonalisation (the
extreme Ritz values converge first and are all that is used); the process
stops early when beta falls to rounding level against the alphas (an
invariant subspace).  S~_0 has the
constant-pressure null vector (B q_c = 0); a start residual in the range of
S~_0 (r_0 = S~_0 x, and every later residual projected onto that range)
keeps the process in its complement, so the smallest Ritz value estimates
the smallest non-zero eigenvalue.

The hyper-power map of one update of order q on the spectrum of the
preconditioned operator is t -> 1 - (1 - t)^q (the eigenvalues of
I - A X_{k+1} are the q-th powers of those of I - A X_k), applied k times.
"""
import numpy as np
import scipy.linalg as sla


def lanczos(apply_M, apply_Pinv, r0, steps, project=None):
    """Tridiagonal coefficients (alpha, beta) of ``steps`` Lanczos steps for
    the pencil (M, P) from residual r0; beta[j] couples steps j and j+1.
    ``project`` (optional) is applied to every residual before P^{-1}."""
    alpha, beta = [], []
    project = project or (lambda r: r)
    r = project(np.array(r0, dtype=np.float64))
    z = apply_Pinv(r)
    b = np.sqrt(r @ z)
    rs_prev = np.zeros_like(r)          # P v_{j-1}
    for _ in range(steps):
        v = z / b
        rs = r / b                      # = P v
        u = apply_M(v)
        a = v @ u
        alpha.append(a)
        r_new = project(u - a * rs - b * rs_prev)
        z_new = apply_Pinv(r_new)
        b_new = np.sqrt(max(r_new @ z_new, 0.0))
        beta.append(b_new)
        if b_new <= 1e-10 * max(abs(x) for x in alpha):
            break                       # invariant subspace reached
        rs_prev = rs
        r, z, b = r_new, z_new, b_new
    return np.array(alpha), np.array(beta[: len(alpha) - 1])


def ritz_extremes(alpha, beta):
    """Smallest and largest eigenvalue of tridiag(beta; alpha; beta)."""
    w = sla.eigh_tridiagonal(alpha, beta, eigvals_only=True)
    return float(w[0]), float(w[-1])


def velocity_lanczos(H, k, r0, steps):
    """Lanczos coefficients of the pencil (A, P_{V,k}) (``H``: a HyperPower,
    whose order q is used), from residual r0."""
    return lanczos(H.P0.A, lambda r: H.apply_V(k, r), r0, steps)


def pressure_null_vector(sysm):
    """The null vector of B (constant pressure): n1 (x) n1 (x) n1 with n1
    spanning the null space of the 1D divergence coupling C^ (B_c is a
    Kronecker product with C^ in direction c), unit Euclidean norm."""
    n1 = sla.null_space(np.asarray(sysm.m.Cc_int))
    assert n1.shape[1] == 1
    n = np.kron(n1[:, 0], np.kron(n1[:, 0], n1[:, 0]))
    return n / np.linalg.norm(n)


def schur_lanczos(H, k, s_level, x0, steps):
    """Lanczos coefficients of the pencil (S~_l, P_{Q,k}), S~_l =
    B^T P_{V,l}^{-1} B with l = s_level (``s_level=None``: the exact
    S = B^T A^{-1} B of eq. Pcq_exact), P_{Q,k} per H's variant, from the
    residual r_0 = S~_l x0.  Every residual is projected Euclidean-
    orthogonally to the null vector n of S~_l (onto the range of S~_l),
    which keeps rounding from bringing the zero eigenvalue into the Ritz
    values."""
    n = pressure_null_vector(H.s)
    if s_level is None:
        S = H.S_exact
    else:
        def S(x):
            return H.S_tilde(s_level, x)

    def project(r):
        return r - n * (n @ r)

    return lanczos(S, lambda r: H.apply_Q(k, r), S(x0), steps, project)


def velocity_block_extremes(pre, steps, seed=0):
    """Ritz extremes of P_{V,0}^{-1} A (``pre``: a BasePreconditioner)."""
    from .precond import HyperPower
    r0 = np.random.default_rng(seed).standard_normal(pre.s.nV)
    return ritz_extremes(*velocity_lanczos(HyperPower(pre.s, 2, 0, base=pre), 0, r0, steps))


def schur_block_extremes(pre, steps, seed=0):
    """Ritz extremes (non-zero part) of P_{Q,0}^{-1} S~_0,
    S~_0 = B^T P_{V,0}^{-1} B."""
    from .precond import HyperPower
    x0 = np.random.default_rng(seed).standard_normal(pre.s.nQ)
    return ritz_extremes(*schur_lanczos(HyperPower(pre.s, 2, 0, base=pre), 0, 0, x0, steps))


def dense_sequence_spectrum(H, block, k, s_level=None):
    """All eigenvalues (ascending) of P_{V,k}^{-1} A (block 'V') or of
    P_{Q,k}^{-1} S~_l (block 'Q'; l = s_level, None for the exact Schur
    complement; the zero of the constant pressure removed), from the
    preconditioners' columns; tiny sizes only (the spectra of Sec. 5.2)."""
    s = H.s
    if block == "V":
        X = np.column_stack([H.apply_V(k, e) for e in np.eye(s.nV)])
        M = s.A.toarray()
    else:
        X = np.column_stack([H.apply_Q(k, e) for e in np.eye(s.nQ)])
        M = np.column_stack([H.S_exact(e) if s_level is None else H.S_tilde(s_level, e)
                             for e in np.eye(s.nQ)])
    ev = np.sort(np.linalg.eigvals(X @ M).real)
    if block == "Q":
        ev = ev[1:]                       # the constant-pressure zero
    return ev


def hyperpower_interval(lmin, lmax, q, k):
    """Image of [lmin, lmax] under k applications of t -> 1 - (1 - t)^q
    (for an interval inside (0, 2)): the extremes of the image are attained
    at the interval ends or, for even q, at t = 1 (value 1)."""
    ts = np.array([lmin, lmax] + ([1.0] if lmin < 1.0 < lmax else []))
    for _ in range(k):
        ts = 1.0 - (1.0 - ts) ** q
    return float(ts.min()), float(ts.max())
