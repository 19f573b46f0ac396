"""Base preconditioner and hyper-power sequences (Secs. 2 and 4 of the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* P0 (eq. ``blockdiagprecond`` with the blocks of Sec. 4): P_{V,0} is the
  block diagonal of A (its three diagonal blocks, which the paper inverts by
  fast diagonalization); here each block is inverted by sparse LU, never by
  fast diagonalization.  P_{Q,0} is the pressure mass matrix
  M^ (x) M^ (x) M^ divided by the viscosity coefficient of the printed
  (nu-free) Kronecker sums of A.  The weak form a = int 2 nu grad^s:grad^s
  makes that coefficient 2 nu, so P_{Q,0}^{-1} = 2 nu (M^^{-1})^{(x)3}.
  With it sigma(P_{Q,0}^{-1} B^T A^{-1} B) lies in (0, 1] (because
  a(v, v) >= 2 nu ||div v||^2), and MINRES counts match Table 1; with
  nu^{-1} M^^{(x)3} against this A the spectrum would lie in (0, 1/2].
  Its inverse is applied as three 1D LU solves along the three directions.
* Hyper-power of order q (eq. ``hyperpower2`` for q = 2; higher orders as
  X_{k+1} = X_k sum_{i<q} (I - A~ X_k)^i, of which q = 2 is
  2 X_k - X_k A~ X_k, eq. ``hyperpowersequence``).  The recursion is taken
  literally: applying X_k applies X_{k-1} q times.
* V block: eq. ``Pcv`` with the exact A.
* Q block with inner updates: eq. ``Pcq1``, S~_l = B^T P_{V,l}^{-1} B at the
  k-th update, with l = 0 for k = 1 and l = k for k > 1 (the schedule of
  option (5) in Sec. 4.1); ``schedule='prev'`` uses l = k - 1 instead.
* Q block without inner updates: eq. ``Pcq2`` with P_V = P_{V,0} (option
  (1) of Sec. 4.1); ``fixed_level=l`` takes the fixed P_{V,l} instead
  (option (2)).
* Q block with the exact Schur complement: eq. ``Pcq_exact``,
  S = B^T A^{-1} B with A^{-1} applied by sparse LU (``variant='Pcq_exact'``).
* ``FastDiagBase``: the same P_0 with the velocity blocks by fast
  diagonalisation (App. A.4, numpy einsum), the CPU timing tier at meshes
  where the sparse LU is too slow to factor; pinned against the LU form.
* Q block with an inner iterative solve (options (3) and (4) of Sec. 4.1):
  the sequence of eq. ``Pcq2`` on S_pcg = B^T PCG(A, P_{V,l}) B, where
  PCG(A, P) b is the preconditioned conjugate gradient iterate for A y = b
  from y = 0 after at most ``pcg_iters`` steps, stopped early once
  sqrt(r.z) <= pcg_tol sqrt(r_0.z_0) (``variant='Pcq_pcg'``, l =
  ``fixed_level``: 0 for option (3), > 0 for option (4)).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla


class BasePreconditioner:
    """P_0^{-1} = diag(P_{V,0}^{-1}, P_{Q,0}^{-1}) of Sec. 4."""

    def __init__(self, sysm):
        self.s = sysm
        off = sysm.offsets
        self.off = off
        blocks = [sysm.A11, sysm.A22, sysm.A33]
        self.lu = [spla.splu(b.tocsc()) for b in blocks]
        self.Mc_lu = sla.lu_factor(sysm.m.Mc)
        self.nM = sysm.m.nM
        self.counts = {"PV0": 0, "PQ0": 0, "A": 0, "B": 0, "Bt": 0}

    def apply_V0(self, x):
        """P_{V,0}^{-1} x for a velocity vector x (n_V)."""
        self.counts["PV0"] += 1
        y = np.empty_like(x)
        for c in range(3):
            sl = slice(self.off[c], self.off[c + 1])
            y[sl] = self.lu[c].solve(x[sl])
        return y

    def apply_Q0(self, x):
        """P_{Q,0}^{-1} x = 2 nu (M^^{-1} (x) M^^{-1} (x) M^^{-1}) x (n_Q)."""
        self.counts["PQ0"] += 1
        n = self.nM
        X = x.reshape(n, n, n)          # [i3, i2, i1]
        X = sla.lu_solve(self.Mc_lu, X.reshape(n * n, n).T).T.reshape(n, n, n)   # dir 1
        X = np.swapaxes(X, 1, 2)        # [i3, i1, i2]
        X = sla.lu_solve(self.Mc_lu, X.reshape(n * n, n).T).T.reshape(n, n, n)   # dir 2
        X = np.swapaxes(X, 1, 2)
        X = X.reshape(n, n * n)         # [i3, (i2, i1)]
        X = sla.lu_solve(self.Mc_lu, X)                                           # dir 3
        return 2.0 * self.s.nu * X.reshape(-1)

    def apply(self, x):
        nV = self.s.nV
        return np.concatenate([self.apply_V0(x[:nV]), self.apply_Q0(x[nV:])])

    # operators counted for the cost bookkeeping of Sec. 4.2
    def A(self, u):
        self.counts["A"] += 1
        return self.s.A @ u

    def B(self, p):
        self.counts["B"] += 1
        return self.s.B @ p

    def Bt(self, u):
        self.counts["Bt"] += 1
        return self.s.B.T @ u


class FastDiagBase(BasePreconditioner):
    """P_0^{-1} with each velocity block applied by fast diagonalisation
    (App. A.4), written with numpy: the block A_cc is the generalised
    Kronecker sum of (K_int, M_int) in direction c and (T^, M^) in the two
    others (Sec. 3.3), so with the generalised eigenpairs U^T M U = I,
    U^T K U = diag(lambda) of each pencil (scipy ``eigh``),

        A_cc^{-1} = (U3 (x) U2 (x) U1) diag(1 / (2 nu (l1 + l2 + l3))) (U3 (x) U2 (x) U1)^T.

    The three mode products each way are plain ``einsum`` contractions.  This
    is the CPU reference tier used to time the oracle at meshes where the
    sparse LU of ``BasePreconditioner`` takes minutes to factor; it is pinned
    against that LU form and against the dense inverse.  P_{Q,0} is the
    parent's (three 1D LU solves)."""

    def __init__(self, sysm):
        self.s = sysm
        self.off = sysm.offsets
        m = sysm.m
        self.Mc_lu = sla.lu_factor(m.Mc)
        self.nM = m.nM
        self.counts = {"PV0": 0, "PQ0": 0, "A": 0, "B": 0, "Bt": 0}
        lK, UK = sla.eigh(m.K_int, m.M_int)
        lT, UT = sla.eigh(m.Tc, m.Mc)
        # (l, U) per direction 1, 2, 3 for each component c: K in direction c
        self.fams = []
        for c in range(3):
            self.fams.append([(lK, UK) if d == c else (lT, UT) for d in range(3)])

    def apply_V0(self, x):
        """P_{V,0}^{-1} x by fast diagonalisation of each diagonal block."""
        self.counts["PV0"] += 1
        y = np.empty_like(x)
        nu = self.s.nu
        for c in range(3):
            (l1, U1), (l2, U2), (l3, U3) = self.fams[c]
            sl = slice(self.off[c], self.off[c + 1])
            X = x[sl].reshape(len(l3), len(l2), len(l1))        # [i3, i2, i1]
            X = np.einsum("ia,kji->kja", U1, X)                  # U1^T along direction 1
            X = np.einsum("jb,kja->kba", U2, X)                  # U2^T along direction 2
            X = np.einsum("kc,kba->cba", U3, X)                  # U3^T along direction 3
            X = X / (2.0 * nu * (l3[:, None, None] + l2[None, :, None] + l1[None, None, :]))
            X = np.einsum("kc,cba->kba", U3, X)                  # back: U3
            X = np.einsum("jb,kba->kja", U2, X)
            X = np.einsum("ia,kja->kji", U1, X)
            y[sl] = X.reshape(-1)
        return y


def hyperpower_apply(X_prev, Aop, q, x):
    """One hyper-power level applied to x:  X_prev sum_{i<q} (I - A~ X_prev)^i x.

    For q = 2 this is (2 X_prev - X_prev A~ X_prev) x (eq. ``hyperpowersequence``).
    """
    z = x
    s = x.copy()
    for _ in range(q - 1):
        z = z - Aop(X_prev(z))
        s = s + z
    return X_prev(s)


class HyperPower:
    """P_k^{-1} = diag(P_{V,k}^{-1}, P_{Q,k}^{-1}) for order q and k updates."""

    def __init__(self, sysm, q=2, k=1, variant="Pcq1", schedule="literal", base=None,
                 fixed_level=0, pcg_iters=5, pcg_tol=0.0):
        if q < 2 or k < 0 or fixed_level < 0:
            raise ValueError("order q >= 2, k >= 0 and fixed_level >= 0 required")
        self.s = sysm
        self.q, self.k = q, k
        self.variant = variant
        self.schedule = schedule
        self.fixed_level = fixed_level
        self.pcg_iters, self.pcg_tol = pcg_iters, pcg_tol
        self.P0 = BasePreconditioner(sysm) if base is None else base
        self._A_lu = None

    # -- V block, eq. Pcv ---------------------------------------------------
    def apply_V(self, level, x):
        """P_{V,level}^{-1} x."""
        if level == 0:
            return self.P0.apply_V0(x)
        return hyperpower_apply(lambda y: self.apply_V(level - 1, y), self.P0.A, self.q, x)

    # -- Q block ----------------------------------------------------------------
    def l_of(self, k):
        """Index l of P_{V,l} used by the k-th update (k >= 1) of eq. Pcq1."""
        if self.schedule == "literal":
            return 0 if k == 1 else k
        return k - 1

    def S_tilde(self, level_v, x):
        """S~_l x = B^T P_{V,l}^{-1} B x."""
        return self.P0.Bt(self.apply_V(level_v, self.P0.B(x)))

    def S_exact(self, x):
        """S x = B^T A^{-1} B x (eq. Pcq_exact), A^{-1} by sparse LU."""
        if self._A_lu is None:
            self._A_lu = spla.splu(self.s.A.tocsc())
        return self.P0.Bt(self._A_lu.solve(self.P0.B(x)))

    def pcg(self, b):
        """Preconditioned conjugate gradients for A y = b from y = 0 with
        P_{V,l}, l = fixed_level (Hestenes-Stiefel), at most pcg_iters steps;
        stops once sqrt(r.z) <= pcg_tol sqrt(r_0.z_0)."""
        y = np.zeros_like(b)
        r = b.copy()
        z = self.apply_V(self.fixed_level, r)
        p = z.copy()
        rz = r @ z
        rz0 = rz
        for _ in range(self.pcg_iters):
            if not rz > 0.0 or np.sqrt(rz) <= self.pcg_tol * np.sqrt(rz0):
                break
            Ap = self.P0.A(p)
            alpha = rz / (p @ Ap)
            y = y + alpha * p
            r = r - alpha * Ap
            z = self.apply_V(self.fixed_level, r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        return y

    def S_pcg(self, x):
        """S_pcg x = B^T PCG(A, P_{V,l}) B x (options (3), (4) of Sec. 4.1)."""
        return self.P0.Bt(self.pcg(self.P0.B(x)))

    def apply_Q(self, level, x):
        """P_{Q,level}^{-1} x for the chosen variant."""
        if level == 0:
            return self.P0.apply_Q0(x)
        if self.variant == "Pcq1":
            lv = self.l_of(level)
            Sop = lambda y: self.S_tilde(lv, y)        # noqa: E731
        elif self.variant == "Pcq2":
            Sop = lambda y: self.S_tilde(self.fixed_level, y)   # noqa: E731
        elif self.variant == "Pcq_exact":
            Sop = self.S_exact
        elif self.variant == "Pcq_pcg":
            Sop = self.S_pcg
        else:
            raise ValueError(self.variant)
        return hyperpower_apply(lambda y: self.apply_Q(level - 1, y), Sop, self.q, x)

    def apply(self, x):
        nV = self.s.nV
        return np.concatenate([self.apply_V(self.k, x[:nV]), self.apply_Q(self.k, x[nV:])])

    __call__ = apply


def dense_hyperpower(Atilde, X0, q, k):
    """Dense matrices X_0..X_k of the hyper-power recursion (tiny sizes)."""
    Xs = [X0]
    n = Atilde.shape[0]
    for _ in range(k):
        X = Xs[-1]
        R = np.eye(n) - Atilde @ X
        S = np.eye(n)
        T = np.eye(n)
        for _ in range(q - 1):
            T = T @ R
            S = S + T
        Xs.append(X @ S)
    return Xs
