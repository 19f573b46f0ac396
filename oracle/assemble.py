"""Assembly of the Stokes saddle-point system (Secs. 3.1-3.3 of the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Unknowns (App. B.2, the discrete Stokes complex, with degree p):

* velocity component c uses N_{.,p} (interior functions only, v.n = 0 is
  strong) in direction c and M_{.,p-1} in the other two directions;
* the pressure uses M_{.,p-1} in all three directions.

Each field is a tensor with direction 1 fastest (App. A.2, vec ordering) and
the system vector is [u1 | u2 | u3 | p].  The matrix is
``[[A, B], [B^T, 0]]`` (eq. ``systemmatrix``) with

    A_ij = a(phi_j, phi_i) + sigma(phi_j, phi_i),   B_ij = b(phi_i, psi_j),

a, b, sigma as in Sec. 3.1 and alpha = C_pen / h (Sec. 3.2).

Two independent assemblies live here:

* ``assemble_quadrature``: direct 3D tensor Gauss quadrature of the weak
  form, written from the definitions of a, b, sigma and the symmetric
  gradient; slow, for E <= 3.  It is the truth that fixes the scaling of
  the Kronecker blocks.
* ``assemble_kron``: the Kronecker forms of Sec. 3.3.  Deriving the blocks
  from a = int 2 nu grad^s w : grad^s v gives the printed diagonal blocks
  times 2 nu and the printed off-diagonal blocks times nu; B carries no nu.
  This reading is verified against ``assemble_quadrature`` by the tests.
"""
import numpy as np
import scipy.sparse as sps

from .matrices1d import Matrices1D
from .splines import SplinePair, gauss_points


def kron3(A3, A2, A1):
    """A3 (x) A2 (x) A1 as a sparse matrix (direction 1 fastest)."""
    return sps.kron(sps.csr_matrix(A3), sps.kron(sps.csr_matrix(A2), sps.csr_matrix(A1)))


def field_shapes(E, p):
    """Shapes (n1, n2, n3) of u1, u2, u3 and p."""
    nN, nM = E + p - 2, E + p - 1
    return [(nN, nM, nM), (nM, nN, nM), (nM, nM, nN), (nM, nM, nM)]


def block_offsets(E, p):
    """Start offsets of u1, u2, u3, p and the total size."""
    sizes = [int(np.prod(s)) for s in field_shapes(E, p)]
    return np.concatenate([[0], np.cumsum(sizes)])


class KronSystem:
    """The saddle-point system by Kronecker products (Sec. 3.3)."""

    def __init__(self, E, p, nu=1.0, c_pen=None):
        self.E, self.p, self.nu = E, p, nu
        self.c_pen = default_c_pen(p) if c_pen is None else c_pen
        m = Matrices1D(E, p, self.c_pen)
        self.m = m
        Mc, Tc, M, K, C, Cc = m.Mc, m.Tc, m.M_int, m.K_int, m.C_int, m.Cc_int
        # diagonal blocks: 2 nu times the printed generalised Kronecker sums
        self.A11 = 2 * nu * (kron3(Mc, Mc, K) + kron3(Mc, Tc, M) + kron3(Tc, Mc, M))
        self.A22 = 2 * nu * (kron3(Mc, M, Tc) + kron3(Mc, K, Mc) + kron3(Tc, M, Mc))
        self.A33 = 2 * nu * (kron3(M, Mc, Tc) + kron3(M, Tc, Mc) + kron3(K, Mc, Mc))
        # off-diagonal blocks: nu times the printed Kronecker products
        self.A12 = nu * kron3(Mc, C.T, C)
        self.A13 = nu * kron3(C.T, Mc, C)
        self.A23 = nu * kron3(C.T, C, Mc)
        self.A = sps.bmat([[self.A11, self.A12, self.A13],
                           [self.A12.T, self.A22, self.A23],
                           [self.A13.T, self.A23.T, self.A33]]).tocsr()
        self.B1 = kron3(Mc, Mc, Cc)
        self.B2 = kron3(Mc, Cc, Mc)
        self.B3 = kron3(Cc, Mc, Mc)
        self.B = sps.vstack([self.B1, self.B2, self.B3]).tocsr()
        self.nV = self.A.shape[0]
        self.nQ = self.B.shape[1]
        self.N = self.nV + self.nQ
        self.K = sps.bmat([[self.A, self.B], [self.B.T, None]]).tocsr()
        self.Mq = kron3(Mc, Mc, Mc).tocsr()
        self.offsets = block_offsets(E, p)

    def lid_rhs(self, U=1.0):
        """Nitsche right-hand side of the moving lid (see ``lid_rhs_vector``)."""
        return lid_rhs_vector(self.m, self.nu, U, self.N)

    def body_force_rhs(self, modes):
        """Load vector int b.v for a separable body force.

        ``modes[c]`` is a list of (a, (k1, k2, k3)) and
        b_c(x) = sum a sin(pi k1 x1) sin(pi k2 x2) sin(pi k3 x3).
        Integrated by element-wise Gauss quadrature with p+8 points.
        """
        E, p = self.E, self.p
        sp = SplinePair(E, p)
        x, w = gauss_points(E, p, p + 8)
        Nv, _ = sp.N(x)
        Nv = Nv[1:-1]
        Mv, _ = sp.M(x)
        F = np.zeros(self.N)
        off = self.offsets
        for c in range(3):
            fam = [Mv, Mv, Mv]
            fam[c] = Nv
            acc = 0.0
            for a, ks in modes[c]:
                s = [fam[d] @ (w * np.sin(np.pi * ks[d] * x)) for d in range(3)]
                acc = acc + a * np.kron(s[2], np.kron(s[1], s[0]))
            F[off[c]:off[c + 1]] = acc
        return F


def lid_rhs_vector(m, nu, U, N):
    """Nitsche right-hand side of the moving lid g = (U, 0, 0) on x3 = 1.

    The weakly imposed tangential data enter through the penalty and
    consistency parts of sigma (Sec. 3.1):
        F(v) = int_{x3=1} 2 nu (alpha g.v - ((grad^s v) n).g).
    Only component 1 is non-zero (v3 = 0 on x3 = 1 strongly).  ``m`` holds
    the univariate matrices, N is the system size.
    """
    f3 = m.alpha * m.M_at1 - 0.5 * m.dM_at1
    f1 = 2 * nu * U * np.kron(f3, np.kron(m.int_M, m.int_N))
    F = np.zeros(N)
    F[: f1.size] = f1
    return F


class KronRows:
    """Selected entries of K x without assembling K, for meshes too large to
    assemble (Sec. 3.3).

    Every block of K is a sum of Kronecker products c * A3 (x) A2 (x) A1 of
    the univariate matrices (the same blocks as ``KronSystem``), and row
    (i1, i2, i3) of A3 (x) A2 (x) A1 is the outer product of rows i3, i2, i1
    of the factors, so one entry of the product costs a few hundred flops.
    """

    def __init__(self, E, p, nu=1.0, c_pen=None):
        self.E, self.p, self.nu = E, p, nu
        self.c_pen = default_c_pen(p) if c_pen is None else c_pen
        m = Matrices1D(E, p, self.c_pen)
        self.m = m
        Mc, Tc, M, K, C, Cc = m.Mc, m.Tc, m.M_int, m.K_int, m.C_int, m.Cc_int
        t = {}
        t[0, 0] = [(2 * nu, Mc, Mc, K), (2 * nu, Mc, Tc, M), (2 * nu, Tc, Mc, M)]
        t[1, 1] = [(2 * nu, Mc, M, Tc), (2 * nu, Mc, K, Mc), (2 * nu, Tc, M, Mc)]
        t[2, 2] = [(2 * nu, M, Mc, Tc), (2 * nu, M, Tc, Mc), (2 * nu, K, Mc, Mc)]
        t[0, 1] = [(nu, Mc, C.T, C)]
        t[0, 2] = [(nu, C.T, Mc, C)]
        t[1, 2] = [(nu, C.T, C, Mc)]
        t[0, 3] = [(1.0, Mc, Mc, Cc)]
        t[1, 3] = [(1.0, Mc, Cc, Mc)]
        t[2, 3] = [(1.0, Cc, Mc, Mc)]
        # the lower triangle: (A3 (x) A2 (x) A1)^T = A3^T (x) A2^T (x) A1^T
        for (r, c) in list(t):
            t[c, r] = [(a, B3.T, B2.T, B1.T) for (a, B3, B2, B1) in t[r, c]]
        self.terms = t
        self.mq_terms = [(1.0, Mc, Mc, Mc)]   # the pressure mass M_q
        self.shapes = field_shapes(E, p)
        self.offsets = block_offsets(E, p)
        self.N = int(self.offsets[-1])

    def block_entries(self, rb, cb, xc, local, terms=None):
        """Entries ``local`` (indices within row block rb) of K_{rb,cb} xc
        (or of the sum of ``terms`` applied to xc)."""
        n1, n2, _ = self.shapes[rb]
        X = np.asarray(xc).reshape(self.shapes[cb][::-1])
        out = np.zeros(len(local))
        for n, li in enumerate(local):
            i1, i2, i3 = li % n1, (li // n1) % n2, li // (n1 * n2)
            acc = 0.0
            for a, A3, A2, A1 in (self.terms.get((rb, cb), []) if terms is None else terms):
                r3, r2, r1 = A3[i3], A2[i2], A1[i1]
                s3, s2, s1 = np.nonzero(r3)[0], np.nonzero(r2)[0], np.nonzero(r1)[0]
                acc += a * np.einsum("k,j,i,kji->", r3[s3], r2[s2], r1[s1],
                                     X[np.ix_(s3, s2, s1)])
            out[n] = acc
        return out

    def mass_q_entries(self, xq, local):
        """Entries ``local`` of M_q xq (pressure mass, M^ (x) M^ (x) M^)."""
        return self.block_entries(3, 3, xq, local, terms=self.mq_terms)

    def lid_rhs(self, U=1.0):
        """The moving-lid right-hand side (as ``KronSystem.lid_rhs``)."""
        return lid_rhs_vector(self.m, self.nu, U, self.N)

    def rows(self, x, idx):
        """(K x)[idx] for a full vector x."""
        idx = np.asarray(idx)
        off = self.offsets
        out = np.zeros(len(idx))
        for rb in range(4):
            sel = np.nonzero((idx >= off[rb]) & (idx < off[rb + 1]))[0]
            if sel.size == 0:
                continue
            local = idx[sel] - off[rb]
            for cb in range(4):
                if (rb, cb) in self.terms:
                    out[sel] += self.block_entries(rb, cb, x[off[cb]:off[cb + 1]], local)
        return out


C_PEN_DEFAULT = 12.5


def default_c_pen(p):
    """Nitsche penalty constant C_pen (alpha = C_pen / h).

    The paper does not print its value.  The reading is
    C_pen = max(12.5, 2.5 (p + 1)): 12.5 up to degree 4, calibrated on the
    paper's printed numbers (the spectrum of P_{V,0}^{-1} A at 2^3
    elements, degree 4, lies within 0.02 of the reported [0.71, 1.41],
    Sec. 5.2; MINRES counts at 8^3 reproduce Table 1 within +-2 for degrees
    2 and 4), growing with the degree beyond, as the inverse-inequality
    constant that the penalty must dominate does: at degree 8 a constant
    12.5 leaves the Nitsche-augmented T^ indefinite below 6 elements and
    widens sigma(P_{V,0}^{-1} A) at 8^3 to [0.54, 1.86] (P_1 then fails to
    be positive definite), while 22.5 gives [0.672, 1.493] and MINRES
    counts 55, 29, 19 at k = 0, 1, 2 against the printed 56, 29, 19.
    """
    return max(C_PEN_DEFAULT, 2.5 * (p + 1))


# --------------------------------------------------------------------------
# direct 3D quadrature of the weak form (truth for small E)
# --------------------------------------------------------------------------

def _families(sp, x):
    """1D families (values, derivatives) at points x: interior N and all M."""
    Nv, dN = sp.N(x)
    Mv, dM = sp.M(x)
    return (Nv[1:-1], dN[1:-1]), (Mv, dM)


def _vector_basis(sp, pts):
    """Values (nb, nq, 3) and gradients (nb, nq, 3, 3) of all velocity basis
    functions at the tensor points ``pts = (x1, x2, x3)`` (1D arrays).

    grad[..., i, j] = d phi_i / d x_j.
    """
    fams = [_families(sp, x) for x in pts]
    vals, grads = [], []
    nq = [len(x) for x in pts]
    for c in range(3):
        f = []
        for d in range(3):
            Nd, Md = fams[d]
            f.append(Nd if d == c else Md)
        n = [f[d][0].shape[0] for d in range(3)]
        # values of the scalar factor and its partial derivatives
        V = np.einsum('ia,jb,kc->kjicba', f[0][0], f[1][0], f[2][0])
        G = [np.einsum('ia,jb,kc->kjicba', f[0][1], f[1][0], f[2][0]),
             np.einsum('ia,jb,kc->kjicba', f[0][0], f[1][1], f[2][0]),
             np.einsum('ia,jb,kc->kjicba', f[0][0], f[1][0], f[2][1])]
        nb = n[0] * n[1] * n[2]
        q = nq[0] * nq[1] * nq[2]
        # basis index with direction 1 fastest; point index with x1 fastest
        V = V.reshape(nb, q)
        G = [g.reshape(nb, q) for g in G]
        val = np.zeros((nb, q, 3))
        val[:, :, c] = V
        grad = np.zeros((nb, q, 3, 3))
        for d in range(3):
            grad[:, :, c, d] = G[d]
        vals.append(val)
        grads.append(grad)
    return np.concatenate(vals), np.concatenate(grads)


def _pressure_basis(sp, pts):
    Ms = [sp.M(x)[0] for x in pts]
    P = np.einsum('ia,jb,kc->kjicba', Ms[0], Ms[1], Ms[2])
    return P.reshape(P.shape[0] * P.shape[1] * P.shape[2], -1)


def _tensor_weights(ws):
    return np.einsum('a,b,c->cba', ws[0], ws[1], ws[2]).reshape(-1)


def assemble_quadrature(E, p, nu=1.0, c_pen=None, U=1.0, modes=None):
    """A, B and the right-hand side by direct 3D/2D quadrature of Sec. 3.1.

    Returns dense (A, B, F_u).  Intended for E <= 3 only.
    """
    c_pen = default_c_pen(p) if c_pen is None else c_pen
    sp = SplinePair(E, p)
    h = 1.0 / E
    alpha = c_pen / h
    nq1 = p + 2
    x, w = gauss_points(E, p, nq1)
    pts = (x, x, x)
    val, grad = _vector_basis(sp, pts)
    wq = _tensor_weights((w, w, w))
    eps = 0.5 * (grad + np.swapaxes(grad, 2, 3))
    nb = val.shape[0]
    Emat = eps.reshape(nb, -1)
    wrep = np.repeat(wq, 9)
    A = 2 * nu * (Emat * wrep) @ Emat.T
    div = np.einsum('bqii->bq', grad)
    P = _pressure_basis(sp, pts)
    B = (div * wq) @ P.T
    F = np.zeros(nb)
    if modes is not None:
        xb, wb = gauss_points(E, p, p + 8)
        valb, _ = _vector_basis(sp, (xb, xb, xb))
        wqb = _tensor_weights((wb, wb, wb))
        nb1 = len(xb)
        X1 = np.broadcast_to(xb[None, None, :], (nb1,) * 3).reshape(-1)
        X2 = np.broadcast_to(xb[None, :, None], (nb1,) * 3).reshape(-1)
        X3 = np.broadcast_to(xb[:, None, None], (nb1,) * 3).reshape(-1)
        for c in range(3):
            bc = np.zeros_like(X1)
            for a, ks in modes[c]:
                bc = bc + a * (np.sin(np.pi * ks[0] * X1) * np.sin(np.pi * ks[1] * X2)
                               * np.sin(np.pi * ks[2] * X3))
            F += valb[:, :, c] @ (bc * wqb)
    # boundary terms: six faces
    for d in range(3):
        for s in (0.0, 1.0):
            normal = np.zeros(3)
            normal[d] = 2 * s - 1
            fpts = [x, x, x]
            fw = [w, w, w]
            fpts[d] = np.array([s])
            fw[d] = np.array([1.0])
            fval, fgrad = _vector_basis(sp, fpts)
            fwq = _tensor_weights(fw)
            feps = 0.5 * (fgrad + np.swapaxes(fgrad, 2, 3))
            epsn = np.einsum('bqij,j->bqi', feps, normal)   # (grad^s v) n
            vw = np.einsum('aqi,bqi,q->ab', fval, fval, fwq)
            cons = np.einsum('aqi,bqi,q->ab', fval, epsn, fwq)  # (eps(phi_b) n).phi_a
            # sigma(w=phi_b, v=phi_a): row a, column b
            A += 2 * nu * (alpha * vw - cons - cons.T)
            if d == 2 and s == 1.0:
                g = np.array([U, 0.0, 0.0])
                gv = np.einsum('aqi,i,q->a', fval, g, fwq)
                eng = np.einsum('aqi,i,q->a', epsn, g, fwq)
                F += 2 * nu * (alpha * gv - eng)
    return A, B, F
