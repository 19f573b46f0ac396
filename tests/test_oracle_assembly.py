"""Pins of the oracle's saddle-point assembly (Secs. 3.1-3.3, App. A).

The Kronecker assembly is compared with direct 3D quadrature of the weak
form (which fixes the nu scaling of each block), and with invariants:
symmetry, definiteness, the pressure null space, the divergence identity
B^T u = M_q D u and the Kronecker-product identities of App. A.1-A.2.
"""
import numpy as np
import pytest
import scipy.sparse as sps

from oracle.assemble import KronSystem, assemble_quadrature, kron3
from oracle.matrices1d import difference_matrix


@pytest.mark.parametrize("E,p,nu", [(1, 2, 1.0), (2, 2, 2.0), (2, 3, 0.5), (3, 2, 1.0)])
def test_kronecker_equals_quadrature(E, p, nu):
    S = KronSystem(E, p, nu)
    A, B, F = assemble_quadrature(E, p, nu, U=1.3)
    assert np.abs(S.A.toarray() - A).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(S.B.toarray() - B).max() <= 1e-13 * np.abs(B).max()
    Fk = S.lid_rhs(1.3)[:S.nV]
    assert np.abs(Fk - F).max() <= 1e-13 * np.abs(F).max()


def test_body_force_rhs_equals_quadrature():
    modes = [[(0.7, (1, 2, 1)), (-0.2, (3, 1, 2))], [(0.4, (2, 2, 1))], [(1.1, (1, 1, 3))]]
    E, p = 2, 3
    S = KronSystem(E, p, 1.0)
    _, _, F0 = assemble_quadrature(E, p, 1.0, U=0.0)
    _, _, F1 = assemble_quadrature(E, p, 1.0, U=0.0, modes=modes)
    Fb = S.body_force_rhs(modes)[:S.nV]
    assert np.abs(Fb - (F1 - F0)).max() <= 1e-12 * np.abs(Fb).max()


@pytest.mark.parametrize("E,p", [(2, 2), (3, 3), (2, 4)])
def test_symmetry_and_definiteness(E, p):
    S = KronSystem(E, p, 1.0)
    K = S.K.toarray()
    assert np.abs(K - K.T).max() <= 1e-14 * np.abs(K).max()
    assert np.linalg.eigvalsh(S.A.toarray()).min() > 0
    ev = np.linalg.eigvalsh(K)
    # saddle point: n_V positive, n_Q - 1 negative, one zero (constant pressure)
    tol = 1e-10 * np.abs(ev).max()
    assert (ev > tol).sum() == S.nV
    assert (ev < -tol).sum() == S.nQ - 1


@pytest.mark.parametrize("E,p", [(2, 2), (5, 3), (4, 4)])
def test_constant_pressure_is_in_null_space_of_B(E, p):
    """B q_c = 0 for the constant pressure: int div v = int v.n = 0."""
    S = KronSystem(E, p, 1.0)
    g = S.m.sp.m_integrals        # 1 = sum_i (int N_{i,p-1}) M_i
    qc = np.kron(g, np.kron(g, g))
    assert np.abs(S.B @ qc).max() <= 1e-13 * np.abs(S.B).max() * np.abs(qc).max()


@pytest.mark.parametrize("E,p", [(3, 2), (4, 3)])
def test_divergence_identity(E, p):
    """B^T u = M_q D u with D the coefficient-wise difference (App. B.1)."""
    S = KronSystem(E, p, 1.0)
    n = S.m.n
    Dh = difference_matrix(n)[:, 1:-1]     # boundary columns removed
    nM = n - 1
    I = np.eye(nM)
    D = sps.hstack([kron3(I, I, Dh), kron3(I, Dh, I), kron3(Dh, I, I)])
    u = np.random.default_rng(3).standard_normal(S.nV)
    assert np.allclose(S.B.T @ u, S.Mq @ (D @ u), atol=1e-12 * np.abs(S.B.T @ u).max())


def test_kronecker_identities():
    """App. A.1 properties and the tensor-contraction form of App. A.2."""
    rng = np.random.default_rng(5)
    A, B, C, Dm = (rng.standard_normal((3, 3)), rng.standard_normal((4, 4)),
                   rng.standard_normal((3, 2)), rng.standard_normal((4, 5)))
    assert np.allclose(np.kron(A, B) @ np.kron(C, Dm), np.kron(A @ C, B @ Dm))
    assert np.allclose(np.linalg.inv(np.kron(A, B)), np.kron(np.linalg.inv(A), np.linalg.inv(B)))
    assert np.allclose(np.kron(A, B).T, np.kron(A.T, B.T))
    assert np.allclose(np.kron(np.kron(A, B), C), np.kron(A, np.kron(B, C)))
    # vec ordering: direction 1 fastest
    D1, D2, D3 = rng.standard_normal((2, 3)), rng.standard_normal((4, 5)), rng.standard_normal((3, 2))
    X = rng.standard_normal((3, 5, 2))            # X[i1, i2, i3]
    vecX = X.reshape(-1, order="F")
    Y = np.einsum("ai,bj,ck,ijk->abc", D1, D2, D3, X)
    assert np.allclose(kron3(D3, D2, D1) @ vecX, Y.reshape(-1, order="F"))


def test_sizes_match_the_complex():
    """dim V_h = 3 (E+p-2)(E+p-1)^2, dim Q_h = (E+p-1)^3 (App. B.2)."""
    for E, p in [(8, 2), (32, 3)]:
        S = KronSystem(E, p, 1.0) if E == 8 else None
        nN, nM = E + p - 2, E + p - 1
        if S is not None:
            assert S.nV == 3 * nN * nM * nM and S.nQ == nM ** 3
    assert 3 * 8 * 81 + 729 == 2673
    assert 3 * 33 * 34 ** 2 + 34 ** 3 == 153748


@pytest.mark.parametrize("E,p", [(4, 2), (3, 3), (5, 4), (2, 2)])
def test_kron_rows_match_the_assembled_matrix(E, p):
    """Row-by-row evaluation of K x (used for sampled checks on meshes too
    large to assemble) equals the assembled Kronecker system on every row."""
    from oracle.assemble import KronRows, KronSystem
    S = KronSystem(E, p, 1.3)
    R = KronRows(E, p, 1.3)
    assert R.N == S.N
    x = np.random.default_rng(7).standard_normal(S.N)
    y = R.rows(x, np.arange(S.N))
    ref = S.K @ x
    assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
    # a single velocity block on its own: rows of A_22 u_2
    o = S.offsets
    loc = np.arange(o[2] - o[1])
    y22 = R.block_entries(1, 1, x[o[1]:o[2]], loc)
    assert np.allclose(y22, S.A22 @ x[o[1]:o[2]], rtol=0, atol=1e-13 * np.abs(y22).max())
    xq = x[o[3]:]
    yq = R.mass_q_entries(xq, np.arange(xq.size))
    assert np.allclose(yq, S.Mq @ xq, rtol=0, atol=1e-13 * np.abs(yq).max())


def _quadrature_flux_apply(E, p, nu, x, shared=False):
    """K x by the pointwise flux form the quadrature-based GPU operator uses:
    gradients and pressure at the points [0, the E(p+1) Gauss points, 1] of
    each direction; volume flux nu (G + G^T) + P I and div u; on a face
    normal to d (outward sign s) and tangential c != d only
    nu (2 alpha u_c v_c - s d_d u_c v_c - s u_c d_d v_c); edges carry
    nothing.  Written with numpy contractions (slow, small meshes).
    shared=True stores the off-diagonal fluxes as one field per pair
    (c, d), S_cd = the coefficient of d_d v_c where c is tangential to the
    face, else of d_c v_d, and reads it for both."""
    from oracle.assemble import block_offsets, default_c_pen, field_shapes
    from oracle.splines import SplinePair, gauss_points
    sp = SplinePair(E, p)
    xg, wg = gauss_points(E, p)
    pts = np.concatenate([[0.0], xg, [1.0]])
    w1 = np.concatenate([[1.0], wg, [1.0]])
    nq = pts.size
    NV, ND = sp.N(pts)
    MV, MD = sp.M(pts)
    tab = {"N": (NV[1:-1].T, ND[1:-1].T), "M": (MV.T, MD.T)}
    alpha = default_c_pen(p) * E
    sh, off = field_shapes(E, p), block_offsets(E, p)
    f = [x[off[b]:off[b + 1]].reshape(sh[b][::-1]) for b in range(4)]   # [i3, i2, i1]

    def mode(A, X, m):       # contract direction m (axis 2 - m)
        ax = 2 - m
        return np.moveaxis(np.tensordot(A, X, axes=([1], [ax])), 0, ax)

    def typ(c, d):
        return "N" if c == d else "M"

    U, G = [], []
    for c in range(3):
        V1, D1 = tab[typ(c, 0)]
        V2, D2 = tab[typ(c, 1)]
        V3, D3 = tab[typ(c, 2)]
        a, b = mode(V1, f[c], 0), mode(D1, f[c], 0)
        U.append(mode(V3, mode(V2, a, 1), 2))
        G.append([mode(V3, mode(V2, b, 1), 2), mode(V3, mode(D2, a, 1), 2),
                  mode(D3, mode(V2, a, 1), 2)])
    Mv = tab["M"][0]
    P = mode(Mv, mode(Mv, mode(Mv, f[3], 0), 1), 2)
    W = w1[:, None, None] * w1[None, :, None] * w1[None, None, :]
    end = np.zeros(nq, bool)
    end[0] = end[-1] = True
    e2, e1, e0 = np.meshgrid(end, end, end, indexing="ij")
    ne = e0.astype(int) + e1 + e2
    vol = ne == 0
    Fq = np.where(vol, W * (G[0][0] + G[1][1] + G[2][2]), 0.0)
    F = [[np.zeros_like(W)] + [np.where(vol, W * nu * (G[c][d] + G[d][c])
                                        + (W * P if c == d else 0.0), 0.0) for d in range(3)]
         for c in range(3)]
    sgn = np.ones(nq)
    sgn[0] = -1.0
    for d, (ed, ax) in enumerate([(e0, 2), (e1, 1), (e2, 0)]):
        face = (ne == 1) & ed
        shp = [1, 1, 1]
        shp[ax] = nq
        s = sgn.reshape(shp)
        for c in range(3):
            if c != d:
                F[c][0] = F[c][0] + np.where(face, W * nu * (2 * alpha * U[c] - s * G[c][d]), 0.0)
                F[c][1 + d] = F[c][1 + d] + np.where(face, -W * nu * s * U[c], 0.0)
    if shared:
        for c in range(3):
            for d in range(c + 1, 3):
                S = F[c][1 + d] + F[d][1 + c]      # never both nonzero off the volume
                vol_ok = np.allclose(np.where(vol, F[c][1 + d] - F[d][1 + c], 0.0), 0.0)
                assert vol_ok
                S = np.where(vol, F[c][1 + d], S)
                F[c][1 + d] = S
                F[d][1 + c] = S
    out = []
    for c in range(3):
        V1, D1 = tab[typ(c, 0)]
        V2, D2 = tab[typ(c, 1)]
        V3, D3 = tab[typ(c, 2)]
        aa = mode(V3.T, F[c][0], 2) + mode(D3.T, F[c][3], 2)
        a = mode(V2.T, aa, 1) + mode(D2.T, mode(V3.T, F[c][2], 2), 1)
        b = mode(V2.T, mode(V3.T, F[c][1], 2), 1)
        out.append((mode(V1.T, a, 0) + mode(D1.T, b, 0)).ravel())
    out.append(mode(Mv.T, mode(Mv.T, mode(Mv.T, Fq, 2), 1), 0).ravel())
    return np.concatenate(out)


@pytest.mark.parametrize("E,p,nu", [(2, 2, 1.0), (3, 2, 1.3), (3, 3, 0.7), (2, 5, 1.0)])
def test_quadrature_flux_form_equals_K(E, p, nu):
    """The reading behind the quadrature-based forward operator (Sec. 5.3):
    the symmetric-gradient volume flux plus the face terms that keep only
    the normal derivative of the tangential components (the normal component
    and its tangential derivatives vanish on the face) reproduce K exactly
    (Gauss with p+1 points is exact for these integrands).  Dropping the
    consistency term or the edge rule breaks the match.  The same holds with
    one field per off-diagonal pair (the storage of the GPU kernel): on a
    face normal to c the value meant for component d is read by component c
    only through its own direction-c value table, which vanishes there."""
    S = KronSystem(E, p, nu)
    x = np.random.default_rng(E * 10 + p).standard_normal(S.N)
    ref = S.K @ x
    for shared in (False, True):
        y = _quadrature_flux_apply(E, p, nu, x, shared=shared)
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max()
