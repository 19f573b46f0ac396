"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (FP64 everywhere on the GPU path):
* sum-factorised operators (K, A, B, B^T, M_V): 1e-12 relative (max-norm);
  the kernels sum the same products as the Kronecker assembly in another
  order, so the gap is a few ulps times the band width;
* P_0^{-1}: fast diagonalisation (GPU) against sparse LU (oracle).  Both
  are backward stable: each velocity block has normwise backward error
  <= 1e-14, so the forward gap is bounded by 1e-14 kappa(A_cc); the test
  asserts max(1e-12, 1e-14 kappa) with kappa the exact condition number of
  the blocks (dense eigenvalues), 1e-12 wherever kappa <= 100;
* P_k^{-1}: q^k applications of P_0^{-1} (Richardson form of eq. Pcv, and
  the Schur recursion), each adding at most that backward error, and
  contractions in between (|1 - lambda| < 1), so the forward gap is bounded
  by max(1e-12, 1e-14 q^k kappa); the velocity block is also checked in
  backward form through the closed form I - A P_{V,k}^{-1} =
  (I - A P_{V,0}^{-1})^{q^k}: |(x - A y) - r_ref| / (|A| |y| + |x|) <=
  1e-14 q^k with r_ref the oracle's q^k-fold residual;
* MINRES/FGMRES: iteration counts within +-1 of the oracle's, solutions
  agree to 1e-6 (tolerance 1e-8 on the residual).
Sizes span several 8-row strips, 16-wide MFMA tiles and 64-row blocks, with
ragged tails (n = 9, 10, 11, 13, 14, 17, 18), degrees 2 to 8, and the meshes
of one and two elements per direction, where the band half-width (the
degree) reaches or exceeds the number of functions in a direction.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2311_06926_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = [(3, 2), (8, 2), (5, 3), (8, 3), (12, 2), (15, 3), (4, 4), (5, 5), (4, 6), (3, 7),
         (6, 8), (1, 2), (1, 3), (1, 5), (2, 2), (2, 3), (2, 8)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


_ORACLE = {}


def oracle_sys(E, p, nu=1.0):
    from oracle.assemble import KronSystem
    key = (E, p, nu)
    if key not in _ORACLE:
        _ORACLE[key] = KronSystem(E, p, nu)
    return _ORACLE[key]


def to_gpu(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


_KAPPA = {}


def block_kappa(S):
    """Largest 2-norm condition number of the three diagonal blocks A_cc
    (dense symmetric eigenvalues; the blocks have at most a few thousand
    rows at the parity sizes)."""
    import scipy.linalg as sla
    key = (S.E, S.p, S.nu)
    if key not in _KAPPA:
        kap = 1.0
        for blk in (S.A11, S.A22, S.A33):
            ev = sla.eigvalsh(blk.toarray())
            kap = max(kap, ev[-1] / ev[0])
        _KAPPA[key] = kap
    return _KAPPA[key]


def pk_forward_bound(S, q, k):
    return max(1e-12, 1e-14 * q ** k * block_kappa(S))


def pv_backward_error(S, P0, q, k, xv, yv):
    """|(x - A y) - r_ref|_inf / (|A|_inf |y|_inf + |x|_inf) with r_ref =
    (I - A P_{V,0}^{-1})^{q^k} x by the oracle (closed form of eq. Pcv)."""
    r_ref = xv.copy()
    for _ in range(q ** k):
        r_ref = r_ref - S.A @ P0.apply_V0(r_ref)
    r = xv - S.A @ yv
    norm_a = abs(S.A).sum(axis=1).max()
    return np.abs(r - r_ref).max() / (norm_a * np.abs(yv).max() + np.abs(xv).max())


@pytest.mark.parametrize("E,p", CASES)
def test_operators(dev, E, p):
    from paper_2311_06926_amd.solver import Solver
    from oracle.cases import velocity_mass
    nu = 1.7
    say(f"[parity] operators E={E} p={p} nu={nu}")
    S = oracle_sys(E, p, nu)
    sol = Solver(E, p, nu)
    assert sol.N == S.N and sol.nV == S.nV
    x = synth.random_vector(S.N, seed=E * 10 + p)
    y = sol.apply_K(to_gpu(x, dev)).cpu().numpy()
    assert rel_err(y, S.K @ x) < 1e-12
    u, pr = x[:S.nV], x[S.nV:]
    assert rel_err(sol.apply_A(to_gpu(u, dev)).cpu().numpy(), S.A @ u) < 1e-12
    assert rel_err(sol.apply_B(to_gpu(pr, dev)).cpu().numpy(), S.B @ pr) < 1e-12
    assert rel_err(sol.apply_Bt(to_gpu(u, dev)).cpu().numpy(), S.B.T @ u) < 1e-12
    MV = velocity_mass(S)
    assert rel_err(sol.apply_MV(to_gpu(u, dev)).cpu().numpy(), MV @ u) < 1e-12
    sol.close()


@pytest.mark.parametrize("E,p", [(2, 2), (3, 2), (8, 2), (5, 3), (9, 3), (4, 4), (3, 6),
                                 (2, 8)])
def test_apply_K_quad_matches_oracle(dev, E, p):
    """The quadrature-based forward operator (Sec. 5.3: Gauss points, flux of
    the weak form, Nitsche face terms) against the oracle's K.  The quadrature
    is exact, so this is the same matrix; two right-hand sides in one call."""
    from paper_2311_06926_amd.solver import Solver
    nu = 1.3
    say(f"[parity] apply_K_quad E={E} p={p} nu={nu}")
    S = oracle_sys(E, p, nu)
    sol = Solver(E, p, nu, max_rhs=2)
    x = np.concatenate([synth.random_vector(S.N, seed=E * 10 + p),
                        synth.random_vector(S.N, seed=E * 10 + p + 1)])
    y = sol.apply_K_quad(to_gpu(x, dev)).cpu().numpy()
    for r in range(2):
        seg = slice(r * S.N, (r + 1) * S.N)
        assert rel_err(y[seg], S.K @ x[seg]) < 1e-12
    sol.close()


@pytest.mark.parametrize("E,p", CASES)
def test_base_preconditioner(dev, E, p):
    """P_0 against sparse LU.  Both are backward stable, so each velocity
    block is checked by its normwise backward error
    |A_cc y - x| / (|A_cc| |y| + |x|) (max norms) <= 1e-14, and the forward
    gap by max(1e-11, 1e-14 kappa), kappa >= |A_cc| |y| / |x| (the blocks'
    condition grows fast with the degree: ~1e11 at degree 8)."""
    from oracle.precond import BasePreconditioner
    from paper_2311_06926_amd.solver import Solver
    nu = 0.8
    say(f"[parity] P0 E={E} p={p}")
    S = oracle_sys(E, p, nu)
    P0 = BasePreconditioner(S)
    sol = Solver(E, p, nu)
    x = synth.random_vector(S.N, seed=100 + E * 10 + p)
    y = sol.apply_P0(to_gpu(x, dev)).cpu().numpy()
    ref = P0.apply(x)
    o = S.offsets
    for c, blk in enumerate([S.A11, S.A22, S.A33]):
        yc, xc = y[o[c]:o[c + 1]], x[o[c]:o[c + 1]]
        norm_a = abs(blk).sum(axis=1).max()
        r = blk @ yc - xc
        eta = np.abs(r).max() / (norm_a * np.abs(yc).max() + np.abs(xc).max())
        assert eta <= 1e-14, (c, eta)
    kappa = block_kappa(S)
    gap = rel_err(y, ref)
    say(f"[parity]   P0 forward gap {gap:.2e}, kappa {kappa:.2e}")
    assert gap < max(1e-12, 1e-14 * kappa)
    # the pressure block alone: 2 nu (M^^{-1})^{(x)3} by three 1D solves (oracle)
    assert rel_err(y[S.nV:], ref[S.nV:]) < 1e-12
    sol.close()


@pytest.mark.parametrize("E,p", [(3, 2), (8, 3), (13, 2)])
@pytest.mark.parametrize("q,k", [(2, 1), (2, 2), (3, 1), (3, 2), (2, 3)])
@pytest.mark.parametrize("variant", ["Pcq1", "Pcq2"])
def test_hyperpower(dev, E, p, q, k, variant):
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] hyperpower E={E} p={p} q={q} k={k} {variant}")
    S = oracle_sys(E, p)
    H = HyperPower(S, q, k, variant=variant)
    sol = Solver(E, p, 1.0, schur=variant)
    x = synth.random_vector(S.N, seed=200 + q * 10 + k)
    y = sol.apply_hyperpower(q, k, to_gpu(x, dev)).cpu().numpy()
    gap = rel_err(y, H.apply(x))
    eta = pv_backward_error(S, H.P0, q, k, x[:S.nV], y[:S.nV])
    say(f"[parity]   forward gap {gap:.2e} (kappa bound {pk_forward_bound(S, q, k):.1e}), "
        f"V backward {eta:.2e}")
    # degrees 2 and 3: the blocks' condition numbers (<= 2e4) leave the
    # kappa bound far above 1e-12; the measured gaps are a few 1e-15
    assert gap < 1e-12
    assert eta <= 1e-15
    sol.close()


@pytest.mark.parametrize("E,p", [(5, 5), (4, 6)])
def test_hyperpower_high_degree(dev, E, p):
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] hyperpower E={E} p={p} q=2 k=2 Pcq1")
    S = oracle_sys(E, p)
    sol = Solver(E, p, 1.0)
    x = synth.random_vector(S.N, seed=300 + p)
    y = sol.apply_hyperpower(2, 2, to_gpu(x, dev)).cpu().numpy()
    H = HyperPower(S, 2, 2)
    gap = rel_err(y, H.apply(x))
    eta = pv_backward_error(S, H.P0, 2, 2, x[:S.nV], y[:S.nV])
    bound = pk_forward_bound(S, 2, 2)
    say(f"[parity]   forward gap {gap:.2e} (bound {bound:.1e}, kappa "
        f"{block_kappa(S):.1e}), V backward {eta:.2e}")
    assert gap < bound
    assert eta <= 1e-15
    sol.close()


def test_penalty_too_small_is_rejected(dev):
    """Degree 8 on 5 elements with C_pen = 12.5: T^ is indefinite."""
    from paper_2311_06926_amd._lib import HPError
    from paper_2311_06926_amd.solver import Solver
    with pytest.raises(HPError) as e:
        Solver(5, 8, 1.0, c_pen=12.5)
    assert e.value.code == -4
    Solver(6, 8, 1.0).close()


def test_hyperpower_prev_schedule(dev):
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    say("[parity] hyperpower schedule=prev")
    S = oracle_sys(5, 3)
    H = HyperPower(S, 2, 3, variant="Pcq1", schedule="prev")
    sol = Solver(5, 3, 1.0, schedule="prev")
    x = synth.random_vector(S.N, seed=301)
    y = sol.apply_hyperpower(2, 3, to_gpu(x, dev)).cpu().numpy()
    gap = rel_err(y, H.apply(x))
    say(f"[parity]   forward gap {gap:.2e}")
    assert gap < 1e-12
    sol.close()


def test_batched_apply_matches_single(dev):
    from paper_2311_06926_amd.solver import Solver
    say("[parity] batched apply_K / P_k, nrhs=3")
    E, p = 7, 3
    sol = Solver(E, p, 1.0, max_rhs=3)
    xs = [synth.random_vector(sol.N, seed=400 + r) for r in range(3)]
    xb = to_gpu(np.concatenate(xs), dev)
    yb = sol.apply_K(xb).cpu().numpy().reshape(3, -1)
    hb = sol.apply_hyperpower(2, 2, xb).cpu().numpy().reshape(3, -1)
    for r in range(3):
        y1 = sol.apply_K(to_gpu(xs[r], dev)).cpu().numpy()
        h1 = sol.apply_hyperpower(2, 2, to_gpu(xs[r], dev)).cpu().numpy()
        assert np.array_equal(yb[r], y1)
        assert np.array_equal(hb[r], h1)
    sol.close()


def test_rhs_matches_oracle(dev):
    from oracle.assemble import KronSystem
    from paper_2311_06926_amd.solver import Solver
    say("[parity] rhs build (lid + body force), nrhs=2")
    E, p = 6, 3
    sol = Solver(E, p, 1.3, max_rhs=2)
    S = KronSystem(E, p, 1.3)
    lids, amps, wavs, refs = [], [], [], []
    for r in range(2):
        modes, U = synth.body_force_modes(r, nmodes=4)
        amp, wav = synth.modes_to_arrays(modes)
        lids.append(U)
        amps.append(amp)
        wavs.append(wav)
        refs.append(S.lid_rhs(U) + S.body_force_rhs(modes))
    b = sol.build_rhs(np.array(lids), (np.stack(amps), np.stack(wavs))).cpu().numpy()
    assert rel_err(b, np.concatenate(refs)) < 1e-12
    sol.close()


@pytest.mark.parametrize("k", [0, 1, 2])
def test_minres_config1(dev, k):
    """8^3 elements, degree 2, q = 2: iteration counts within +-1 of the oracle."""
    from oracle.cases import cavity
    from oracle.direct import mean_zero_pressure
    from oracle.krylov import minres
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] MINRES 8^3 p=2 k={k}")
    S, b = cavity(8, 2)
    ref = minres(lambda v: S.K @ v, HyperPower(S, 2, k).apply, b, tol=1e-8)
    sol = Solver(8, 2, 1.0, iters=k)
    bg = sol.build_rhs([1.0])
    assert rel_err(bg.cpu().numpy(), b) < 1e-13
    x, info = sol.solve(bg, tol=1e-8)
    say(f"[parity]   {info.iterations} iterations (oracle {ref.iters}), true relres "
        f"{info.true_relres:.2e} (oracle {ref.true_relres:.2e})")
    assert abs(info.iterations - ref.iters) <= 1
    assert info.converged == 1
    # MINRES stops on the P^{-1}-norm; the 2-norm residual is also below tol here
    assert info.true_relres <= 1.01 * 1e-8
    xg = mean_zero_pressure(x.cpu().numpy(), S.nV)
    xr = mean_zero_pressure(ref.x, S.nV)
    assert np.linalg.norm(xg[:S.nV] - xr[:S.nV]) <= 1e-6 * np.linalg.norm(xr[:S.nV])
    sol.close()


@pytest.mark.parametrize("m", [1, 2, 3, 7])
@pytest.mark.parametrize("graph", [1, 0])
def test_minres_iteration_limit_matches_oracle_iterates(dev, m, graph):
    """MINRES stopped by the iteration limit (tol 0): the GPU iterate after m
    steps equals the oracle's m-th iterate (the same recurrences), and the
    solve reports m iterations and HP_ENOCONV."""
    from oracle.cases import cavity
    from oracle.krylov import minres
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] MINRES iteration limit m={m} graph={graph}")
    S, b = cavity(5, 2)
    ref = minres(lambda v: S.K @ v, HyperPower(S, 2, 1).apply, b, tol=0.0, maxit=m)
    sol = Solver(5, 2, 1.0, iters=1, maxit=m, use_graph=graph)
    x, info = sol.solve(sol.build_rhs([1.0]), tol=1e-300, raise_on_noconv=False)
    assert info.iterations == m and info.converged == 0
    xs = x.cpu().numpy()
    assert np.abs(xs[:S.nV] - ref.x[:S.nV]).max() <= 1e-10 * np.abs(ref.x[:S.nV]).max()
    sol.close()


@pytest.mark.parametrize("krylov,graph", [("minres", 0), ("minres", 1), ("fgmres", 0)])
def test_solve_with_quadrature_forward(dev, krylov, graph):
    """The solve with the quadrature-based forward operator in the Krylov loop:
    iteration count within +-1 of the oracle's MINRES, and the solution of the
    same system (its true residual is taken with the Kronecker operator)."""
    from oracle.cases import cavity
    from oracle.direct import mean_zero_pressure
    from oracle.krylov import minres
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] quadrature forward {krylov} graph={graph}")
    S, b = cavity(6, 3)
    ref = minres(lambda v: S.K @ v, HyperPower(S, 2, 1).apply, b, tol=1e-8)
    sol = Solver(6, 3, 1.0, iters=1, krylov=krylov, use_graph=graph, forward="quadrature")
    x, info = sol.solve(sol.build_rhs([1.0]), tol=1e-8)
    assert info.converged == 1 and info.true_relres < 1e-7
    if krylov == "minres":
        assert abs(info.iterations - ref.iters) <= 1
    xg = mean_zero_pressure(x.cpu().numpy(), S.nV)
    xr = mean_zero_pressure(ref.x, S.nV)
    assert np.linalg.norm(xg[:S.nV] - xr[:S.nV]) <= 1e-6 * np.linalg.norm(xr[:S.nV])
    sol.close()


def test_batched_fgmres_with_quadrature_forward(dev):
    """Two lid speeds in one FGMRES solve with the quadrature-based forward
    operator: each right-hand side matches its own single solve with the
    Kronecker operator (the same system), and the lid data scale linearly."""
    from paper_2311_06926_amd.solver import Solver
    say("[parity] batched FGMRES, quadrature forward")
    sq = Solver(5, 3, 1.0, iters=1, krylov="fgmres", max_rhs=2, forward="quadrature")
    xq, iq = sq.solve(sq.build_rhs([1.0, 2.5]), tol=1e-10)
    sk = Solver(5, 3, 1.0, iters=1, krylov="fgmres")
    xk, ik = sk.solve(sk.build_rhs([1.0]), tol=1e-10)
    assert iq.converged == 1 and ik.converged == 1
    N, nV = sq.N, sq.nV
    xq = xq.cpu().numpy()
    xk = xk.cpu().numpy()
    u0, u1, uk = xq[:nV], xq[N:N + nV], xk[:nV]
    assert np.linalg.norm(u0 - uk) <= 1e-6 * np.linalg.norm(uk)
    assert np.linalg.norm(u1 - 2.5 * uk) <= 1e-6 * np.linalg.norm(2.5 * uk)
    sq.close()
    sk.close()


def test_fgmres_matches_oracle(dev):
    from oracle.cases import cavity
    from oracle.krylov import fgmres
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    say("[parity] FGMRES 6^3 p=3 k=1")
    S, b = cavity(6, 3)
    H = HyperPower(S, 2, 1)
    ref = fgmres(lambda v: S.K @ v, lambda v, j: H.apply(v), b, tol=1e-8, restart=50)
    sol = Solver(6, 3, 1.0, iters=1, krylov="fgmres")
    x, info = sol.solve(sol.build_rhs([1.0]), tol=1e-8)
    assert abs(info.iterations - ref.iters) <= 1
    assert info.true_relres <= 1e-8 * 1.01
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs[:S.nV] - ref.x[:S.nV]) <= 1e-6 * np.linalg.norm(ref.x[:S.nV])
    sol.close()


@pytest.mark.parametrize("level,k,m", [(0, 1, 4), (1, 1, 3), (0, 2, 3)])
def test_inner_pcg_schur_variant(dev, level, k, m):
    """Options (3)/(4) of Sec. 4.1: eq. Pcq2 on B' PCG(A, P_{V,l}) B with a
    fixed number of inner steps (tolerance 0), single and batched, against
    the oracle's PCG variant."""
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    E, p = 5, 3
    say(f"[parity] inner-PCG Schur E={E} p={p} l={level} k={k} m={m}")
    S = oracle_sys(E, p)
    H = HyperPower(S, 2, k, variant="Pcq_pcg", fixed_level=level, pcg_iters=m, pcg_tol=0.0)
    sol = Solver(E, p, 1.0, schur="Pcq_pcg", schur_level=level, schur_pcg_iters=m,
                 schur_pcg_tol=0.0, max_rhs=2, krylov="fgmres")
    x = synth.random_vector(2 * S.N, seed=400 + 10 * level + k)
    y = sol.apply_hyperpower(2, k, to_gpu(x, dev)).cpu().numpy()
    for r in range(2):
        xr = x[r * S.N:(r + 1) * S.N]
        gap = rel_err(y[r * S.N:(r + 1) * S.N], H.apply(xr))
        say(f"[parity]   rhs {r}: forward gap {gap:.2e}")
        assert gap < 1e-12, r
    y1 = sol.apply_hyperpower(2, k, to_gpu(x[:S.N], dev)).cpu().numpy()
    assert np.array_equal(y1, y[:S.N])
    sol.close()


def test_inner_pcg_fgmres_solve(dev):
    from oracle.cases import cavity
    from oracle.krylov import fgmres
    from oracle.precond import HyperPower
    from paper_2311_06926_amd._lib import HPError
    from paper_2311_06926_amd.solver import Solver
    say("[parity] FGMRES with the inner-PCG Schur variant, 6^3 p=2 k=1")
    S, b = cavity(6, 2)
    H = HyperPower(S, 2, 1, variant="Pcq_pcg", pcg_iters=5, pcg_tol=0.0)
    ref = fgmres(lambda v: S.K @ v, lambda v, j: H.apply(v), b, tol=1e-8, restart=50)
    sol = Solver(6, 2, 1.0, iters=1, krylov="fgmres", schur="Pcq_pcg", schur_pcg_iters=5,
                 schur_pcg_tol=0.0)
    x, info = sol.solve(sol.build_rhs([1.0]), tol=1e-8)
    assert abs(info.iterations - ref.iters) <= 1
    assert info.true_relres <= 1e-8 * 1.01
    sol.close()
    tolsol = Solver(6, 2, 1.0, iters=2, krylov="fgmres", schur="Pcq_pcg", schur_level=1)
    _, info = tolsol.solve(tolsol.build_rhs([1.0]), tol=1e-8)
    say(f"[parity]   tol 1e-2 inner CG, l=1, k=2: {info.iterations} iterations")
    assert info.converged and info.true_relres <= 1e-8 * 1.01
    tolsol.close()
    mr = Solver(6, 2, 1.0, iters=1, schur="Pcq_pcg")
    with pytest.raises(HPError):
        mr.solve(mr.build_rhs([1.0]), tol=1e-8)
    mr.close()


def test_fp32_preconditioner_error_is_small(dev):
    from paper_2311_06926_amd.solver import Solver
    say("[parity] FP32 P0 vs FP64 P0")
    E, p = 9, 3
    s64 = Solver(E, p, 1.0)
    s32 = Solver(E, p, 1.0, precision="fp32", krylov="fgmres")
    x = to_gpu(synth.random_vector(s64.N, seed=501), dev)
    y64 = s64.apply_P0(x).cpu().numpy()
    y32 = s32.apply_P0(x).cpu().numpy()
    assert rel_err(y32, y64) < 1e-5
    s64.close()
    s32.close()


def test_gradient_matches_oracle(dev):
    from oracle.cases import CavityLoss, cavity
    from oracle.direct import DirectSolver
    from paper_2311_06926_amd.solver import Solver
    say("[parity] adjoint gradient pieces 4^3 p=2")
    E, p, nu = 4, 2, 1.2
    St, bt = cavity(E, p, U=1.5)
    ut = DirectSolver(St).solve(bt)[:St.nV]
    loss = CavityLoss(E, p, U=1.0, u_target=ut)
    beta = synth.random_vector(St.nV, seed=601, scale=0.3)
    L, gb_ref, gn_ref = loss.gradient(beta, nu)
    S, MV, b, x = loss.solve(beta, nu)
    d = x[:S.nV] - ut
    rhs = np.zeros(S.N)
    rhs[:S.nV] = 2.0 * (MV @ d)
    lam = DirectSolver(S).solve(rhs)
    sol = Solver(E, p, nu)
    gb, gn = sol.grad(to_gpu(x, dev), to_gpu(lam, dev), [1.0])
    assert rel_err(gb.cpu().numpy(), gb_ref) < 1e-12
    assert abs(gn[0] - gn_ref) <= 1e-10 * max(abs(gn_ref), 1e-12)
    sol.close()


def test_invalid_arguments(dev):
    from paper_2311_06926_amd._lib import HPError
    from paper_2311_06926_amd.solver import Solver
    say("[parity] invalid arguments")
    sol = Solver(3, 2, 1.0)
    x = torch.zeros(sol.N, dtype=torch.float64, device=dev)
    with pytest.raises(HPError):
        sol.apply_hyperpower(1, 1, x)          # order < 2
    with pytest.raises(HPError):
        sol.apply_K(x, x)                      # aliasing
    with pytest.raises(HPError):
        sol.apply_K(torch.zeros(2 * sol.N, dtype=torch.float64, device=dev))  # nrhs > max_rhs
    with pytest.raises(HPError):
        sol.apply_K_quad(x, x)                 # aliasing
    with pytest.raises(HPError):
        sol.apply_K_quad(torch.zeros(2 * sol.N, dtype=torch.float64, device=dev))
    with pytest.raises(HPError):
        Solver(3, 2, 1.0, precision="fp32").solve(x)    # MINRES needs FP64
    sol.close()


@pytest.mark.parametrize("krylov", ["minres", "fgmres"])
def test_graph_replay_equals_eager_and_is_deterministic(dev, krylov):
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] graph vs eager {krylov}")
    E, p = 7, 3
    sg = Solver(E, p, 1.0, iters=2, krylov=krylov, use_graph=1)
    se = Solver(E, p, 1.0, iters=2, krylov=krylov, use_graph=0)
    b = sg.build_rhs([1.0])
    xg, ig = sg.solve(b, 1e-8)
    xg2, ig2 = sg.solve(b, 1e-8)
    xe, ie = se.solve(b, 1e-8)
    xe2, ie2 = se.solve(b, 1e-8)
    assert ig.iterations == ie.iterations == ig2.iterations == ie2.iterations
    assert torch.equal(xg, xe) and torch.equal(xg, xg2) and torch.equal(xe, xe2)
    sg.close()
    se.close()


@pytest.mark.parametrize("graph", [0, 1])
def test_minres_poll_lag_leaves_solution_unchanged(dev, graph):
    """The host reads the convergence flags poll_lag iterations behind the
    device, so up to poll_lag iterations run past convergence: they must
    leave the solution and the reported iteration count unchanged."""
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] MINRES poll_lag 1..3 graph={graph}")
    E, p = 6, 3
    out = []
    for lag in (1, 2, 3):
        s = Solver(E, p, 1.0, iters=1, poll_lag=lag, use_graph=graph, max_rhs=2)
        b = s.build_rhs([1.0, 0.7])
        x, info = s.solve(b, 1e-8)
        out.append((x, info.iterations, list(info.iters_per_rhs[:2])))
        s.close()
    for x, its, per in out[1:]:
        assert its == out[0][1] and per == out[0][2]
        assert torch.equal(x, out[0][0])


@pytest.mark.parametrize("krylov", ["minres", "fgmres"])
def test_batched_solve_matches_single(dev, krylov):
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] batched solve nrhs=3 {krylov}")
    E, p, R = 6, 2, 3
    # the same P_0 plan in both contexts: the plan sets how P_k's last
    # launches split the Krylov dot into partials (the summation order)
    sb = Solver(E, p, 1.0, iters=1, krylov=krylov, max_rhs=R, fd_plan=1)
    ss = Solver(E, p, 1.0, iters=1, krylov=krylov, fd_plan=1)
    lids, amps, wavs = [], [], []
    for r in range(R):
        modes, U = synth.body_force_modes(r, nmodes=16)
        amp, wav = synth.modes_to_arrays(modes)
        lids.append(U)
        amps.append(amp)
        wavs.append(wav)
    b = sb.build_rhs(np.array(lids), (np.stack(amps), np.stack(wavs)))
    xb, ib = sb.solve(b, 1e-8)
    assert ib.converged == 1
    for r in range(R):
        br = b[r * sb.N:(r + 1) * sb.N].clone()
        xs, is_ = ss.solve(br, 1e-8)
        assert ib.iters_per_rhs[r] == is_.iterations
        assert torch.equal(xb[r * sb.N:(r + 1) * sb.N], xs)
    sb.close()
    ss.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_fgmres_mixed_preconditioner_solves_to_fp64_tolerance(dev, prec):
    """Mixed precision: FP32 (or split-BF16) fast diagonalisation inside FP64
    FGMRES reaches 1e-8 in the true FP64 residual; the solution matches the
    FP64 solve."""
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] FGMRES with {prec} preconditioner")
    E, p = 10, 3
    s64 = Solver(E, p, 1.0, iters=1, krylov="fgmres")
    s32 = Solver(E, p, 1.0, iters=1, krylov="fgmres", precision=prec)
    b = s64.build_rhs([1.0])
    x64, i64 = s64.solve(b, 1e-8)
    x32, i32 = s32.solve(b, 1e-8)
    assert i32.true_relres <= 1e-8 * 1.01 and i64.true_relres <= 1e-8 * 1.01
    nv = s64.nV
    assert abs(i32.iterations - i64.iterations) <= 2
    err = (x32[:nv] - x64[:nv]).norm() / x64[:nv].norm()
    assert err < 1e-6
    s64.close()
    s32.close()


def test_bf16x3_preconditioner(dev):
    """Split-BF16 fast diagonalisation: error vs FP64 well below FP16 levels,
    and FGMRES with it still reaches 1e-8 in the FP64 residual."""
    from paper_2311_06926_amd.solver import Solver
    say("[parity] bf16x3 P0 and FGMRES")
    E, p = 9, 3
    s64 = Solver(E, p, 1.0)
    sbf = Solver(E, p, 1.0, precision="bf16x3", krylov="fgmres", iters=1)
    x = to_gpu(synth.random_vector(s64.N, seed=502), dev)
    y64 = s64.apply_P0(x).cpu().numpy()
    ybf = sbf.apply_P0(x).cpu().numpy()
    err = rel_err(ybf, y64)
    assert 1e-9 < err < 5e-4
    xs, info = sbf.solve(sbf.build_rhs([1.0]), 1e-8)
    assert info.converged == 1 and info.true_relres <= 1e-8 * 1.01
    s64.close()
    sbf.close()


@pytest.mark.parametrize("E,p", [(4, 2), (8, 3)])
def test_autograd_adjoint_matches_oracle(dev, E, p):
    """HyperPowerSolve backward (adjoint solve + gradient kernels) against the
    oracle's dense-direct gradient (8^3 is the size the differentiable-solve
    workload is checked at)."""
    from oracle.cases import CavityLoss, cavity
    from oracle.direct import DirectSolver
    from paper_2311_06926_amd.autograd import cavity_loss
    from paper_2311_06926_amd.solver import Solver
    say(f"[parity] autograd adjoint vs oracle gradient {E}^3 p={p}")
    nu = 1.1
    St, bt = cavity(E, p, U=1.5)
    ut = DirectSolver(St).solve(bt)[:St.nV]
    ref = CavityLoss(E, p, U=1.0, u_target=ut)
    beta_np = synth.random_vector(St.nV, seed=603, scale=0.4)
    L_ref, gb_ref, gn_ref = ref.gradient(beta_np, nu)
    sol = Solver(E, p, nu, krylov="fgmres", iters=1, maxit=400)
    beta = to_gpu(beta_np, dev).requires_grad_(True)
    nu_t = torch.tensor(nu, dtype=torch.float64, device=dev, requires_grad=True)
    L = cavity_loss(beta, nu_t, sol, to_gpu(ut, dev), lid=1.0, tol=1e-12)
    L.backward()
    assert abs(L.item() - L_ref) <= 1e-9 * abs(L_ref)
    assert rel_err(beta.grad.cpu().numpy(), gb_ref) < 1e-8
    assert abs(nu_t.grad.item() - gn_ref) <= 1e-8 * abs(gn_ref)
    sol.close()
