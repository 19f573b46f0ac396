"""GPU tests of the C ABI's remaining paths: the body-force coefficient field
in hp_build_rhs, the warm start of hp_solve, the damping factor of P_0, the
set-up gate on sigma(P_0^{-1} A~) (Sec. 2, Lemma Sk_posdef and Remark
rmk:convergence_Pk), and the error paths HP_ENAN, HP_ENOTSPD and
HP_EBREAKDOWN.  Every expected outcome is predicted by the oracle (or by
exact arithmetic, stated where used) before it is asserted here.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2311_06926_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu

HP_ENOTSPD, HP_EBREAKDOWN, HP_ENAN = -4, -5, -7


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_gpu(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def damped_hyperpower(S, q, k, w):
    """The oracle's P_k built on the damped base w P_0^{-1} (both blocks)."""
    from oracle.precond import BasePreconditioner, HyperPower

    class Damped(BasePreconditioner):
        def apply_V0(self, x):
            return w * super().apply_V0(x)

        def apply_Q0(self, x):
            return w * super().apply_Q0(x)

    return HyperPower(S, q, k, base=Damped(S))


def test_rhs_with_body_force_coefficients(dev):
    """b = [F_lid + F_modes + M_V beta; 0] against the oracle (two rhs)."""
    from oracle.assemble import KronSystem
    from oracle.cases import velocity_mass
    from paper_2311_06926_amd.solver import Solver
    E, p, nu = 5, 3, 0.9
    say(f"[boundary] rhs with beta E={E} p={p}")
    S = KronSystem(E, p, nu)
    MV = velocity_mass(S)
    sol = Solver(E, p, nu, max_rhs=2)
    lids, amps, wavs, betas, refs = [], [], [], [], []
    for r in range(2):
        modes, U = synth.body_force_modes(r, nmodes=3)
        a, w = synth.modes_to_arrays(modes)
        beta = synth.random_vector(S.nV, seed=70 + r, scale=0.5)
        lids.append(U)
        amps.append(a)
        wavs.append(w)
        betas.append(beta)
        ref = S.lid_rhs(U) + S.body_force_rhs(modes)
        ref[:S.nV] += MV @ beta
        refs.append(ref)
    b = sol.build_rhs(np.array(lids), (np.stack(amps), np.stack(wavs)),
                      beta=to_gpu(np.concatenate(betas), dev)).cpu().numpy()
    assert rel_err(b, np.concatenate(refs)) < 1e-12
    # beta alone (no lid): [M_V beta; 0]
    b1 = sol.build_rhs([0.0], beta=to_gpu(betas[0], dev)).cpu().numpy()
    ref1 = np.zeros(S.N)
    ref1[:S.nV] = MV @ betas[0]
    assert rel_err(b1, ref1) < 1e-12
    sol.close()


@pytest.mark.parametrize("krylov", ["minres", "fgmres"])
def test_warm_start_matches_oracle(dev, krylov):
    """Warm start from x_0: the solve runs on r_0 = b - K x_0 with the stopping
    test still relative to b.  Oracle: the same Krylov method on r_0 from
    zero, with the tolerance rescaled by |b| / |r_0| in the method's norm
    (P_k^{-1}-norm for MINRES, 2-norm for FGMRES), then x = x_0 + d."""
    from oracle.cases import cavity
    from oracle.krylov import fgmres, minres
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    E, p, tol = 6, 3, 1e-8
    say(f"[boundary] warm start {krylov} E={E} p={p}")
    S, b = cavity(E, p)
    H = HyperPower(S, 2, 1)
    Kop = lambda v: S.K @ v  # noqa: E731
    cold = minres(Kop, H.apply, b, tol=tol)
    x0 = 0.5 * cold.x + 1e-2 * np.abs(cold.x).max() * synth.random_vector(S.N, seed=81)
    r0 = b - Kop(x0)
    if krylov == "minres":
        scale = np.sqrt(b @ H.apply(b)) / np.sqrt(r0 @ H.apply(r0))
        d = minres(Kop, H.apply, r0, tol=tol * scale)
    else:
        scale = np.linalg.norm(b) / np.linalg.norm(r0)
        d = fgmres(Kop, lambda v, j: H.apply(v), r0, tol=tol * scale, restart=50)
    x_ref = x0 + d.x
    sol = Solver(E, p, 1.0, iters=1, krylov=krylov, use_x0=True)
    x = to_gpu(x0, dev)
    _, info = sol.solve(to_gpu(b, dev), tol, x=x)
    xs = x.cpu().numpy()
    say(f"[boundary]   {info.iterations} iterations (oracle {d.iters}, cold {cold.iters}), "
        f"true relres {info.true_relres:.2e}")
    assert abs(info.iterations - d.iters) <= 1
    assert info.iterations < cold.iters
    assert info.converged == 1 and info.true_relres <= 1.01 * tol
    nV = S.nV
    assert np.linalg.norm(xs[:nV] - x_ref[:nV]) <= 1e-6 * np.linalg.norm(x_ref[:nV])
    # a start that already meets the tolerance: MINRES stops before its first
    # iteration and leaves x untouched; FGMRES takes one Arnoldi step
    xc = to_gpu(xs, dev)
    xc0 = xc.clone()
    _, info = sol.solve(to_gpu(b, dev), tol, x=xc)
    if krylov == "minres":
        assert info.iterations == 0 and torch.equal(xc, xc0)
    else:
        assert info.iterations <= 1
    assert info.converged == 1
    sol.close()


def test_damped_base_preconditioner_matches_oracle(dev):
    """p0_scale = w: every P_0^{-1} inside P_k is w P_0^{-1}, also where the
    Schur recursion forms B P_{Q,0}^{-1} s as 2 nu w D' s.  Against the
    oracle's P_k on the damped base (w = 0.8 keeps sigma in (0, 2))."""
    from oracle.assemble import KronSystem
    from paper_2311_06926_amd.solver import Solver
    E, p, w = 5, 3, 0.8
    say(f"[boundary] damped P_0, w={w}")
    S = KronSystem(E, p, 1.0)
    sol = Solver(E, p, 1.0, p0_scale=w)
    x = synth.random_vector(S.N, seed=91)
    for q, k in ((2, 0), (2, 1), (2, 2), (3, 1)):
        y = sol.apply_hyperpower(q, k, to_gpu(x, dev)).cpu().numpy()
        gap = rel_err(y, damped_hyperpower(S, q, k, w).apply(x))
        say(f"[boundary]   q={q} k={k}: gap {gap:.2e}")
        assert gap < 1e-12
    sol.close()


def test_spectrum_gate_and_indefinite_preconditioner(dev):
    """w = 1.5 lifts the largest eigenvalue of w P_{V,0}^{-1} A above 2 (the
    oracle's dense spectrum in test_damped_base_leaves_the_convergence_interval
    predicts it at this mesh): the set-up gate refuses the context
    (HP_ENOTSPD); without the gate, MINRES with P_1 meets r' P_1^{-1} r < 0
    (HP_ENOTSPD, as the oracle's MINRES does), while MINRES with P_0 alone
    is unaffected: scaling the preconditioner by a constant leaves the
    MINRES iterates unchanged (same Krylov space, same minimisation)."""
    from oracle.cases import cavity
    from oracle.krylov import minres
    from paper_2311_06926_amd._lib import HPError
    from paper_2311_06926_amd.solver import Solver
    E, p, w = 4, 3, 1.5
    say(f"[boundary] spectrum gate E={E} p={p} w={w}")
    S, b = cavity(E, p)
    with pytest.raises(FloatingPointError):
        minres(lambda v: S.K @ v, damped_hyperpower(S, 2, 1, w).apply, b, tol=1e-8)
    Solver(E, p, 1.0, spectrum_gate=30).close()               # plain P_0 passes
    with pytest.raises(HPError) as e:
        Solver(E, p, 1.0, p0_scale=w, spectrum_gate=30)
    assert e.value.code == HP_ENOTSPD
    sol = Solver(E, p, 1.0, p0_scale=w, iters=1)
    bg = to_gpu(b, dev)
    with pytest.raises(HPError) as e:
        sol.solve(bg, 1e-8)
    assert e.value.code == HP_ENOTSPD
    sol.close()
    s0 = Solver(E, p, 1.0, p0_scale=w, iters=0)
    s1 = Solver(E, p, 1.0, iters=0)
    x0, i0 = s0.solve(bg, 1e-8)
    x1, i1 = s1.solve(bg, 1e-8)
    assert i0.iterations == i1.iterations
    assert float((x0 - x1).norm() / x1.norm()) < 1e-10
    s0.close()
    s1.close()


@pytest.mark.parametrize("krylov", ["minres", "fgmres"])
def test_nan_in_rhs_or_start_gives_enan(dev, krylov):
    """A NaN (or Inf) in b, or in x_0 for a warm start, is reported as
    HP_ENAN (the oracle's MINRES rejects the same right-hand side)."""
    from oracle.cases import cavity
    from oracle.krylov import minres
    from oracle.precond import HyperPower
    from paper_2311_06926_amd._lib import HPError
    from paper_2311_06926_amd.solver import Solver
    E, p = 4, 2
    say(f"[boundary] NaN -> HP_ENAN ({krylov})")
    S, b = cavity(E, p)
    bad = b.copy()
    bad[S.nV // 2] = np.nan
    with pytest.raises(FloatingPointError):
        minres(lambda v: S.K @ v, HyperPower(S, 2, 1).apply, bad, tol=1e-8)
    sol = Solver(E, p, 1.0, iters=1, krylov=krylov, maxit=50)
    for v in (np.nan, np.inf):
        bb = b.copy()
        bb[S.nV // 2] = v
        with pytest.raises(HPError) as e:
            sol.solve(to_gpu(bb, dev), 1e-8)
        assert e.value.code == HP_ENAN, v
    sol.close()
    warm = Solver(E, p, 1.0, iters=1, krylov=krylov, maxit=50, use_x0=True)
    x0 = np.zeros(S.N)
    x0[3] = np.nan
    with pytest.raises(HPError) as e:
        warm.solve(to_gpu(b, dev), 1e-8, x=to_gpu(x0, dev))
    assert e.value.code == HP_ENAN
    warm.close()


@pytest.mark.parametrize("krylov", ["minres", "fgmres"])
def test_breakdown_threshold(dev, krylov):
    """breakdown_tol >= 1 forces the breakdown test at the first iteration
    (the rotated pivot never exceeds the sum of, or the 2-norm of, its
    column's entries), so the solve stops with HP_EBREAKDOWN after one
    iteration at most; a tiny positive threshold changes nothing."""
    from paper_2311_06926_amd._lib import HPError
    from paper_2311_06926_amd.solver import Solver
    E, p = 4, 3
    say(f"[boundary] breakdown threshold ({krylov})")
    ref = Solver(E, p, 1.0, iters=1, krylov=krylov)
    b = ref.build_rhs([1.0])
    xr, ir = ref.solve(b, 1e-8)
    tiny = Solver(E, p, 1.0, iters=1, krylov=krylov, breakdown_tol=1e-300)
    xt, it = tiny.solve(b, 1e-8)
    assert it.iterations == ir.iterations and torch.equal(xt, xr)
    forced = Solver(E, p, 1.0, iters=1, krylov=krylov, breakdown_tol=1.0)
    with pytest.raises(HPError) as e:
        forced.solve(b, 1e-8)
    assert e.value.code == HP_EBREAKDOWN
    for s in (ref, tiny, forced):
        s.close()


@pytest.mark.parametrize("q,k", [(2, 0), (2, 2), (3, 1)])
def test_velocity_block_alone_matches_oracle(dev, q, k):
    """hp_apply_PV (eq. Pcv, the operator of the Sec. 5.1 cost study) against
    the oracle's literal recursion, and equal bit for bit to the velocity
    part of hp_apply_hyperpower (the same launch sequence)."""
    from oracle.assemble import KronSystem
    from oracle.precond import HyperPower
    from paper_2311_06926_amd.solver import Solver
    E, p = 7, 3
    say(f"[boundary] P_V,k alone q={q} k={k}")
    S = KronSystem(E, p, 1.0)
    sol = Solver(E, p, 1.0, max_rhs=2)
    x = synth.random_vector(S.N, seed=171)
    u = np.ascontiguousarray(x[:S.nV])
    yv = sol.apply_PV(q, k, to_gpu(u, dev)).cpu().numpy()
    ref = HyperPower(S, q, k).apply_V(k, u)
    assert rel_err(yv, ref) < 1e-12
    yfull = sol.apply_hyperpower(q, k, to_gpu(x, dev)).cpu().numpy()
    assert np.array_equal(yv, yfull[:S.nV])
    ub = np.concatenate([u, 0.5 * u])
    yb = sol.apply_PV(q, k, to_gpu(ub, dev)).cpu().numpy()
    assert np.array_equal(yb[:S.nV], yv)
    sol.close()
