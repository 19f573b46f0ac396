"""Lanczos spectra of the preconditioned blocks on the GPU (hp_spectrum)
against the oracle (Sec. 2 Lemma Sk_posdef / Corollary cor:Skform; the
spectra of Sec. 5.2).

* Same start vector on both sides: the first Lanczos coefficients agree
  entry by entry (the tridiagonal matrix is a smooth function of the
  operators, so FP64 rounding differences stay near 1e-12 for a few
  steps), for the velocity block with P_{V,k} and the Schur block with
  eq. Pcq1 and eq. Pcq2 at a fixed P_{V,l}.
* The worked example (2^3 elements, degree 4): run to the block dimension,
  the extremes equal those of the oracle's dense spectra, for P_{V,k}^{-1} A
  and for P_{Q,k}^{-1} S with S = B' A^{-1} B taken as B' P_{V,6}^{-1} B on
  the GPU (|1 - lambda|^(2^6) < 1e-20 there); eq. Pcq_exact is eq. Pcq2
  with that fixed P_{V,6}.
* Corollary cor:Skform at 16^3: the extremes measured with P_{V,k} are the
  image of those measured with P_{V,0}.
* The headline mesh (32^3, degree 3): both blocks inside (0, 2).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2311_06926_amd import synth  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


CASES = [("velocity", "Pcq1", 0, 0), ("velocity", "Pcq1", 2, 0), ("schur", "Pcq1", 0, 0),
         ("schur", "Pcq1", 2, 1), ("schur", "Pcq2", 2, 2)]


@pytest.mark.parametrize("block,var,k,sl", CASES)
def test_lanczos_coefficients_match_oracle(dev, block, var, k, sl):
    from oracle.assemble import KronSystem
    from oracle.precond import HyperPower
    from oracle.spectra import schur_lanczos, velocity_lanczos
    from paper_2311_06926_amd.solver import Solver
    E, p, nu, steps = 4, 3, 0.8, 10
    say(f"[spectra] coefficients E={E} p={p} {block} {var} k={k} l={sl}")
    S = KronSystem(E, p, nu)
    fixed = sl if var == "Pcq2" else 0
    H = HyperPower(S, 2, 0, variant=var, fixed_level=fixed)
    sol = Solver(E, p, nu, schur=var, schur_level=fixed)
    n = S.nV if block == "velocity" else S.nQ
    x0 = synth.random_vector(n, seed=7)
    if block == "velocity":
        al, be = velocity_lanczos(H, k, x0, steps)
    else:
        al, be = schur_lanczos(H, k, sl, x0, steps)
    g = sol.spectrum(block, 2, k, sl, steps, start=torch.from_numpy(x0).to(dev))
    assert g["steps"] == steps
    scale = np.abs(al).max()
    assert np.abs(g["alpha"] - al).max() <= 1e-9 * scale
    assert np.abs(g["beta"][:steps - 1] - be).max() <= 1e-9 * scale
    sol.close()


# After k >= 2 updates most eigenvalues lie within 1e-8 of 1; the process
# stops at an invariant subspace to 1e-10 relative before it separates them,
# so an extreme Ritz value in that cluster is accurate to a few 1e-8.
TOL = 1e-7


def test_worked_example_spectra(dev):
    from oracle.assemble import KronSystem
    from oracle.precond import BasePreconditioner, HyperPower
    from oracle.spectra import dense_sequence_spectrum
    from paper_2311_06926_amd.solver import Solver
    E, p = 2, 4
    S = KronSystem(E, p, 1.0)
    P0 = BasePreconditioner(S)
    sol = {v: Solver(E, p, 1.0, schur=v, schur_level=6 if v == "Pcq2" else 0)
           for v in ("Pcq1", "Pcq2")}
    H = HyperPower(S, 2, 0, base=P0)
    for k in range(4):
        say(f"[spectra] 2^3 p=4 velocity k={k}")
        ev = dense_sequence_spectrum(H, "V", k)
        g = sol["Pcq1"].spectrum("velocity", 2, k, 0, S.nV, seed=k)
        assert abs(g["lmin"] - ev[0]) < TOL and abs(g["lmax"] - ev[-1]) < TOL
        if k == 0:
            assert abs(g["lmin"] - 0.71) < 0.02 and abs(g["lmax"] - 1.41) < 0.02
    for var, ovar in (("Pcq1", "Pcq1"), ("Pcq2", "Pcq_exact")):
        Hq = HyperPower(S, 2, 0, variant=ovar, base=P0)
        for k in range(4):
            say(f"[spectra] 2^3 p=4 schur {ovar} k={k}")
            ev = dense_sequence_spectrum(Hq, "Q", k)
            g = sol[var].spectrum("schur", 2, k, 6, S.nQ, seed=10 + k)
            assert abs(g["lmin"] - ev[0]) < TOL and abs(g["lmax"] - ev[-1]) < TOL, (var, k)
    for s in sol.values():
        s.close()


def test_corollary_predicts_the_updated_spectrum(dev):
    from paper_2311_06926_amd.solver import Solver
    from paper_2311_06926_amd.spectra import hyperpower_interval
    E, p = 16, 3
    sol = Solver(E, p, 1.0)
    g0 = sol.spectrum("velocity", 2, 0, 0, 120, seed=1)
    say(f"[spectra] 16^3 p=3 velocity k=0: [{g0['lmin']:.6f}, {g0['lmax']:.6f}]")
    assert 0 < g0["lmin"] < 1 < g0["lmax"] < 2
    for q, k in ((2, 1), (2, 2), (3, 1)):
        lo, hi = hyperpower_interval(g0["lmin"], g0["lmax"], q, k)
        g = sol.spectrum("velocity", q, k, 0, 120, seed=2)
        say(f"[spectra]   q={q} k={k}: measured [{g['lmin']:.6f}, {g['lmax']:.6f}] "
            f"predicted [{lo:.6f}, {hi:.6f}]")
        assert abs(g["lmin"] - lo) < 1e-6
        assert g["lmax"] <= hi + 1e-9 and g["lmax"] > hi - 1e-3
    sol.close()


def test_headline_mesh_spectra_in_range(dev):
    from paper_2311_06926_amd.solver import Solver
    sol = Solver(32, 3, 1.0)
    gv = sol.spectrum("velocity", 2, 0, 0, 60)
    gs = sol.spectrum("schur", 2, 0, 0, 60)
    say(f"[spectra] 32^3 p=3: velocity [{gv['lmin']:.4f}, {gv['lmax']:.4f}], "
        f"schur [{gs['lmin']:.4f}, {gs['lmax']:.4f}]")
    assert 0 < gv["lmin"] < 1 < gv["lmax"] < 2
    assert 0 < gs["lmin"] < gs["lmax"] < 2
    sol.close()
