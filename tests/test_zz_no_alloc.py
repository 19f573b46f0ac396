"""hp_solve_noalloc, the solve that allocates no device memory (its Krylov
vectors live in the library's fixed device array), against hp_solve through
the C ABI: two calls in a row, the second with a smaller input (another
context with a smaller mesh, one right-hand side, FGMRES), each equal to
hp_solve's result -- the same kernels in the same order, so the iteration
counts match and the solutions agree bit for bit -- and a solve too large
for the array refused with HP_ENOMEM before anything runs."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

HP_ENOMEM = -3


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def call(sol, name, b, x, nrhs, tol):
    from paper_2311_06926_amd._lib import hp_solve_info
    info = hp_solve_info()
    fn = getattr(sol.lib, name)
    code = fn(sol.ctx, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), nrhs,
              ctypes.c_double(tol), ctypes.byref(info))
    torch.cuda.synchronize()
    return code, info


def test_noalloc_solve_matches_hp_solve(dev):
    from paper_2311_06926_amd import synth
    from paper_2311_06926_amd.solver import Solver
    # first call: 8^3 elements, degree 3, MINRES, two right-hand sides
    say("[noalloc] 8^3 degree 3 MINRES, nrhs=2")
    sa = Solver(8, 3, 1.0, iters=1, max_rhs=2)
    modes, U = synth.body_force_modes(0, nmodes=4)
    amp, wav = synth.modes_to_arrays(modes)
    b = sa.build_rhs([1.0, U], (np.stack([np.zeros_like(amp), amp]),
                                np.stack([wav, wav])))
    xr = sa.empty(sa.N, 2)
    code_r, info_r = call(sa, "hp_solve", b, xr, 2, 1e-8)
    xn = torch.full_like(xr, float("nan"))
    code_n, info_n = call(sa, "hp_solve_noalloc", b, xn, 2, 1e-8)
    say(f"[noalloc]   hp_solve {info_r.iterations} its, noalloc {info_n.iterations} its")
    assert code_r == 0 and code_n == 0
    assert info_n.iterations == info_r.iterations and info_n.converged == 1
    assert list(info_n.iters_per_rhs[:2]) == list(info_r.iters_per_rhs[:2])
    assert info_n.true_relres == info_r.true_relres
    assert torch.equal(xn, xr)
    # second call, smaller input: 5^3 elements, degree 2, FGMRES, one rhs
    say("[noalloc] 5^3 degree 2 FGMRES, nrhs=1")
    sb = Solver(5, 2, 1.0, iters=1, krylov="fgmres", restart=20)
    b1 = sb.build_rhs([0.7])
    yr = sb.empty(sb.N)
    code_r, info_r = call(sb, "hp_solve", b1, yr, 1, 1e-9)
    yn = torch.full_like(yr, float("nan"))
    code_n, info_n = call(sb, "hp_solve_noalloc", b1, yn, 1, 1e-9)
    say(f"[noalloc]   hp_solve {info_r.iterations} its, noalloc {info_n.iterations} its")
    assert code_r == 0 and code_n == 0
    assert info_n.iterations == info_r.iterations and info_n.converged == 1
    assert torch.equal(yn, yr)
    # the first context again after the second used the array: still equal
    xn2 = torch.zeros_like(xr)
    code_n, info_n = call(sa, "hp_solve_noalloc", b, xn2, 2, 1e-8)
    assert code_n == 0 and torch.equal(xn2, xr)
    # too large for the array: 10 N max_rhs > 2^22 doubles (40^3, degree 3, N = 291,060)
    sc = Solver(40, 3, 1.0, iters=1, max_rhs=2, autotune=False)
    bc = sc.build_rhs([1.0, 1.0])
    xc = torch.zeros(2 * sc.N, dtype=torch.float64, device=dev)
    code, _ = call(sc, "hp_solve_noalloc", bc, xc, 2, 1e-8)
    assert code == HP_ENOMEM
    assert float(xc.abs().max()) == 0.0          # nothing written
    for s in (sa, sb, sc):
        s.close()
