"""GPU checks at the benchmark sizes and of the launch-shape choices.

* Full-size parity: apply_K on the 32^3 and 192^3 (p = 3) meshes in the
  launch configuration the benchmark times (autotuned shapes), checked on
  sampled entries that the oracle evaluates one by one (``KronRows``: a row
  of a Kronecker product is the outer product of the factors' rows), with
  every block's first and last entries among the samples.  Tolerance 1e-12
  relative to max |K x|, as for the small meshes.
* P_0 at 32^3 and at 96^3 (the differentiable-solve mesh, seven MFMA
  tiles per direction, with the 2x2-tile plan the tuner picks there and
  with every other plan that fits): the normwise backward error of each
  velocity block, |A_cc y_c - x_c|_i / (|A_cc| |y_c| + |x_c|), and of the
  pressure block, M_q y_p = 2 nu x_p, on sampled rows (|A_cc| |y_c| from
  the oracle's rows of the factors in absolute value), at most 1e-14.
* The MINRES sweep of the headline mesh (32^3, degree 3, q in {2, 3},
  k in {0..3}, eq. Pcq1): iteration counts within +-1 of the oracle's and
  the solution on sampled velocity entries within 1e-10 (tests/golden/,
  written by a script that calls only the oracle).
* P_1 at 32^3 through its definition with the separately checked operators.
* The solve at 32^3 (q = 2, k = 1, MINRES): the oracle's lid right-hand side
  in, and on sampled rows |b - K x|_i <= ||b - K x||_2 <= tol ||b||_2.
* The single-pass operator kernel against the two-kernel path and the oracle.
* Launch shapes: every i3-chunk length and workgroup order, and every P_0
  plan that fits, gives the same result (bit for bit for the operators,
  whose per-point arithmetic does not depend on the shape; within the P_0
  tolerance for the plans); the autotuner reports shapes in range.
* The mixed-precision solve at 64^3 and the batched solve at 48^3 x 32: residual
  rows against the oracle's rows of K.
* The differentiable solve at 96^3 (FP32 P_k in FP64 FGMRES): adjoint
  gradients against central differences with step 1e-6.
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


def samples(offsets, n_random, seed):
    """Random indices plus the first and last three entries of each block."""
    rng = np.random.default_rng(seed)
    idx = [rng.integers(0, offsets[-1], n_random)]
    for b in range(len(offsets) - 1):
        lo, hi = offsets[b], offsets[b + 1]
        idx.append(np.arange(lo, min(lo + 3, hi)))
        idx.append(np.arange(max(hi - 3, lo), hi))
    return np.unique(np.concatenate(idx))


@pytest.mark.parametrize("E", [32, 192])
def test_apply_K_full_size_sampled(dev, E):
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    p, nu = 3, 1.0
    say(f"[fullsize] apply_K E={E} p={p}")
    R = KronRows(E, p, nu)
    sol = Solver(E, p, nu)
    assert sol.N == R.N
    x = synth.random_vector(R.N, seed=3)
    y = sol.apply_K(torch.from_numpy(x).to(dev)).cpu().numpy()
    idx = samples(R.offsets, 3000 if E == 32 else 1500, seed=E)
    ref = R.rows(x, idx)
    scale = np.abs(y).max()
    err = np.abs(y[idx] - ref).max() / scale
    say(f"[fullsize]   {idx.size} samples, max rel err {err:.2e}, tuning {sol.tuning(1)}")
    assert err < 1e-12
    sol.close()


def test_apply_K_quad_full_size(dev):
    """The quadrature-based operator at 32^3, degree 3 (about 2.2 M points):
    sampled rows against the oracle, the whole vector against apply_K."""
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    E, p, nu = 32, 3, 1.0
    say(f"[fullsize] apply_K_quad E={E} p={p}")
    R = KronRows(E, p, nu)
    sol = Solver(E, p, nu)
    x = torch.from_numpy(synth.random_vector(R.N, seed=4)).to(dev)
    yq = sol.apply_K_quad(x).cpu().numpy()
    yk = sol.apply_K(x).cpu().numpy()
    idx = samples(R.offsets, 3000, seed=7)
    ref = R.rows(x.cpu().numpy(), idx)
    scale = np.abs(yq).max()
    err = np.abs(yq[idx] - ref).max() / scale
    gap = np.abs(yq - yk).max() / scale
    say(f"[fullsize]   {idx.size} samples, max rel err {err:.2e}; vs apply_K {gap:.2e}")
    assert err < 1e-12 and gap < 1e-12
    sol.close()


def p0_backward_errors(R, x, y, nu, nsamp, seed):
    """Sampled normwise backward errors of P_0's blocks: per velocity block
    max_i |A_cc y - x|_i / (max_i (|A_cc| |y|)_i + |x|_inf), and for the
    pressure |M_q y - 2 nu x|_i / (max_i (M_q |y|)_i + 2 nu |x|_inf)."""
    o = R.offsets
    rng = np.random.default_rng(seed)
    out = []
    for c in range(4):
        n = o[c + 1] - o[c]
        loc = np.unique(np.concatenate([rng.integers(0, n, nsamp), [0, n - 1]]))
        yc, xc = y[o[c]:o[c + 1]], x[o[c]:o[c + 1]]
        terms = R.terms[c, c] if c < 3 else R.mq_terms
        absterms = [(abs(a), np.abs(A3), np.abs(A2), np.abs(A1)) for a, A3, A2, A1 in terms]
        rhs = xc[loc] if c < 3 else 2.0 * nu * xc[loc]
        r = R.block_entries(c, c, yc, loc, terms=terms) - rhs
        scale = R.block_entries(c, c, np.abs(yc), loc, terms=absterms).max()
        scale += np.abs(xc).max() * (1.0 if c < 3 else 2.0 * nu)
        out.append(np.abs(r).max() / scale)
    return out


def test_P0_full_size_backward_error(dev):
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    E, p, nu = 32, 3, 0.7
    say(f"[fullsize] P0 E={E} p={p}")
    R = KronRows(E, p, nu)
    sol = Solver(E, p, nu)
    x = synth.random_vector(R.N, seed=11)
    y = sol.apply_P0(torch.from_numpy(x).to(dev)).cpu().numpy()
    eta = p0_backward_errors(R, x, y, nu, 800, seed=5)
    say(f"[fullsize]   backward errors {['%.1e' % e for e in eta]}, tuning {sol.tuning(1)}")
    assert max(eta) <= 1e-14
    sol.close()


def test_P0_96_every_plan_backward_error(dev):
    """P_0 at 96^3, degree 3 (nN = 97, nM = 98: seven 16-wide MFMA tiles per
    direction, the last ragged) in FP64 with every plan that fits, among
    them the 2x2-tile plan the tuner picks at this size: sampled backward
    errors <= 1e-14; the 16-wave plans and the row-block plan 9 agree with
    each other bit for bit (same contraction order per output), the 4-wave
    plans likewise."""
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    E, p, nu = 96, 3, 1.1
    say(f"[fullsize] P0 plans E={E} p={p}")
    R = KronRows(E, p, nu)
    x = synth.random_vector(R.N, seed=96)
    xg = torch.from_numpy(x).to(dev)
    wide, narrow = None, None
    tuned = Solver(E, p, nu)
    say(f"[fullsize]   tuned plans {tuned.tuning(1)['fd_plan']}")
    yt = tuned.apply_P0(xg)
    tuned.close()
    for plan in list(range(8)) + [9]:
        s = Solver(E, p, nu, autotune=False, fd_plan=plan)
        if s.tuning(1)["fd_plan"][0] != plan:
            s.close()
            continue
        yg = s.apply_P0(xg)
        s.close()
        if plan & 1:
            if wide is None:
                wide = yg
            assert torch.equal(yg, wide), plan
        else:
            if narrow is None:
                narrow = yg
            assert torch.equal(yg, narrow), plan
        eta = p0_backward_errors(R, x, yg.cpu().numpy(), nu, 300, seed=plan)
        say(f"[fullsize]   plan {plan}: backward errors {['%.1e' % e for e in eta]}")
        assert max(eta) <= 1e-14, plan
    assert wide is not None
    assert torch.equal(yt, wide) or (narrow is not None and torch.equal(yt, narrow))


def golden_sweep(name="minres_oracle_32cube_p3.txt"):
    """The oracle's MINRES reference data for the headline mesh."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows, idx, N = {}, None, None
    for line in open(path):
        if line.startswith("# N "):
            N = int(line.split()[2])
        elif line.startswith("# sample_indices"):
            idx = np.array([int(t) for t in line.split()[2:]])
        elif line.strip() and not line.startswith("#"):
            v = line.split()
            rows[(int(v[0]), int(v[1]))] = (int(v[2]), float(v[3]), float(v[4]),
                                            np.array([float(t) for t in v[5:]]))
    return N, idx, rows


SWEEP = [(2, 0), (2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)]


@pytest.mark.parametrize("q,k", SWEEP)
def test_headline_sweep_matches_oracle(dev, q, k):
    """The benchmark's sweep at 32^3, degree 3 (MINRES to 1e-8, eq. Pcq1,
    literal schedule): iteration count within +-1 of the oracle's, the true
    residual below the tolerance, and the solution on the oracle's sampled
    velocity entries within 1e-10 of the oracle's (relative to their max)."""
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    E, p, tol = 32, 3, 1e-8
    N, idx, rows = golden_sweep()
    its_ref, res_ref, _, xs_ref = rows[(q, k)]
    say(f"[fullsize] headline sweep q={q} k={k} (oracle {its_ref} iterations)")
    R = KronRows(E, p, 1.0)
    assert R.N == N
    sol = Solver(E, p, 1.0, order=q, iters=k)
    xg, info = sol.solve(torch.from_numpy(R.lid_rhs(1.0)).to(dev), tol)
    x = xg.cpu().numpy()
    say(f"[fullsize]   GPU {info.iterations} iterations, true relres {info.true_relres:.2e} "
        f"(oracle {res_ref:.2e})")
    assert abs(info.iterations - its_ref) <= 1
    assert info.converged == 1 and info.true_relres <= 1.01 * tol
    vel = idx < sol.nV
    gap = np.abs(x[idx][vel] - xs_ref[vel]).max() / np.abs(xs_ref[vel]).max()
    say(f"[fullsize]   sampled velocity gap {gap:.2e}")
    # the same recurrences in the same order: the iterates agree to rounding
    # (measured 1e-14 .. 3e-14)
    assert gap <= 1e-10
    sol.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_P0_above_the_tile_cap(dev, prec):
    """130^3 elements, degree 2 (nM = 131: beyond the 128 a direction of the
    in-LDS kernels holds), so P_0 runs as mode-product GEMMs: sampled
    backward errors <= 1e-14 in FP64, and the FP32 products within 1e-5."""
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    E, p, nu = 130, 2, 0.9
    say(f"[fullsize] P0 above the tile cap E={E} p={p} {prec}")
    R = KronRows(E, p, nu)
    s64 = Solver(E, p, nu, autotune=False)
    assert s64.tuning(1)["fd_plan"][0] == 8
    x = synth.random_vector(R.N, seed=130)
    xg = torch.from_numpy(x).to(dev)
    y = s64.apply_P0(xg)
    if prec == "fp64":
        eta = p0_backward_errors(R, x, y.cpu().numpy(), nu, 200, seed=130)
        say(f"[fullsize]   backward errors {['%.1e' % e for e in eta]}")
        assert max(eta) <= 1e-14
    else:
        s32 = Solver(E, p, nu, autotune=False, precision="fp32", krylov="fgmres")
        y32 = s32.apply_P0(xg)
        gap = float((y32 - y).abs().max() / y.abs().max())
        say(f"[fullsize]   FP32 vs FP64 {gap:.2e}")
        assert gap < 1e-5
        s32.close()
    s64.close()


def test_solve_above_the_tile_cap(dev):
    """MINRES with P_1 at 130^3 elements, degree 2 (N = 8.9 M): converged to
    1e-8 with the true residual below the tolerance, and on sampled rows
    |b - K x|_i <= tol ||b||_2 with the oracle's rows of K."""
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    E, p, tol = 130, 2, 1e-8
    say(f"[fullsize] solve above the tile cap E={E} p={p}")
    R = KronRows(E, p, 1.0)
    b = R.lid_rhs(1.0)
    sol = Solver(E, p, 1.0, iters=1)
    xg, info = sol.solve(torch.from_numpy(b).to(dev), tol)
    say(f"[fullsize]   {info.iterations} iterations, true relres {info.true_relres:.2e}, "
        f"{info.seconds * 1e3:.1f} ms")
    assert info.converged and info.true_relres <= 1.01 * tol
    x = xg.cpu().numpy()
    idx = samples(R.offsets, 600, seed=131)
    r = b[idx] - R.rows(x, idx)
    assert np.abs(r).max() <= 1.01 * tol * np.linalg.norm(b)
    sol.close()


def test_hyperpower_full_size_composition(dev):
    """P_1 (q = 2, eq. Pcq1) at 32^3, degree 3, in the benchmark's launch
    configuration, checked through its definition with the separately
    verified operators (apply_A/B/Bt against the oracle's rows, P_0 by its
    backward error): velocity y = X0 (2x - A X0 x), pressure
    y = Q0 (2x - B' X0 B Q0 x) with X0 = P_{V,0}^{-1}, Q0 = P_{Q,0}^{-1}."""
    from paper_2311_06926_amd.solver import Solver
    E, p = 32, 3
    say(f"[fullsize] P_1 composition E={E} p={p}")
    sol = Solver(E, p, 1.0)
    nV, N = sol.nV, sol.N
    x = torch.from_numpy(synth.random_vector(N, seed=17)).to(dev)
    y = sol.apply_hyperpower(2, 1, x)

    def P0(v):
        return sol.apply_P0(v)

    def vel(v):
        full = torch.zeros(N, dtype=torch.float64, device=dev)
        full[:nV] = v
        return P0(full)[:nV]

    def pres(q):
        full = torch.zeros(N, dtype=torch.float64, device=dev)
        full[nV:] = q
        return P0(full)[nV:]

    xv, xq = x[:nV].contiguous(), x[nV:].contiguous()
    y0 = vel(xv)
    yv = vel(2 * xv - sol.apply_A(y0))
    t = pres(xq)
    yq = pres(2 * xq - sol.apply_Bt(vel(sol.apply_B(t))))
    ev = float((y[:nV] - yv).abs().max() / yv.abs().max())
    eq = float((y[nV:] - yq).abs().max() / yq.abs().max())
    say(f"[fullsize]   velocity {ev:.2e}, pressure {eq:.2e}")
    assert ev < 1e-12 and eq < 1e-12
    sol.close()


def test_solve_full_size_residual_on_samples(dev):
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    E, p, tol = 32, 3, 1e-8
    say(f"[fullsize] solve E={E} p={p} q=2 k=1 MINRES")
    R = KronRows(E, p, 1.0)
    b = R.lid_rhs(1.0)
    sol = Solver(E, p, 1.0, order=2, iters=1)
    xg, info = sol.solve(torch.from_numpy(b).to(dev), tol)
    x = xg.cpu().numpy()
    say(f"[fullsize]   {info.iterations} iterations, true relres {info.true_relres:.2e}")
    assert info.converged and info.true_relres <= tol
    idx = samples(R.offsets, 3000, seed=9)
    r = b[idx] - R.rows(x, idx)
    assert np.abs(r).max() <= 1.01 * tol * np.linalg.norm(b)
    sol.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_mixed_precision_solve_full_size(dev, prec):
    """The mixed-precision workload (64^3, degree 3, FGMRES(50) in FP64 with
    P_1 in FP32 or split BF16): the oracle's lid right-hand side in, and on
    sampled rows |b - K x|_i <= tol ||b||_2 with the oracle's rows of K."""
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    E, p, tol = 64, 3, 1e-8
    say(f"[fullsize] mixed-precision solve E={E} p={p} {prec}")
    R = KronRows(E, p, 1.0)
    b = R.lid_rhs(1.0)
    sol = Solver(E, p, 1.0, krylov="fgmres", precision=prec, iters=1)
    xg, info = sol.solve(torch.from_numpy(b).to(dev), tol)
    x = xg.cpu().numpy()
    say(f"[fullsize]   {info.iterations} iterations, true relres {info.true_relres:.2e}")
    assert info.converged and info.true_relres <= 1.01 * tol
    idx = samples(R.offsets, 2000, seed=64)
    r = b[idx] - R.rows(x, idx)
    assert np.abs(r).max() <= 1.01 * tol * np.linalg.norm(b)
    sol.close()


def test_batched_solve_full_size(dev):
    """The batched workload (48^3, degree 2, 32 seeded right-hand sides, one
    FGMRES with P_1 in FP32): for four of the systems, sampled rows of
    b_r - K x_r against the oracle's rows of K."""
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    E, p, nr, tol = 48, 2, 32, 1e-8
    say(f"[fullsize] batched solve E={E} p={p} nrhs={nr}")
    lids, amps, wavs = [], [], []
    for r in range(nr):
        modes, U = synth.body_force_modes(r)
        a, w = synth.modes_to_arrays(modes)
        lids.append(U)
        amps.append(a)
        wavs.append(w)
    sol = Solver(E, p, 1.0, krylov="fgmres", precision="fp32", iters=1, max_rhs=nr)
    bg = sol.build_rhs(np.array(lids), (np.stack(amps), np.stack(wavs)))
    xg, info = sol.solve(bg, tol)
    say(f"[fullsize]   {info.iterations} iterations, true relres {info.true_relres:.2e}")
    assert info.converged and info.true_relres <= 1.01 * tol
    R = KronRows(E, p, 1.0)
    b = bg.cpu().numpy().reshape(nr, sol.N)
    x = xg.cpu().numpy().reshape(nr, sol.N)
    for r in (0, 7, 19, 31):
        idx = samples(R.offsets, 800, seed=100 + r)
        res = b[r, idx] - R.rows(x[r], idx)
        assert np.abs(res).max() <= 1.01 * tol * np.linalg.norm(b[r]), r
    sol.close()


@pytest.mark.parametrize("E,p", [(8, 3), (15, 3), (5, 2), (4, 4), (20, 3), (19, 2)])
def test_operator_shapes_agree_bitwise(dev, E, p):
    from paper_2311_06926_amd.solver import Solver
    say(f"[shapes] operators E={E} p={p}")
    nu = 1.3
    base = Solver(E, p, nu, autotune=False, max_rhs=2)
    x = torch.from_numpy(synth.random_vector(2 * base.N, seed=E + p)).to(dev)
    u = x[:base.nV].contiguous()
    q = x[base.N:base.N + base.nQ].contiguous()

    def run(s):
        return [s.apply_K(x), s.apply_K(x[:s.N].contiguous()), s.apply_A(u), s.apply_B(q),
                s.apply_Bt(u), s.apply_MV(u), s.apply_hyperpower(2, 1, x[:s.N].contiguous())]

    ref = run(base)
    nM = E + p - 1
    shapes = [(kc, order, slabs, 0) for kc in sorted({1, 2, 5, nM}) for order in (0, 1)
              for slabs in (1, 3)]
    # the all-planes kernels (K and A; chunks 2, 4, 8, degree <= 4, 8 only to 3); other
    # chunks requested with op_staged=1 must fall back to the streaming kernels
    def has_staged(kc):
        return kc in (2, 4, 8) and p <= 4 and (kc < 8 or p <= 3)

    shapes += [(kc, order, slabs, 1) for kc in (2, 3, 4, 5, 8, 18, 20, 36, 52)
               for order in (0, 1) for slabs in (1, 3)]
    for kc, order, slabs, staged in shapes:
        s = Solver(E, p, nu, autotune=False, max_rhs=2, op_kchunk=kc, op_order=order,
                   op_slabs=slabs, op_staged=staged)
        t = s.tuning(1)
        kk = min(kc, nM)
        assert t["op_kchunk"] == kk and t["op_order"] == order and t["op_slabs"] == slabs
        assert t["op_staged"] == (1 if staged and has_staged(kk) else 0), (kc, t)
        for a, b in zip(run(s), ref):
            assert torch.equal(a, b), (kc, order, slabs, staged)
        s.close()
    # the streaming velocity kernel with register staging (op_dma = 0) against
    # the default direct-to-LDS staging
    for kc in sorted({1, 5, nM}):
        s = Solver(E, p, nu, autotune=False, max_rhs=2, op_kchunk=kc, op_order=1, op_slabs=1,
                   op_staged=0, op_dma=0)
        for a, b in zip(run(s), ref):
            assert torch.equal(a, b), (kc, "op_dma=0")
        s.close()
    # the streaming pressure kernel on 32 x 8 tiles against 16 x 8
    for kc, slabs in ((1, 1), (5, 3), (nM, 1)):
        s = Solver(E, p, nu, autotune=False, max_rhs=2, op_kchunk=kc, op_order=0,
                   op_slabs=slabs, op_staged=0, op_pres_wide=1)
        assert s.tuning(1)["op_pres_wide"] == 1
        for a, b in zip(run(s), ref):
            assert torch.equal(a, b), (kc, slabs, "op_pres_wide=1")
        s.close()
    base.close()


@pytest.mark.parametrize("E,p", [(4, 5), (3, 6), (5, 7), (3, 8)])
def test_direct_to_lds_velocity_kernel_high_degree(dev, E, p):
    """Degrees 5-8 (the streaming kernels only): the velocity kernel staging
    through direct-to-LDS loads (op_dma = 1, the default) against register
    staging (op_dma = 0), bit for bit, for K, A and M_V at two i3-chunk
    lengths."""
    from paper_2311_06926_amd.solver import Solver
    say(f"[shapes] direct-to-LDS velocity kernel E={E} p={p}")
    for kc in (1, 3):
        a = Solver(E, p, 1.1, autotune=False, op_kchunk=kc, op_staged=0, op_dma=1)
        b = Solver(E, p, 1.1, autotune=False, op_kchunk=kc, op_staged=0, op_dma=0)
        x = torch.from_numpy(synth.random_vector(a.N, seed=E * p + kc)).to(dev)
        u = x[:a.nV].contiguous()
        assert torch.equal(a.apply_K(x), b.apply_K(x)), kc
        assert torch.equal(a.apply_A(u), b.apply_A(u)), kc
        assert torch.equal(a.apply_MV(u), b.apply_MV(u)), kc
        a.close()
        b.close()


@pytest.mark.parametrize("E,p", [(3, 2), (8, 3), (13, 2), (4, 4), (33, 3)])
def test_single_pass_operator_matches(dev, E, p):
    """The single-pass kernel (op_fused=1: D_c^T M_q z applied as a Kronecker
    product, no w) against the two-kernel path and, at the small meshes, the
    oracle: K, A, the A-residual of P_1, single and batched."""
    from paper_2311_06926_amd.solver import Solver
    say(f"[shapes] single-pass operator E={E} p={p}")
    nu = 0.7
    two = Solver(E, p, nu, autotune=False, op_fused=0, max_rhs=2)
    one = Solver(E, p, nu, autotune=False, op_fused=1, max_rhs=2)
    for nr in (1, 2):
        x = torch.from_numpy(synth.random_vector(nr * two.N, seed=E + p + nr)).to(dev)
        u = torch.from_numpy(synth.random_vector(nr * two.nV, seed=5 + E)).to(dev)
        for a, b in ((two.apply_K(x), one.apply_K(x)), (two.apply_A(u), one.apply_A(u)),
                     (two.apply_hyperpower(2, 1, x), one.apply_hyperpower(2, 1, x))):
            assert float((a - b).abs().max() / a.abs().max()) < 1e-14
    if E <= 13:
        from oracle.assemble import KronSystem
        S = KronSystem(E, p, nu)
        xh = synth.random_vector(S.N, seed=7)
        y = one.apply_K(torch.from_numpy(xh).to(dev)).cpu().numpy()
        ref = S.K @ xh
        assert np.abs(y - ref).max() / np.abs(ref).max() < 1e-12
    two.close()
    one.close()


@pytest.mark.parametrize("E,p", [(8, 3), (13, 2), (4, 4), (30, 3), (45, 3)])
def test_fd_plans_agree(dev, E, p):
    """Every P_0 plan that fits, FP64 against the oracle's sparse LU and FP32
    within 1e-5 of it; at 30^3 (two MFMA tiles per direction) and 45^3
    (three, an odd count, so the 2x2-tile plan has a partial block) the
    second row and column tiles of every plan run.  Plans of the same
    kernel family (16-wave and the row-block plan 9: odd codes; 4-wave: even
    codes) give the same result bit for bit in each precision; plan 8 (the
    mode products as batched GEMMs over HBM, the path for directions longer
    than 128) is checked the same way."""
    from oracle.assemble import KronRows
    from paper_2311_06926_amd.solver import Solver
    say(f"[shapes] P0 plans E={E} p={p}")
    nu = 0.9
    R = KronRows(E, p, nu)
    xh = synth.random_vector(R.N, seed=21)
    x = torch.from_numpy(xh).to(dev)
    seen = set()
    first = {}
    for plan in range(10):
        s = Solver(E, p, nu, autotune=False, fd_plan=plan)
        used = s.tuning(1)["fd_plan"][0]
        if used != plan:          # the plan does not fit in LDS at this size
            s.close()
            continue
        seen.add(plan)
        yg = s.apply_P0(x)
        y = yg.cpu().numpy()
        eta = p0_backward_errors(R, xh, y, nu, 400, seed=plan)
        say(f"[shapes]   plan {plan}: FP64 backward errors {['%.1e' % e for e in eta]}")
        assert max(eta) <= 1e-14, plan
        s.close()
        s32 = Solver(E, p, nu, autotune=False, fd_plan=plan, precision="fp32", krylov="fgmres")
        y32g = s32.apply_P0(x)
        y32 = y32g.cpu().numpy()
        assert np.abs(y32 - y).max() / np.abs(y).max() < 1e-5, plan
        s32.close()
        # split BF16 where the plan takes it (hi + lo BF16 halves keep 16
        # significant bits per operand, so each product is good to ~2^-16
        # relative and P_0's six contractions to ~1e-5; the 4-wave plans run
        # FP32 products for this precision: FP32-level gaps)
        s16 = Solver(E, p, nu, autotune=False, fd_plan=plan, precision="bf16x3", krylov="fgmres")
        if s16.tuning(1)["fd_plan"][2] == plan:
            y16 = s16.apply_P0(x).cpu().numpy()
            e16 = np.abs(y16 - y).max() / np.abs(y).max()
            say(f"[shapes]   plan {plan}: split-BF16 gap {e16:.1e}")
            assert e16 < (2e-4 if plan & 1 else 1e-5), plan
        s16.close()
        fam = 2 if plan == 8 else plan & 1
        if fam in first:
            assert torch.equal(yg, first[fam][0]), plan
            assert torch.equal(y32g, first[fam][1]), plan
        else:
            first[fam] = (yg, y32g)
    assert seen, "no P0 plan fits"


@pytest.mark.parametrize("krylov", ["minres", "fgmres"])
def test_row_block_plan_solve(dev, krylov):
    """A batched solve (two right-hand sides) with the row-block P_0 plan 9,
    whose last launches also write the Krylov dot partials (one per plane row
    block), against the 16-wave plan 1 (one per plane): P_0 agrees bit for
    bit, so the only difference is the order of the partial sums; the same
    iteration counts and solutions within 1e-12 of each other."""
    from paper_2311_06926_amd.solver import Solver
    E, p = 20, 3
    say(f"[shapes] row-block plan solve E={E} p={p} {krylov}")
    a = Solver(E, p, 1.0, autotune=False, fd_plan=1, max_rhs=2, krylov=krylov)
    b = Solver(E, p, 1.0, autotune=False, fd_plan=9, max_rhs=2, krylov=krylov)
    assert b.tuning(1)["fd_plan"][0] == 9
    rhs = a.build_rhs([1.0, -0.6])
    xa, ia = a.solve(rhs, 1e-9)
    xb, ib = b.solve(rhs, 1e-9)
    gap = ((xa - xb).abs().max() / xa.abs().max()).item()
    say(f"[shapes]   iterations {ia.iterations} / {ib.iterations}, gap {gap:.1e}")
    assert ia.iterations == ib.iterations and ib.converged == 1
    assert gap <= 1e-12
    a.close()
    b.close()


@pytest.mark.parametrize("krylov", ["minres", "fgmres"])
def test_batched_equals_single_above_dot_chunk_switch(dev, krylov):
    """From 2^19 unknowns on the Krylov dot products use 480 chunks per
    vector instead of 240 (the count depends on the length alone): a batch
    of two right-hand sides still reproduces each one's single solve bit for
    bit, and the MINRES iterations end where the single solves end.  The
    operator shapes are tuned per context (results do not depend on them);
    the P_0 plan is fixed for both, since the plan sets how the last launches
    of P_k split the Krylov dot into partials (the row-block plan per row
    block, the others per plane), i.e. its summation order."""
    from paper_2311_06926_amd.solver import Solver
    E, p = 50, 3
    say(f"[shapes] batched vs single above 2^19 unknowns E={E} p={p} {krylov}")
    sb = Solver(E, p, 1.0, iters=1, krylov=krylov, max_rhs=2, fd_plan=9)
    ss = Solver(E, p, 1.0, iters=1, krylov=krylov, fd_plan=9)
    N = sb.N
    assert N >= 1 << 19
    rhs = sb.build_rhs([1.0, -0.6])
    xb, ib = sb.solve(rhs, 1e-8)
    assert ib.converged == 1
    for r in range(2):
        xs, is_ = ss.solve(rhs[r * N:(r + 1) * N].clone(), 1e-8)
        say(f"[shapes]   rhs {r}: {ib.iters_per_rhs[r]} / {is_.iterations} iterations")
        assert ib.iters_per_rhs[r] == is_.iterations
        assert torch.equal(xb[r * N:(r + 1) * N], xs)
    sb.close()
    ss.close()


def test_autotuner_reports_shapes_in_range(dev):
    from paper_2311_06926_amd.solver import Solver
    E, p = 12, 3
    say(f"[shapes] autotune E={E} p={p}")
    s = Solver(E, p, 1.0, max_rhs=3)
    plain = Solver(E, p, 1.0, autotune=False, max_rhs=3)
    for nr in (1, 3):
        t = s.tuning(nr)
        say(f"[shapes]   nrhs={nr}: {t}")
        assert t["op_tuned"] and 1 <= t["op_kchunk"] <= E + p - 1 and t["op_order"] in (0, 1)
        assert t["op_us"] > 0
        assert all(0 <= f <= 9 for f in t["fd_plan"]) and all(us > 0 for us in t["fd_us"])
        x = torch.from_numpy(synth.random_vector(nr * s.N, seed=nr)).to(dev)
        assert torch.equal(s.apply_K(x), plain.apply_K(x))
    assert not s.tuning(2)["op_tuned"]      # a batch size the tuner did not time
    s.close()
    plain.close()


def test_differentiable_solve_96_matches_central_differences(dev):
    """The differentiable-solve workload at 96^3, degree 3, FP32 P_k inside
    FP64 FGMRES: dL/dnu and the derivative of L along a random direction of
    the body-force field (adjoint) against central differences with step
    1e-6.  L is quadratic in beta, so the central difference along beta is
    exact up to the solve tolerance; along nu its truncation error is
    O(h^2).  With tol 1e-11 the gap is ~tol |L| / h ~ 1e-5 relative."""
    from paper_2311_06926_amd.autograd import cavity_loss
    from paper_2311_06926_amd.solver import Solver
    E, p, nu, h, tol = 96, 3, 1.0, 1e-6, 1e-11
    say(f"[fullsize] differentiable solve E={E} p={p} (fp32 P_k, FGMRES)")
    sol = Solver(E, p, nu, krylov="fgmres", precision="fp32", iters=1, maxit=2000)
    ut, _ = sol.solve(sol.build_rhs([1.5]), tol)          # target: another lid speed
    ut = ut[:sol.nV].clone()
    beta0 = torch.from_numpy(synth.random_vector(sol.nV, seed=961, scale=0.3)).to(dev)
    d = torch.from_numpy(synth.random_vector(sol.nV, seed=962)).to(dev)
    beta = beta0.clone().requires_grad_(True)
    nu_t = torch.tensor(nu, dtype=torch.float64, device=dev, requires_grad=True)
    L = cavity_loss(beta, nu_t, sol, ut, lid=1.0, tol=tol)
    L.backward()
    g_nu = nu_t.grad.item()
    g_dir = float((beta.grad * d).sum())

    def loss(b, n):
        with torch.no_grad():
            return cavity_loss(b, torch.tensor(n, dtype=torch.float64, device=dev), sol, ut,
                               lid=1.0, tol=tol).item()

    fd_nu = (loss(beta0, nu + h) - loss(beta0, nu - h)) / (2 * h)
    fd_dir = (loss(beta0 + h * d, nu) - loss(beta0 - h * d, nu)) / (2 * h)
    say(f"[fullsize]   L={L.item():.6e} dL/dnu adjoint {g_nu:.8e} fd {fd_nu:.8e}; "
        f"dL/dbeta.d adjoint {g_dir:.8e} fd {fd_dir:.8e}")
    assert abs(g_nu - fd_nu) <= 1e-4 * abs(fd_nu)
    assert abs(g_dir - fd_dir) <= 1e-4 * abs(fd_dir)
    sol.close()
