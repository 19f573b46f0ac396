"""Benchmark: hyper-power preconditioned Stokes solve on one MI355X.

Workload (default step): 3D lid-driven cavity, 32^3 elements, velocity
degree 3, nu = 1, FP64, preconditioned MINRES to a relative residual of
1e-8 with the order-2 hyper-power preconditioner after one update (q = 2,
k = 1; eqs. Pcv, Pcq1).  One step is one complete solve; the right-hand
side is resident in HBM and set-up (tables, eigen-decompositions, graph
capture) is excluded.  value = solved degrees of freedom per second
(N / time-to-solution).

The JSON line also carries
  operators   DOF/s of apply_K, apply_P0 and apply_hyperpower(q, k)
  sweep       iterations and time-to-solution for q in {2,3} x k in {0..3}
  schur_options  FGMRES iterations and time for the Schur options (1)-(5) of
              Sec. 4.1 at k = 1, 2
  spectra     Lanczos spectra of P_0 (GPU), the predicted condition numbers and
              MINRES bound per k (Corollary cor:Skform), and the (q, k) they
              choose a priori against the sweep's fastest
  quadrature_forward  the quadrature-based forward operator of Sec. 5.3
              (apply_K_quad) against apply_K, and the solve with it as the
              Krylov loop's forward problem for k = 0, 1, 2 (times normalised
              by k = 0, the normalisation of Table 1)
  mixed       64^3, degree 3 FGMRES: FP64 vs FP32 vs split-BF16 preconditioner
  batched     48^3, degree 2: 32 right-hand sides in one FGMRES vs one at a time
  hbm         apply_K on an HBM-sized mesh (working set > Infinity Cache)
  roofline    the kernel group that dominates the step (fast diagonalisation,
              FP64 MFMA), timed live with HIP events on the solver's stream
  cpu_baseline  the FP64 oracle timed on this host at the benchmark mesh
              (one full solve, P_{V,0} by the oracle's einsum fast diagonalisation)
  sec51_operator_study  P_{V,0}, P^_{V,1}, P^_{V,2} and A at 256^3 (Sec. 5.1):
              measured c_A / c_P and the cost-model ratios of eq. hyperpower_scaling

    python bench.py [--steps K] [--warmup W] [--order q] [--iters k]
    python bench.py --only {solve,apply_K,apply_K_quad,apply_P0,copy} ...   (profiling runs)
    python bench.py --only table1 [--forward quadrature]
                                      (Table 1: 8^3..64^3, degrees 2..8, k = 0..4)
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 (vector and MFMA), published
METRIC = "hyper-power Stokes solve: time-to-1e-8 residual + operator DOF/s vs plain FP64"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sizes(E, p):
    nN, nM = E + p - 2, E + p - 1
    nV = 3 * nN * nM * nM
    nQ = nM ** 3
    return nN, nM, nV, nQ, nV + nQ


def pk_counts(q, k):
    """Q-block base applications inside one P_k (eq. Pcq1, literal schedule):
    (P_{Q,0}, B/B' pairs, P_{V,0}, A) by the recursion T(k) = q T(k-1) +
    (q-1) [pair + P_{V,l(k)}], l(1) = 0, l(k) = k (Appendix B)."""
    pq, pb, pv, pa = 1, 0, 0, 0
    for kk in range(1, k + 1):
        lv = 0 if kk == 1 else kk
        pq, pb, pv, pa = (q * pq, q * pb + (q - 1), q * pv + (q - 1) * q ** lv,
                          q * pa + (q - 1) * (q ** lv - 1))
    return pq, pb, pv, pa


def p0_flops(E, p):
    """Algorithmic flops of one P_0^{-1} application (fast diagonalisation):
    per velocity block two transforms of three mode products, pressure three."""
    nN, nM, nV, nQ, N = sizes(E, p)
    return 4.0 * nV * (nN + 2 * nM) + 6.0 * nQ * nM


def timed_loop(fn, reps, stream):
    import torch
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    s.record(stream)
    for _ in range(reps):
        fn()
    e.record(stream)
    e.synchronize()
    return s.elapsed_time(e) / reps / 1e3   # seconds per call


def timed_solve(sol, b, reps):
    import torch
    x, info = sol.solve(b, 1e-8)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x, info = sol.solve(b, 1e-8, x=x)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return x, info, float(np.median(ts))


def measured_peaks():
    """Reference rates measured on this GPU with library kernels: a 1 GiB
    device-to-device copy (HBM) and a large FP64 / FP32 GEMM (rocBLAS or
    hipBLASLt through torch.matmul; MFMA)."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    t = timed_loop(lambda: b.copy_(a), 10, stream)
    out = {"copy_GBps": 2 * 8.0 * n / t / 1e9}
    del a, b
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        m = 8192
        x = torch.randn(m, m, dtype=dt, device="cuda")
        y = torch.randn(m, m, dtype=dt, device="cuda")
        t = timed_loop(lambda: torch.matmul(x, y), 5, stream)
        out[f"gemm_{name}_TFLOPs"] = 2.0 * m ** 3 / t / 1e12
        del x, y
    return out


def differentiable_leg(E, p, tol=1e-10, h=1e-6):
    """Loss ||u(beta, nu) - u_t||^2 over the cavity at E^3 (u_t: the solution
    for lid speed 1.5), FP32 P_k inside FP64 FGMRES: forward solve, adjoint
    backward, and the adjoint gradients against central differences along nu
    and along a random direction of the body-force field (step h); the same
    forward + backward with an FP64 P_k for the speed-up."""
    import torch
    from paper_2311_06926_amd import synth
    from paper_2311_06926_amd.autograd import cavity_loss
    from paper_2311_06926_amd.solver import Solver
    out = {"E": E, "p": p, "tol": tol}
    for prec in ("fp32", "fp64"):
        sol = Solver(E, p, 1.0, krylov="fgmres", precision=prec, iters=1, maxit=2000)
        ut, _ = sol.solve(sol.build_rhs([1.5]), tol)
        ut = ut[:sol.nV].clone()
        beta0 = torch.from_numpy(synth.random_vector(sol.nV, seed=961, scale=0.3)).to("cuda")
        nu_t = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
        beta = beta0.clone().requires_grad_(True)
        cavity_loss(beta, nu_t, sol, ut, tol=tol).backward()      # warm-up
        beta.grad = None
        nu_t.grad = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = cavity_loss(beta, nu_t, sol, ut, tol=tol)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        r = {"forward_ms": 1e3 * (t1 - t0), "backward_ms": 1e3 * (t2 - t1), "loss": L.item(),
             "dL_dnu": nu_t.grad.item()}
        if prec == "fp32":
            d = torch.from_numpy(synth.random_vector(sol.nV, seed=962)).to("cuda")
            g_dir = float((beta.grad * d).sum())

            def loss(b, n):
                with torch.no_grad():
                    return cavity_loss(b, torch.tensor(n, dtype=torch.float64, device="cuda"),
                                       sol, ut, tol=tol).item()

            fd_nu = (loss(beta0, 1.0 + h) - loss(beta0, 1.0 - h)) / (2 * h)
            fd_dir = (loss(beta0 + h * d, 1.0) - loss(beta0 - h * d, 1.0)) / (2 * h)
            r.update({"N": sol.N, "fd_dL_dnu": fd_nu,
                      "dnu_rel_gap_vs_fd": abs(r["dL_dnu"] - fd_nu) / abs(fd_nu),
                      "dbeta_dir_rel_gap_vs_fd": abs(g_dir - fd_dir) / abs(fd_dir)})
        out[prec] = r
        sol.close()
    out["speedup_fp32_vs_fp64"] = ((out["fp64"]["forward_ms"] + out["fp64"]["backward_ms"]) /
                                   (out["fp32"]["forward_ms"] + out["fp32"]["backward_ms"]))
    return out


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2311_06926_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pmc_traffic(profile, src_files):
    """HBM bytes per launch from a committed rocprofv3 --pmc summary, or None
    when the summary is missing or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.split(":", 1)[0].strip() in ("source_hash", "traffic_bytes_per_launch"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != source_hash(*src_files):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(p, q, k, E_full, gpu_iterations):
    """The oracle (numpy/scipy, FP64, BLAS pinned to one thread) on this host
    at the benchmark mesh: one full MINRES solve of the same problem with the
    oracle's P_k, its P_{V,0} by the oracle's einsum fast-diagonalisation
    tier (the sparse-LU form takes minutes to factor at 32^3).  Above about
    half a million unknowns only a fixed number of iterations is timed and
    scaled to the GPU's iteration count (said in `sample`)."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle.cases import cavity
    from oracle.krylov import minres
    from oracle.precond import FastDiagBase, HyperPower
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        S, b = cavity(E_full, p)
        H = HyperPower(S, q, k, base=FastDiagBase(S))
        t1 = time.perf_counter()
        full = S.N <= 500_000
        r = minres(lambda v: S.K @ v, H.apply, b, tol=1e-8 if full else 0.0,
                   maxit=1000 if full else 4)
        t2 = time.perf_counter()
        x = np.random.default_rng(0).standard_normal(S.N)
        t3 = time.perf_counter()
        for _ in range(3):
            S.K @ x
        t4 = time.perf_counter()
    t_iter = (t2 - t1) / max(r.iters, 1)
    t_solve = (t2 - t1) if full else t_iter * gpu_iterations
    # a few iterations with the BLAS pools unrestricted (the sparse products
    # and einsum contractions stay single-threaded)
    t5 = time.perf_counter()
    minres(lambda v: S.K @ v, H.apply, b, tol=0.0, maxit=3)
    t6 = time.perf_counter()
    nthreads = max((pool.get("num_threads", 1) for pool in threadpool_info()), default=1)
    what = (f"one full oracle MINRES solve at {E_full}^3 elements, degree {p}, q={q}, k={k} "
            f"(N={S.N}, {r.iters} iterations, {t2 - t1:.1f} s)" if full else
            f"4 oracle MINRES iterations at {E_full}^3 elements, degree {p}, q={q}, k={k} "
            f"(N={S.N}, {t_iter:.2f} s each), scaled to the GPU's {gpu_iterations} iterations")
    return {
        "value": S.N / t_solve,
        "unit": "DOF/s (solved to 1e-8)",
        "cores": 1,
        "kind": "oracle",
        "sample": (what + "; P_{V,0} by the oracle's einsum fast-diagonalisation tier, P_k "
                   "by its literal recursion, K as scipy CSR; assembly "
                   f"({t1 - t0:.1f} s) excluded like the GPU set-up"),
        "oracle_iterations": r.iters if full else None,
        "seconds_per_iteration": t_iter,
        "apply_K_dofs": S.N / ((t4 - t3) / 3),
        "host_cpus": os.cpu_count(),
        "all_threads": {"seconds_per_iteration": (t6 - t5) / 3, "blas_threads": nthreads},
    }


def cpu_baseline_configs(c1_gpu, c4_gpu):
    """The oracle on one host core at the two other configurations the
    measurement names: the 8^3, degree-2 cavity (q = 2, k = 1, MINRES to
    1e-8, a full solve) and one right-hand side of the 48^3, degree-2 batch
    (right-hand side 0: 16 seeded Fourier modes per component and its lid
    speed; q = 2, k = 1; FGMRES(50); three iterations timed and scaled to
    the GPU's iteration count for that right-hand side).  P_{V,0} by the
    oracle's einsum fast-diagonalisation tier; assembly excluded."""
    from threadpoolctl import threadpool_limits
    from oracle.cases import cavity
    from oracle.krylov import fgmres, minres
    from oracle.precond import FastDiagBase, HyperPower
    from paper_2311_06926_amd import synth
    out = {}
    with threadpool_limits(limits=1):
        S, b = cavity(8, 2)
        H = HyperPower(S, 2, 1, base=FastDiagBase(S))
        t0 = time.perf_counter()
        r = minres(lambda v: S.K @ v, H.apply, b, tol=1e-8)
        t1 = time.perf_counter()
        out["C1"] = {"E": 8, "p": 2, "N": S.N, "oracle_iterations": r.iters,
                     "oracle_ms": 1e3 * (t1 - t0), "oracle_dofs": S.N / (t1 - t0),
                     "gpu": c1_gpu,
                     "sample": "one full oracle MINRES solve, q=2, k=1, one core"}
        modes, U = synth.body_force_modes(0)
        S, b = cavity(48, 2, U=U, modes=modes)
        H = HyperPower(S, 2, 1, base=FastDiagBase(S))
        t0 = time.perf_counter()
        fgmres(lambda v: S.K @ v, lambda v, j: H.apply(v), b, tol=0.0, restart=50, maxit=3)
        t1 = time.perf_counter()
        t_it = (t1 - t0) / 3
        its = c4_gpu.get("iterations") if c4_gpu else None
        out["C4_one_rhs"] = {
            "E": 48, "p": 2, "N": S.N, "oracle_seconds_per_iteration": t_it,
            "oracle_dofs": S.N / (t_it * its) if its else None, "gpu": c4_gpu,
            "sample": ("3 oracle FGMRES(50) iterations on right-hand side 0 of the batch, "
                       "q=2, k=1, one core, scaled to the GPU's iteration count")}
    return out


def sec51_leg(E, p, hbm_peak, fp64_peak):
    """The operator study of Sec. 5.1 (eq. hyperpower_scaling) at E^3: the
    velocity block P_{V,k}^{-1} for k = 0, 1, 2 (q = 2) and the operator A,
    the measured c_A / c_P, and the cost-model ratios C_k / C_0 =
    2^k + (2^k - 1) c_A / c_P it implies against the measured ones (the
    paper's 384^3 one-thread CPU run: 4.47 and 11.44, model 4.5 and 11.5)."""
    import torch
    from paper_2311_06926_amd import synth
    from paper_2311_06926_amd.solver import Solver
    s = Solver(E, p, 1.0)
    u = torch.from_numpy(synth.random_vector(s.nV, 8)).to("cuda")
    y = s.empty(s.nV)
    t = {}
    for kk in (0, 1, 2):
        t[kk] = timed_loop(lambda: s.apply_PV(2, kk, u, y), 5, s.stream)
    tA = timed_loop(lambda: s.apply_A(u, y), 10, s.stream)
    nN, nM, nV, nQ, N = sizes(E, p)
    fl_v = 4.0 * nV * (nN + 2 * nM)
    ratio = tA / t[0]
    out = {"E": E, "p": p, "n_V": nV, "PV0_ms": 1e3 * t[0], "PV1_ms": 1e3 * t[1],
           "PV2_ms": 1e3 * t[2], "A_ms": 1e3 * tA, "cA_over_cP": ratio,
           "C1_over_C0_measured": t[1] / t[0], "C1_over_C0_model": 2 + ratio,
           "C2_over_C0_measured": t[2] / t[0], "C2_over_C0_model": 4 + 3 * ratio,
           "PV0_TFLOPs": fl_v / t[0] / 1e12, "PV0_mfma_frac": fl_v / t[0] / 1e12 / fp64_peak,
           "A_algorithmic_GBps": 16.0 * nV / tA / 1e9,
           "A_hbm_frac": 16.0 * nV / tA / 1e9 / hbm_peak, "tuning": s.tuning(1)}
    s.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--E", type=int, default=32)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--order", type=int, default=2)
    ap.add_argument("--iters", type=int, default=1)
    ap.add_argument("--schur", default="Pcq1")
    ap.add_argument("--only", default=None,
                    choices=["solve", "apply_K", "apply_K_quad", "apply_P0", "copy", "table1"])
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3"],
                    help="preconditioner precision for --only apply_P0")
    ap.add_argument("--op-kchunk", type=int, default=0,
                    help="--only solve/apply_K/apply_P0: force the operator i3-chunk (no autotuning)")
    ap.add_argument("--op-order", type=int, default=-1,
                    help="--only solve/apply_K/apply_P0: force the velocity workgroup order")
    ap.add_argument("--op-staged", type=int, default=-1,
                    help="--only solve/apply_K/apply_P0: force the all-planes operator kernels "
                         "(1) or the streaming ones (0); -1: tuned")
    ap.add_argument("--op-dma", type=int, default=-1,
                    help="--only apply_K/solve: the streaming velocity kernel's staging "
                         "(1 direct-to-LDS loads, 0 registers, -1 default)")
    ap.add_argument("--op-pres-wide", type=int, default=-1,
                    help="--only apply_K/solve: the streaming pressure kernel's tiles "
                         "(1 32 x 8, 0 16 x 8, -1 tuned)")
    ap.add_argument("--fd-plan", type=int, default=-1,
                    help="--only solve/apply_P0: force the fast-diagonalisation plan (-1: tuned)")
    ap.add_argument("--forward", default="kronecker", choices=["kronecker", "quadrature"],
                    help="forward problem of the solve and table1 legs (quadrature: Sec. 5.3)")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip mixed/batched/hbm legs")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--hbm-E", type=int, default=192)
    ap.add_argument("--diff-E", type=int, default=96)
    ap.add_argument("--sec51-E", type=int, default=256,
                    help="mesh of the Sec. 5.1 operator study (P_{V,k} for k = 0, 1, 2)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(multi-GPU sharding is not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_06926_amd import synth
    from paper_2311_06926_amd.solver import Solver

    torch.cuda.set_device(0)
    E, p, q, k = args.E, args.p, args.order, args.iters
    nN, nM, nV, nQ, N = sizes(E, p)

    if args.only == "copy":
        # calibration for the PMC byte counters: a plain device copy of 1 GiB
        n = 1 << 27
        xa = torch.ones(n, dtype=torch.float64, device="cuda")
        ya = torch.empty_like(xa)
        for _ in range(args.reps):
            ya.copy_(xa)
        torch.cuda.synchronize()
        log(f"[bench] copied {args.reps} x {8 * n} bytes")
        return
    if args.only == "table1":
        # Table 1 of Sec. 5.3: MINRES iterations and solution time normalised
        # by that of P^_0, meshes 8^3..64^3, degrees 2..8, k = 0..4
        rows = []
        for Et in (8, 16, 32, 64):
            for pt in (2, 4, 6, 8):
                its, ms = [], []
                for kk in range(5):
                    s2 = Solver(Et, pt, 1.0, order=2, iters=kk, forward=args.forward)
                    b2 = s2.build_rhs([1.0])
                    _, inf2, t2 = timed_solve(s2, b2, 3)
                    its.append(inf2.iterations)
                    ms.append(1e3 * t2)
                    s2.close()
                rows.append({"E": Et, "p": pt, "iterations": its, "ms": ms,
                             "T_sol": [m / ms[0] for m in ms]})
                log(f"[bench] table1 {Et}^3 p={pt}: {its} ms {[round(m, 2) for m in ms]}")
        print(json.dumps({"table1": rows, "forward": args.forward}), flush=True)
        return
    if args.only in ("apply_K", "apply_K_quad", "apply_P0"):
        forced = args.op_kchunk > 0
        sol = Solver(E, p, 1.0, precision=args.prec,
                     krylov="minres" if args.prec == "fp64" else "fgmres",
                     autotune=not forced, op_kchunk=args.op_kchunk, op_order=args.op_order,
                     op_slabs=1 if forced else 0, fd_plan=args.fd_plan,
                     op_staged=args.op_staged, op_dma=args.op_dma,
                     op_pres_wide=args.op_pres_wide)
        xr = torch.from_numpy(synth.random_vector(sol.N, 3)).to("cuda")
        yr = sol.empty(sol.N)
        fn = {"apply_K": sol.apply_K, "apply_K_quad": sol.apply_K_quad,
              "apply_P0": sol.apply_P0}[args.only]
        fn(xr, yr)
        t = timed_loop(lambda: fn(xr, yr), args.reps, sol.stream)
        log(f"[bench] {args.only} E={E} p={p} N={sol.N}: {t * 1e6:.2f} us per call "
            f"({args.reps} timed calls after 1 warm-up; tuning {sol.tuning(1)})")
        return

    log(f"[bench] setup E={E} p={p} q={q} k={k} N={N}")
    forced = args.op_kchunk > 0
    sol = Solver(E, p, 1.0, order=q, iters=k, schur=args.schur, fd_plan=args.fd_plan,
                 op_kchunk=args.op_kchunk, op_order=args.op_order, op_slabs=1 if forced else 0,
                 op_staged=args.op_staged, op_dma=args.op_dma,
                 op_pres_wide=args.op_pres_wide, forward=args.forward)
    stream = sol.stream
    b = sol.build_rhs([1.0])
    x, info = sol.solve(b, 1e-8)
    for _ in range(args.warmup):
        x, info = sol.solve(b, 1e-8, x=x)
    log(f"[bench] warmup done: {info.iterations} iterations, true relres {info.true_relres:.2e}, "
        f"tuning {sol.tuning(1)}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, info = sol.solve(b, 1e-8, x=x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps
    log(f"[bench] timed {args.steps} solves: {step_s * 1e3:.3f} ms each, {info.iterations} iterations")
    if args.only == "solve":
        return

    # ---- operator throughput (events on the solver's stream)
    xr = torch.from_numpy(synth.random_vector(N, 3)).to("cuda")
    yk = sol.empty(N)
    t_K = timed_loop(lambda: sol.apply_K(xr, yk), 50, stream)
    t_P0 = timed_loop(lambda: sol.apply_P0(xr, yk), 50, stream)
    t_Pk = timed_loop(lambda: sol.apply_hyperpower(q, k, xr, yk), 20, stream)
    ops = {
        "apply_K_dofs": N / t_K, "apply_K_us": t_K * 1e6,
        "apply_P0_dofs": N / t_P0, "apply_P0_us": t_P0 * 1e6,
        f"apply_hyperpower_q{q}_k{k}_dofs": N / t_Pk,
        f"apply_hyperpower_q{q}_k{k}_us": t_Pk * 1e6,
    }
    log(f"[bench] operators: {ops}")

    # ---- roofline: fast diagonalisation dominates the step's GPU time
    flops = p0_flops(E, p)
    achieved = flops / t_P0 / 1e12
    # each operator against its own roof at this mesh (the working set, about
    # 40 MB, sits in the 256 MB Infinity Cache, so the HBM figures are
    # effective rates), and P_k weighted: the time its base operators would
    # take at their roofs (Appendix B counts) over its measured time
    nN_, nM_, nV_, nQ_, N_ = sizes(E, p)
    fl_pv0 = 4.0 * nV_ * (nN_ + 2 * nM_)
    fl_pq0 = 6.0 * nQ_ * nM_
    t_roof = lambda fl=0.0, by=0.0: max(fl / (FP64_PEAK_TFLOPS * 1e12), by / (HBM_PEAK_GBS * 1e9))
    nv_pv0, nv_a = q ** k, q ** k - 1
    if k == 0:
        nq_pq0, nq_b, nq_pv0, nq_a = 1, 0, 0, 0
    else:
        nq_pq0, nq_b, nq_pv0, nq_a = pk_counts(q, k)
    ideal = ((nv_pv0 + nq_pv0) * t_roof(fl=fl_pv0) + (nv_a + nq_a) * t_roof(by=16.0 * nV_)
             + nq_pq0 * t_roof(fl=fl_pq0) + nq_b * t_roof(by=16.0 * (nV_ + nQ_)))
    per_op = {
        "apply_K": {"bound": "hbm", "unit": "GB/s", "achieved": 16.0 * N / t_K / 1e9,
                    "peak": HBM_PEAK_GBS, "frac": 16.0 * N / t_K / 1e9 / HBM_PEAK_GBS,
                    "note": "effective: 16 B/DOF algorithmic, working set in the Infinity Cache"},
        "apply_P0": {"bound": "mfma", "unit": "TFLOP/s", "achieved": achieved,
                     "peak": FP64_PEAK_TFLOPS, "frac": achieved / FP64_PEAK_TFLOPS},
        f"apply_hyperpower_q{q}_k{k}": {
            "bound": "weighted", "ideal_us": ideal * 1e6, "measured_us": t_Pk * 1e6,
            "frac": ideal / t_Pk,
            "note": ("sum over its base applications (Appendix B counts) of each at its roof "
                     "(P_0 blocks at FP64 MFMA peak, A and the B pairs at 16 B/DOF over HBM), "
                     "over the measured time")},
    }
    plan = sol.tuning(1)["fd_plan"][0]
    if plan == 9:
        kname = ("apply_P0 (plan 9): k_fd_xy_s (16-row blocks, modes 1,2) + k_fd_z_w (16 rows, "
                 "mode 3 + scaling) + k_fd_xy_s (inverse), FP64 16x16x4 MFMA")
    elif plan == 8:
        kname = "apply_P0 (plan 8): k_mode_gemm (six mode products per component), FP64 MFMA"
    else:
        kname = (f"apply_P0 (plan {plan}): k_fd_xy_w (modes 1,2) + k_fd_z_w (mode 3 + scaling) "
                 "+ k_fd_xy_w (inverse), FP64 16x16x4 MFMA")
    roof = {
        "kernel": kname,
        "bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved / FP64_PEAK_TFLOPS,
        "traffic": pmc_traffic(f"apply_P0_E{E}p{p}_pmc.txt", ["fd.hip"]),
        "algorithmic_flops_per_launch": flops, "avg_launch_us": t_P0 * 1e6,
        "per_operator": per_op,
    }

    # ---- the same solve with each iteration replayed as a captured HIP graph
    # against direct launches (the default; identical results)
    launch_modes = {}
    if not args.no_sweep:
        for g in (True, False):
            s2 = Solver(E, p, 1.0, order=q, iters=k, schur=args.schur, use_graph=g)
            b2 = s2.build_rhs([1.0])
            _, inf2, t2 = timed_solve(s2, b2, 5)
            launch_modes["graph" if g else "direct"] = {"iterations": inf2.iterations,
                                                        "ms": 1e3 * t2}
            s2.close()
        log(f"[bench] launch modes: {launch_modes}")

    # ---- sweep q x k
    sweep = {}
    if not args.no_sweep:
        for qq, kk in [(2, 0), (2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)]:
            s2 = Solver(E, p, 1.0, order=qq, iters=kk, schur=args.schur)
            b2 = s2.build_rhs([1.0])
            _, inf2, t2 = timed_solve(s2, b2, 3)
            sweep[f"q{qq}_k{kk}"] = {"iterations": inf2.iterations, "ms": 1e3 * t2,
                                     "true_relres": inf2.true_relres}
            log(f"[bench] sweep q={qq} k={kk}: {sweep[f'q{qq}_k{kk}']}")
            s2.close()

    # ---- the quadrature-based forward operator (Sec. 5.3): its time against
    # apply_K, and solves with it as the forward problem (the paper's T_f)
    quad = {}
    if not args.no_sweep:
        sol.apply_K_quad(xr, yk)
        t_Q = timed_loop(lambda: sol.apply_K_quad(xr, yk), 20, stream)
        quad = {"apply_K_quad_us": t_Q * 1e6, "apply_K_quad_dofs": N / t_Q,
                "apply_K_us": t_K * 1e6, "quad_over_kron": t_Q / t_K,
                "points": (E * (p + 1) + 2) ** 3,
                f"Tp_over_Tf_q{q}_k{k}": t_Pk / t_Q, "solves": {}}
        base = {}
        for kk in (0, 1, 2):
            for fw in ("quadrature", "kronecker"):
                s2 = Solver(E, p, 1.0, order=2, iters=kk, schur=args.schur, forward=fw)
                b2 = s2.build_rhs([1.0])
                _, inf2, t2 = timed_solve(s2, b2, 3)
                base.setdefault(fw, t2)
                quad["solves"][f"{fw}_q2_k{kk}"] = {
                    "iterations": inf2.iterations, "ms": 1e3 * t2,
                    "T_sol_normalised": t2 / base[fw], "true_relres": inf2.true_relres}
                s2.close()
        log(f"[bench] quadrature forward: {quad}")

    # ---- Schur options of Sec. 4.1 at this mesh (FGMRES, q = 2, k = 1, 2):
    # (1) eq. Pcq2 with P_{V,0}, (2) eq. Pcq2 with a fixed P_{V,2}, (3)/(4)
    # eq. Pcq2 on an inner CG solve (tol 1e-2, at most 20 steps) with P_{V,0}
    # or P_{V,1}, (5) eq. Pcq1 (the default)
    schur_opts = {}
    if not args.no_sweep:
        variants = [("opt1_Pcq2_l0", dict(schur="Pcq2", schur_level=0)),
                    ("opt2_Pcq2_l2", dict(schur="Pcq2", schur_level=2)),
                    ("opt3_pcg_l0", dict(schur="Pcq_pcg", schur_level=0)),
                    ("opt4_pcg_l1", dict(schur="Pcq_pcg", schur_level=1)),
                    ("opt5_Pcq1", dict(schur="Pcq1"))]
        for kk in (1, 2):
            for name, kw in variants:
                s2 = Solver(E, p, 1.0, order=2, iters=kk, krylov="fgmres", **kw)
                b2 = s2.build_rhs([1.0])
                _, inf2, t2 = timed_solve(s2, b2, 3)
                schur_opts[f"{name}_k{kk}"] = {"iterations": inf2.iterations, "ms": 1e3 * t2,
                                               "true_relres": inf2.true_relres}
                log(f"[bench] schur option {name} k={kk}: {schur_opts[f'{name}_k{kk}']}")
                s2.close()

    # ---- a-priori depth from the P_0 spectra (Lanczos on the GPU): predicted
    # condition numbers and MINRES bound per k, times the measured cost of
    # one iteration (apply_K + apply_hyperpower), against the sweep
    spectra = {}
    if not args.no_sweep:
        from paper_2311_06926_amd import spectra as spm
        cost = {}
        for qq in (2, 3):
            s2 = Solver(E, p, 1.0, order=qq, iters=1, schur=args.schur)
            torch.cuda.synchronize()
            t0s = time.perf_counter()
            pred = spm.predict(s2, qq, 3)
            t_lanczos = time.perf_counter() - t0s
            per_it = {}
            for kk in range(0 if qq == 2 else 1, 4):
                t_pk = timed_loop(lambda: s2.apply_hyperpower(qq, kk, xr, yk), 5, s2.stream)
                per_it[kk] = t_K + t_pk
                cost[f"q{qq}_k{kk}"] = pred["k"][kk]["minres_bound"] * per_it[kk]
            spectra[f"q{qq}"] = {
                "lanczos_s": t_lanczos, "velocity_0": pred["velocity_0"],
                "schur_0": pred["schur_0"], "schur_level": pred["schur_level"],
                "predicted": [{key: r[key] for key in ("k", "kappa_v", "kappa_s", "minres_bound")}
                              for r in pred["k"]],
                "us_per_iteration": {kk: 1e6 * v for kk, v in per_it.items()},
                "chosen_k": spm.choose_iters(pred, per_it),
            }
            log(f"[bench] spectra q={qq}: {spectra[f'q{qq}']}")
            s2.close()
        choice = min(cost, key=cost.get)
        spectra["chosen"] = choice
        if sweep:
            best = min(sweep, key=lambda key: sweep[key]["ms"])
            spectra["measured_best"] = best
            spectra["chosen_ms_over_best_ms"] = sweep[choice]["ms"] / sweep[best]["ms"]
        log(f"[bench] a-priori choice {choice}; measured best {spectra.get('measured_best')}")

    mixed, batched, hbm, diff, large = {}, {}, {}, {}, {}
    if not args.no_extra:
        # ---- mixed precision, 64^3 degree 3, FGMRES(50), q = 2, k = 1
        Em, pm = 64, 3
        ref = None
        for prec in ["fp64", "fp32", "bf16x3"]:
            sm = Solver(Em, pm, 1.0, krylov="fgmres", precision=prec, order=2, iters=1)
            bm = sm.build_rhs([1.0])
            xm, im, tm = timed_solve(sm, bm, 3)
            if ref is None:
                ref = xm.clone()
            err = float((xm[:sm.nV] - ref[:sm.nV]).norm() / ref[:sm.nV].norm())
            mixed[prec] = {"ms": 1e3 * tm, "iterations": im.iterations,
                           "true_relres": im.true_relres, "velocity_rel_err_vs_fp64": err}
            log(f"[bench] mixed {prec}: {mixed[prec]}")
            sm.close()
        for prec in ["fp32", "bf16x3"]:
            mixed[prec]["speedup_vs_fp64"] = mixed["fp64"]["ms"] / mixed[prec]["ms"]
        # ---- batched right-hand sides, 48^3 degree 2, 32 RHS
        Eb, pb, R = 48, 2, 32
        lids, amps, wavs = [], [], []
        for r in range(R):
            modes, U = synth.body_force_modes(r)
            a, w = synth.modes_to_arrays(modes)
            lids.append(U)
            amps.append(a)
            wavs.append(w)
        sb = Solver(Eb, pb, 1.0, krylov="fgmres", precision="fp32", order=2, iters=1, max_rhs=R)
        bb = sb.build_rhs(np.array(lids), (np.stack(amps), np.stack(wavs)))
        _, ib, tb = timed_solve(sb, bb, 2)
        s1 = Solver(Eb, pb, 1.0, krylov="fgmres", precision="fp32", order=2, iters=1)
        b1 = bb[:s1.N].clone()
        _, i1, t1s = timed_solve(s1, b1, 3)
        s64 = Solver(Eb, pb, 1.0, krylov="fgmres", precision="fp64", order=2, iters=1, max_rhs=R)
        _, ib64, tb64 = timed_solve(s64, bb, 2)
        # the same batch with every Arnoldi step replayed as a captured graph
        sg = Solver(Eb, pb, 1.0, krylov="fgmres", precision="fp32", order=2, iters=1, max_rhs=R,
                    use_graph=True)
        _, ibg, tbg = timed_solve(sg, bb, 2)
        batched = {"rhs": R, "N": sb.N, "ms": 1e3 * tb, "iterations": ib.iterations,
                   "true_relres": ib.true_relres, "dofs": R * sb.N / tb,
                   "single_rhs_ms": 1e3 * t1s, "single_rhs_iterations": i1.iterations,
                   "speedup_vs_sequential": R * t1s / tb,
                   "fp64_batched_ms": 1e3 * tb64, "speedup_vs_fp64_batched": tb64 / tb,
                   "graph_ms": 1e3 * tbg, "graph_iterations": ibg.iterations}
        log(f"[bench] batched: {batched}")
        sb.close()
        s1.close()
        s64.close()
        sg.close()
        # ---- apply_K on an HBM-sized mesh
        Eh = args.hbm_E
        sh = Solver(Eh, p, 1.0)
        xh = torch.from_numpy(synth.random_vector(sh.N, 4)).to("cuda")
        yh = sh.empty(sh.N)
        th = timed_loop(lambda: sh.apply_K(xh, yh), 10, sh.stream)
        gbs = 16.0 * sh.N / th / 1e9
        hbm = {"E": Eh, "p": p, "N": sh.N, "apply_K_us": th * 1e6, "apply_K_dofs": sh.N / th,
               "algorithmic_GBps": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
               "vector_MB": 8.0 * sh.N / 1e6,
               "traffic": pmc_traffic(f"apply_K_E{Eh}p{p}_pmc.txt", ["ops.hip"])}
        log(f"[bench] hbm: {hbm}")
        sh.close()
        del xh, yh
        # ---- HBM sweep of apply_K (vectors of 17 MB .. 550 MB) and measured peaks
        sweep_hbm = []
        for Es in (128, 192, 256):
            for ps in (2, 3):
                ss = Solver(Es, ps, 1.0)
                xs = torch.from_numpy(synth.random_vector(ss.N, 6)).to("cuda")
                ys = ss.empty(ss.N)
                ts = timed_loop(lambda: ss.apply_K(xs, ys), 10, ss.stream)
                gs = 16.0 * ss.N / ts / 1e9
                sweep_hbm.append({"E": Es, "p": ps, "N": ss.N, "vector_MB": 8.0 * ss.N / 1e6,
                                  "apply_K_us": ts * 1e6, "algorithmic_GBps": gs,
                                  "hbm_frac": gs / HBM_PEAK_GBS, "tuning": ss.tuning(1)})
                log(f"[bench] hbm sweep: {sweep_hbm[-1]}")
                ss.close()
                del xs, ys
        hbm["sweep"] = sweep_hbm
        hbm["measured_peaks"] = measured_peaks()
        log(f"[bench] measured peaks: {hbm['measured_peaks']}")
        # ---- the same kernels on the 96^3, degree-3 mesh (MFMA-sized direction tiles)
        El = args.diff_E
        sl = Solver(El, p, 1.0)
        xl = torch.from_numpy(synth.random_vector(sl.N, 5)).to("cuda")
        yl = sl.empty(sl.N)
        tlk = timed_loop(lambda: sl.apply_K(xl, yl), 20, sl.stream)
        tlp = timed_loop(lambda: sl.apply_P0(xl, yl), 20, sl.stream)
        fl = p0_flops(El, p)
        large = {"E": El, "p": p, "N": sl.N, "apply_K_us": tlk * 1e6,
                 "apply_K_algorithmic_GBps": 16.0 * sl.N / tlk / 1e9,
                 "apply_K_hbm_frac": 16.0 * sl.N / tlk / 1e9 / HBM_PEAK_GBS,
                 "apply_P0_us": tlp * 1e6, "apply_P0_TFLOPs": fl / tlp / 1e12,
                 "apply_P0_mfma_frac": fl / tlp / 1e12 / FP64_PEAK_TFLOPS,
                 "tuning": sl.tuning(1)}
        log(f"[bench] large mesh: {large}")
        sl.close()
        del xl, yl
        # ---- differentiable solve, 96^3 degree 3: forward + adjoint backward
        diff = differentiable_leg(args.diff_E, 3)
        log(f"[bench] differentiable: {diff}")

    sec51 = []
    if not args.no_extra:
        # ---- the operator study of Sec. 5.1 at 256^3 (beyond the in-LDS
        # tiles: P_0 as mode-product GEMMs)
        for ps in (2, 3):
            sec51.append(sec51_leg(args.sec51_E, ps, HBM_PEAK_GBS, FP64_PEAK_TFLOPS))
            log(f"[bench] sec 5.1: {sec51[-1]}")
        roof["per_operator"]["apply_P0_E%d" % args.sec51_E] = {
            r["p"]: {"bound": "mfma", "unit": "TFLOP/s", "achieved": r["PV0_TFLOPs"],
                     "peak": FP64_PEAK_TFLOPS, "frac": r["PV0_mfma_frac"]} for r in sec51}
        if hbm:
            best = max(hbm["sweep"], key=lambda r: r["hbm_frac"])
            roof["per_operator"]["apply_K_hbm_sweep_best"] = {
                "bound": "hbm", "unit": "GB/s", "achieved": best["algorithmic_GBps"],
                "peak": HBM_PEAK_GBS, "frac": best["hbm_frac"], "E": best["E"], "p": best["p"]}
        if large:
            roof["per_operator"][f"apply_P0_E{large['E']}"] = {
                "bound": "mfma", "unit": "TFLOP/s", "achieved": large["apply_P0_TFLOPs"],
                "peak": FP64_PEAK_TFLOPS, "frac": large["apply_P0_mfma_frac"]}

    cpu = None
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(p, q, k, E, info.iterations)
        # the 8^3 degree-2 cavity on the GPU (median of 5 solves) beside the
        # oracle there and at one right-hand side of the batch
        s8 = Solver(8, 2, 1.0, order=2, iters=1)
        b8 = s8.build_rhs([1.0])
        _, i8, t8 = timed_solve(s8, b8, 5)
        s8.close()
        c1_gpu = {"iterations": i8.iterations, "ms": 1e3 * t8, "dofs": s8.N / t8}
        c4_gpu = ({"iterations": batched["single_rhs_iterations"], "ms": batched["single_rhs_ms"],
                   "precision": "fp32 P_k, FP64 FGMRES"} if batched else None)
        cpu["other_configs"] = cpu_baseline_configs(c1_gpu, c4_gpu)
        log(f"[bench] cpu: {cpu}")

    out = {
        "metric": METRIC,
        "value": N / step_s,
        "unit": "DOF/s (solved to 1e-8)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (analytic lid-driven cavity right-hand side; seeded body forces)",
        "config": {"workload": (f"lid-driven cavity {E}^3 elements, degree {p}, nu=1, FP64 MINRES "
                                f"to 1e-8, hyper-power q={q} k={k} ({args.schur})"),
                   "elements": E, "degree": p, "N": N, "order": q, "updates": k,
                   "iterations": info.iterations, "true_relres": info.true_relres},
        "operators": ops,
        "roofline": roof,
        "cpu_baseline": cpu,
        "launch_modes": launch_modes,
        "sweep": sweep,
        "spectra": spectra,
        "schur_options": schur_opts,
        "quadrature_forward": quad,
        "mixed": mixed,
        "batched": batched,
        "hbm": hbm,
        "large_mesh": large,
        "differentiable": diff,
        "sec51_operator_study": sec51,
    }
    print(json.dumps(out), flush=True)
    sol.close()


if __name__ == "__main__":
    main()
