"""Writes oracle MINRES reference data for the hyper-power sweep of the
lid-driven cavity at 32^3 elements, degree 3 (Sec. 5: MINRES from x_0 = 0 to
a relative preconditioned residual of 1e-8; eq. Pcq1 with the literal schedule
of Sec. 4.1 option (5); orders q in {2, 3}, updates k in {0, 1, 2, 3}).

    python tests/golden/make_oracle_minres_counts.py [E degree] > out.txt

Only ``oracle/`` is called: the assembled Kronecker system, P_0 by sparse LU
and the literal hyper-power recursion.  For every (q, k) the file records the
iteration count, the oracle's true residual ||b - K x||_2 / ||b||_2, the
final recurrence residual, and the solution at a fixed set of sampled
indices (drawn once with a seeded generator and written to the file), so a
test can compare both the count and the converged solution.  The sparse LU
of P_0 is factored once and shared by all runs (about 7 minutes at 32^3 on
one core; the whole sweep about 25 minutes).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.cases import cavity  # noqa: E402
from oracle.krylov import minres  # noqa: E402
from oracle.precond import BasePreconditioner, HyperPower  # noqa: E402

SWEEP = [(2, 0), (2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)]
NSAMPLE = 48


def main():
    E = int(sys.argv[1]) if len(sys.argv) > 1 else 32
    p = int(sys.argv[2]) if len(sys.argv) > 2 else 3
    t0 = time.time()
    S, b = cavity(E, p)
    base = BasePreconditioner(S)
    print(f"# oracle set-up {time.time() - t0:.0f} s", file=sys.stderr, flush=True)
    idx = np.sort(np.random.default_rng(2311_06926).choice(S.N, NSAMPLE, replace=False))
    out = [
        "# Oracle MINRES (x_0 = 0, stop at ||r||_{P^-1} <= 1e-8 ||b||_{P^-1}) on the",
        f"# lid-driven cavity, {E}^3 elements, degree {p}, nu = 1, lid speed 1, no body",
        "# force; P_k of eq. Pcq1 (literal schedule), hyper-power order q, k updates.",
        "# Written by tests/golden/make_oracle_minres_counts.py (calls oracle/ only).",
        f"# N {S.N}",
        "# sample_indices " + " ".join(str(int(i)) for i in idx),
        "# q k iterations true_relres monitored_relres x[sample_indices]...",
    ]
    for q, k in SWEEP:
        t = time.time()
        H = HyperPower(S, q, k, base=base)
        r = minres(lambda v: S.K @ v, H.apply, b, tol=1e-8)
        vals = " ".join(repr(float(v)) for v in r.x[idx])
        out.append(f"{q} {k} {r.iters} {float(r.true_relres)!r} {float(r.history[-1])!r} {vals}")
        print(f"# q={q} k={k}: {r.iters} iterations, true relres {r.true_relres:.3e} "
              f"({time.time() - t:.0f} s)", file=sys.stderr, flush=True)
    print("\n".join(out))


if __name__ == "__main__":
    main()
