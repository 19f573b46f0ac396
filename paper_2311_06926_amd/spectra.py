"""A-priori choice of the hyper-power depth from the spectra of P_0.

The spectrum of P_k^{-1} A~ after k updates of order q is the image of that
of P_0^{-1} A~ under k applications of t -> 1 - (1 - t)^q (Sec. 2, Lemma
Sk_posdef and Corollary cor:Skform; the q = 2 map is 2t - t^2), so two
Lanczos runs at k = 0 (``Solver.spectrum``) predict the block spectra at
every k.  For the Schur block the prediction uses the sequence on the
exact Schur complement (eq. Pcq_exact), which the updated sequence eq.
Pcq1 follows closely (Sec. 5.2).

From the block intervals sigma(P_V^{-1} A) in [d, D] and
sigma(P_Q^{-1} B' A^{-1} B) in [g, G], the eigenvalues of the block-diagonally
preconditioned saddle-point matrix lie in

    [(d - sqrt(d^2 + 4 D G)) / 2, (D - sqrt(D^2 + 4 d g)) / 2]
      U [d, (D + sqrt(D^2 + 4 D G)) / 2]

(the classical inclusion for block-diagonal preconditioners of saddle-point
problems, Rusten and Winther 1992; Silvester and Wathen 1994), and MINRES
on two intervals [-a, -b] U [c, e] of equal length reduces the residual
by at least ((sqrt(a e) - sqrt(b c)) / (sqrt(a e) + sqrt(b c)))^m every 2m
steps (the shorter interval is widened to equal length).  The iteration
bound times the measured cost of one iteration ranks the depths; the bound
is pessimistic in absolute terms, so only its ratios across k are used.
"""
import math


def hyperpower_map(t, q):
    """One update of order q on an eigenvalue t of P_k^{-1} A~."""
    return 1.0 - (1.0 - t) ** q


def hyperpower_interval(lo, hi, q, k):
    """Bounds of the spectrum after k updates from [lo, hi] inside (0, 2):
    the map is increasing on (0, 1] and, for even q, decreasing on [1, 2)
    with its maximum 1 at t = 1, so the bounds are the images of lo, hi
    and (when inside) 1."""
    pts = [lo, hi] + ([1.0] if lo < 1.0 < hi else [])
    for _ in range(k):
        pts = [hyperpower_map(t, q) for t in pts]
    return min(pts), max(pts)


def saddle_intervals(v, s):
    """Negative and positive eigenvalue intervals ((a, b), (c, e)) as
    magnitudes, [-a, -b] U [c, e], of the preconditioned saddle-point matrix
    from the velocity interval v = (d, D) and the Schur interval s = (g, G)."""
    d, D = v
    g, G = s
    a = 0.5 * (math.sqrt(d * d + 4.0 * D * G) - d)
    b = 0.5 * (math.sqrt(D * D + 4.0 * d * g) - D)
    return (a, b), (d, 0.5 * (D + math.sqrt(D * D + 4.0 * D * G)))


def minres_bound(neg, pos, tol):
    """Iterations after which the two-interval MINRES bound is below tol."""
    (a, b), (c, e) = neg, pos
    la, lp = a - b, e - c
    if la < lp:
        a = b + lp
    else:
        e = c + la
    rho = (math.sqrt(a * e) - math.sqrt(b * c)) / (math.sqrt(a * e) + math.sqrt(b * c))
    if rho <= 0.0:
        return 2
    return 2 * max(1, math.ceil(math.log(tol / 2.0) / math.log(rho)))


def schur_level_for(v0, q, target=1e-8, kmax=6):
    """Smallest l with max |1 - t|^(q^l) <= target over v0 = (d, D): then
    B' P_{V,l}^{-1} B stands for the exact Schur complement."""
    r = max(abs(1.0 - v0[0]), abs(1.0 - v0[1]))
    for lvl in range(kmax + 1):
        if r ** (q ** lvl) <= target:
            return lvl
    return kmax


def predict(sol, q, kmax, tol=1e-8, steps=60, seed=0):
    """Measured P_0 spectra and the predicted block intervals, condition
    numbers and MINRES bound for k = 0..kmax updates of order q."""
    gv = sol.spectrum("velocity", q, 0, 0, steps, seed=seed)
    v0 = (gv["lmin"], gv["lmax"])
    lvl = schur_level_for(v0, 2)
    gs = sol.spectrum("schur", 2, 0, lvl, steps, seed=seed + 1)
    s0 = (gs["lmin"], gs["lmax"])
    out = {"velocity_0": v0, "schur_0": s0, "schur_level": lvl, "k": []}
    for k in range(kmax + 1):
        v = hyperpower_interval(*v0, q, k)
        s = hyperpower_interval(*s0, q, k)
        neg, pos = saddle_intervals(v, s)
        out["k"].append({"k": k, "velocity": v, "schur": s, "kappa_v": v[1] / v[0],
                         "kappa_s": s[1] / s[0], "minres_bound": minres_bound(neg, pos, tol)})
    return out


def choose_iters(pred, seconds_per_iteration):
    """Depth k minimising (MINRES bound) x (measured seconds per iteration
    at depth k); ``seconds_per_iteration`` maps k to seconds."""
    best = None
    for row in pred["k"]:
        k = row["k"]
        if k not in seconds_per_iteration:
            continue
        cost = row["minres_bound"] * seconds_per_iteration[k]
        if best is None or cost < best[1]:
            best = (k, cost)
    return best[0]
