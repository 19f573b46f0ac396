"""Krylov solvers of the oracle (Sec. 5 runs MINRES to a relative tolerance
of 1e-8; FGMRES serves the inexact, mixed-precision preconditioner).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* ``minres``: preconditioned MINRES for a symmetric (indefinite) matrix and
  a symmetric positive definite preconditioner: the Lanczos process in the
  P^{-1} inner product, with the tridiagonal least-squares problem solved
  by Givens rotations and a three-term update of the iterate.  It stops at
  the first iteration whose preconditioned residual norm
  ||r_j||_{P^{-1}} = sqrt(r_j^T P^{-1} r_j) (carried by the recurrence)
  is <= tol * ||b||_{P^{-1}}, with x_0 = 0.
* ``fgmres``: right-preconditioned flexible GMRES(m) with modified
  Gram-Schmidt Arnoldi and Givens rotations; the preconditioner may change
  from step to step.  It stops when the Arnoldi residual estimate is
  <= tol * ||b||_2 and reports the true residual.
"""
import numpy as np


class Result:
    def __init__(self, x, iters, converged, history, true_relres):
        self.x = x
        self.iters = iters
        self.converged = converged
        self.history = history
        self.true_relres = true_relres


def minres(Kop, Minv, b, tol=1e-8, maxit=1000, callback=None):
    """Preconditioned MINRES from x_0 = 0.

    Kop(x) -> K x, Minv(r) -> P^{-1} r (SPD).  Returns ``Result`` with
    ``history`` the relative preconditioned residual norms, one per
    iteration (index 0 is the start).
    """
    n = b.size
    x = np.zeros(n)
    v_old = np.zeros(n)
    v = b.copy()
    z = Minv(v)
    gamma = np.sqrt(z @ v)
    if not np.isfinite(gamma) or gamma < 0:
        raise FloatingPointError("preconditioner is not positive definite on b")
    gamma_old = 1.0
    beta0 = gamma
    eta = gamma
    w_old = np.zeros(n)
    w = np.zeros(n)
    c_old, c = 1.0, 1.0
    s_old, s = 0.0, 0.0
    hist = [1.0]
    it = 0
    converged = beta0 == 0.0
    while not converged and it < maxit:
        it += 1
        z = z / gamma
        Kz = Kop(z)
        delta = Kz @ z
        v_new = Kz - (delta / gamma) * v - (gamma / gamma_old) * v_old
        z_new = Minv(v_new)
        zv = z_new @ v_new
        if zv < 0:
            raise FloatingPointError("preconditioner is not positive definite")
        gamma_new = np.sqrt(zv)
        a0 = c * delta - c_old * s * gamma
        a1 = np.hypot(a0, gamma_new)
        a2 = s * delta + c_old * c * gamma
        a3 = s_old * gamma
        c_new = a0 / a1
        s_new = gamma_new / a1
        w_new = (z - a3 * w_old - a2 * w) / a1
        x = x + c_new * eta * w_new
        eta = -s_new * eta
        # shift the recurrences
        v_old, v = v, v_new
        z = z_new
        gamma_old, gamma = gamma, gamma_new
        w_old, w = w, w_new
        c_old, c = c, c_new
        s_old, s = s, s_new
        rel = abs(eta) / beta0
        hist.append(rel)
        if callback is not None:
            callback(it, x, rel)
        if rel <= tol:
            converged = True
        elif gamma_new == 0.0:
            converged = True
    r = b - Kop(x)
    return Result(x, it, converged, np.array(hist), np.linalg.norm(r) / np.linalg.norm(b))


def fgmres(Kop, precond, b, tol=1e-8, restart=50, maxit=1000):
    """Right-preconditioned flexible GMRES(restart) from x_0 = 0.

    ``precond(v, j)`` returns z_j ~= P^{-1} v for the j-th Arnoldi vector
    (the preconditioner may differ per step).  ``history`` holds the
    relative Arnoldi residual estimates.
    """
    n = b.size
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = [1.0]
    total = 0
    if bnorm == 0.0:
        return Result(x, 0, True, np.array(hist), 0.0)
    converged = False
    while total < maxit and not converged:
        r = b - Kop(x)
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        j_done = 0
        for j in range(restart):
            z = precond(V[j], total)
            Z.append(z)
            w = Kop(z)
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            rel = abs(g[j + 1]) / bnorm
            hist.append(rel)
            if rel <= tol or total >= maxit:
                break
            if hn == 0.0:
                break   # happy breakdown: the Krylov space is invariant
            V.append(w / hn)
        # back substitution for the least-squares coefficients
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:j_done]) / H[i, i]
        for i in range(j_done):
            x = x + y[i] * Z[i]
        converged = hist[-1] <= tol
    return Result(x, total, converged, np.array(hist), np.linalg.norm(b - Kop(x)) / bnorm)
