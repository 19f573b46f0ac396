"""Differentiable hyper-power Stokes solve (adjoint method).

``HyperPowerSolve.apply(beta, nu, solver, lid, tol)`` solves

    K(nu) x = [F_lid(nu) + M_V beta ; 0]

(lid-driven cavity with body-force coefficient field beta in the velocity
space, f_u = M_V beta) and returns the velocity block u of x.  Its
backward is the adjoint solve K lambda = [dL/du ; 0] with the same
preconditioned operator (K is symmetric) followed by the library's gradient
kernels: dL/dbeta = M_V lambda_u and dL/dnu = lambda_u . (F_lid - A u) / nu
(A and F_lid are linear in nu, B is nu-free).  Only x is kept from the
forward solve, not the Krylov history.

``MassMatrix.apply(u, solver)`` is y = M_V u (self-adjoint), so the L2 loss
||u_h - u_t||^2 = (u - u_t)^T M_V (u - u_t) is differentiable end to end.
"""
import torch


class HyperPowerSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, beta, nu, solver, lid=1.0, tol=1e-10):
        nu_f = float(nu)
        solver.set_nu(nu_f)
        b = solver.build_rhs([lid], beta=beta.detach().contiguous())
        x, info = solver.solve(b, tol)
        ctx.save_for_backward(x)
        ctx.solver, ctx.lid, ctx.tol, ctx.nu = solver, lid, tol, nu_f
        ctx.info = info
        return x[:solver.nV].clone()

    @staticmethod
    def backward(ctx, grad_u):
        (x,) = ctx.saved_tensors
        s = ctx.solver
        s.set_nu(ctx.nu)
        rhs = torch.zeros(s.N, dtype=torch.float64, device=x.device)
        rhs[:s.nV] = grad_u
        lam, _ = s.solve(rhs, ctx.tol)
        g_beta, g_nu = s.grad(x, lam, [ctx.lid])
        return g_beta, torch.tensor(g_nu[0], dtype=torch.float64, device=x.device), None, None, None


class MassMatrix(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, solver):
        ctx.solver = solver
        return solver.apply_MV(u.contiguous())

    @staticmethod
    def backward(ctx, g):
        return ctx.solver.apply_MV(g.contiguous()), None


def cavity_loss(beta, nu, solver, u_target, lid=1.0, tol=1e-10):
    """L = ||u_h(beta, nu) - u_t||_{L2}^2 for the cavity."""
    u = HyperPowerSolve.apply(beta, nu, solver, lid, tol)
    d = u - u_target
    return (d * MassMatrix.apply(d, solver)).sum()
