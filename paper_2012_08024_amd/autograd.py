"""torch.autograd bindings of the solve and of the mass matrix.

Forward u = A(kappa)^{-1} M_0 f.  Backward, with the incoming gradient
g = dL/du: lambda = A^{-T} g through the same hierarchy (A is symmetric),
dL/dkappa_e = -lambda^T (dA/dkappa_e) u from the element-local kernel, and
dL/df = M_0 lambda.  All products run in the library; torch only carries the
tensors.  Both solves are strict: one that stops at max_iter raises
CdgmgError instead of returning an unconverged u, lambda or gradient.
"""
import torch


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, f, solver):
        solver.ensure_kappa(kappa)
        u, _ = solver.solve(f.detach(), strict=True)
        ctx.solver = solver
        ctx.save_for_backward(kappa, u)
        ctx.mark_non_differentiable()
        return u

    @staticmethod
    def backward(ctx, grad_u):
        solver = ctx.solver
        kappa, u = ctx.saved_tensors
        solver.ensure_kappa(kappa)
        lam, _ = solver.solve_transpose(grad_u.contiguous(), strict=True)
        gk = solver.grad_kappa(u, lam) if ctx.needs_input_grad[0] else None
        gf = solver.apply_mass(lam) if ctx.needs_input_grad[1] else None
        return gk, gf, None


class _Mass(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, solver):
        ctx.solver = solver
        return solver.apply_mass(x.detach())

    @staticmethod
    def backward(ctx, g):
        return ctx.solver.apply_mass(g.contiguous()), None


def solve(solver, kappa, f):
    """Differentiable u(kappa, f) (float64 tensors on the GPU)."""
    return _Solve.apply(kappa, f, solver)


def apply_mass(solver, x):
    """Differentiable y = M_0 x."""
    return _Mass.apply(x, solver)


def mass_misfit(solver, u, u_target):
    """L = 1/2 (u - u_t)^T M_0 (u - u_t)."""
    r = u - u_target
    return 0.5 * torch.dot(r, apply_mass(solver, r))
