"""Differentiable free-space solve: torch.autograd.Function over hp_solve /
hp_solve_adjoint.

The solve map f -> (psi, d psi) is linear, so its vector-Jacobian product is
the transposed map applied to the upstream gradients, which the library runs
as its own pass sequence (hp_solve_adjoint): the Green's convolution is
symmetric, the spectral curl symmetric and the gradient's transpose is minus
the divergence.  Nothing is saved for backward.
"""
import torch


class SpectralPoisson(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver, *f):
        src = list(f) if solver.ncomp == 3 else f[0]
        psi, der = solver.solve(src)
        ctx.solver = solver
        return tuple(psi) + tuple(der)

    @staticmethod
    def backward(ctx, *grads):
        s = ctx.solver
        g_psi = grads[:s.ncomp]
        g_der = grads[s.ncomp:]
        gp = None if all(g is None for g in g_psi) else [
            (g if g is not None else torch.zeros(s.out_shape, dtype=s.dtype, device=s.device)).contiguous()
            for g in g_psi]
        gd = None if (len(g_der) == 0 or all(g is None for g in g_der)) else [
            (g if g is not None else torch.zeros(s.out_shape, dtype=s.dtype, device=s.device)).contiguous()
            for g in g_der]
        if gp is None and gd is None:
            return (None,) + (None,) * s.ncomp
        grad_f = s.adjoint(gp, gd)
        return (None,) + tuple(grad_f)


def poisson_solve(solver, f):
    """Differentiable solve.  f: tensor (scalar) or list of 3 tensors.
    Returns (psi list, derivative list)."""
    fs = list(f) if solver.ncomp == 3 else [f]
    outs = SpectralPoisson.apply(solver, *fs)
    return list(outs[:solver.ncomp]), list(outs[solver.ncomp:])
