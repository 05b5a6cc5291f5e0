"""torch.autograd.Function over the GL solver: forward through gl_step_n, backward through
gl_adjoint (the reverse-time sweep with transposed GL weights and d psi / d gamma).

    uT = GLSolve.apply(u0, alpha, gamma, rate, problem, memory, nsteps)

u0 is a CUDA float64 tensor; alpha, gamma and rate are 0-dim tensors (any device); the
problem dict supplies the grid, dt, dx and reaction kind (its own alpha, gamma and rate
are replaced by the tensor values).  dt and dx are held fixed.  Every memory mode (adaptive
memory through the transposed schedule) and both history-sum paths.
"""
import torch

from . import gl


class GLSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, alpha, gamma, rate, problem, memory, nsteps, sum_path="gemv",
                ckpt_every=0, block_B=0):
        p = dict(problem, alpha=float(alpha), gamma=float(gamma), rate=float(rate))
        solver = gl.Solver(p, memory, u0.detach().to(torch.float64), max_steps=nsteps,
                           sum_path=sum_path, ckpt_every=ckpt_every, block_B=block_B,
                           device=u0.device)
        uT = solver.step(nsteps)
        ctx.solver = solver
        ctx.param_meta = [(t.device, t.dtype) for t in (alpha, gamma, rate)]
        ctx.u0_meta = (u0.device, u0.dtype)
        return uT

    @staticmethod
    def backward(ctx, g):
        solver = ctx.solver
        du0, dpar = solver.adjoint(g.to(torch.float64).contiguous())
        solver.close()
        ctx.solver = None
        grads = [dpar[0, i].to(device=dev, dtype=dt) for i, (dev, dt) in enumerate(ctx.param_meta)]
        return (du0.to(device=ctx.u0_meta[0], dtype=ctx.u0_meta[1]), *grads,
                None, None, None, None, None, None)


def gl_solve(u0, alpha, gamma, rate, problem, memory, nsteps, sum_path="gemv", ckpt_every=0,
             block_B=0):
    """u[nsteps] as a differentiable function of u0, alpha, gamma and the reaction rate."""
    return GLSolve.apply(u0, alpha, gamma, rate, problem, memory, nsteps, sum_path, ckpt_every,
                         block_B)
