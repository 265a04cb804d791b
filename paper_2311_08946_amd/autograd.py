"""torch.autograd.Function around assemble + solve, with the hand-written
adjoint of the library as its backward.

Forward:  u = C(theta)^-1 r(theta), theta = node samples of the coefficients
(a_xx, a_xy, a_yy, b_x, b_y, c, f on the floating circles' collocation nodes).
Backward: lambda = C^-T dL/du (BiCGStab on the transpose), then
pdd_assemble_G_backward gives dL/dtheta.  Monte Carlo and boundary rows do not
depend on theta.
"""
from __future__ import annotations

import torch

from . import binding

NAMES = ("axx", "axy", "ayy", "bx", "by", "c", "f")


def node_samples(cover, problem, device=None):
    """The problem's seven fields at the cover's collocation nodes (device)."""
    device = device or torch.device("cuda", torch.cuda.current_device())
    xy, _, _ = cover.nodes()
    xy_d = torch.tensor(xy, dtype=torch.float64, device=device)
    return {k: binding.eval_field(problem, k, xy_d) for k in NAMES}


class PDDSolve(torch.autograd.Function):
    """u = solve(assemble(theta)); gradients w.r.t. the seven sample tensors."""

    @staticmethod
    def forward(ctx, axx, axy, ayy, bx, by, c, f, cover, problem, mc, rtol):
        samples = dict(zip(NAMES, (t.detach().contiguous() for t in (axx, axy, ayy, bx, by, c, f))))
        sysm = binding.System(cover, problem, mc, samples=samples, keep_factors=True)
        u, info = sysm.solve(rtol=rtol)
        ctx.sysm = sysm
        ctx.rtol = rtol
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu):
        (u,) = ctx.saved_tensors
        lam, _ = ctx.sysm.solve(rhs=gu.contiguous().to(torch.float64), transpose=True, rtol=ctx.rtol)
        g = ctx.sysm.backward(u, lam)
        grads = tuple(g[k] if ctx.needs_input_grad[t] else None for t, k in enumerate(NAMES))
        return grads + (None, None, None, None)


def solve(samples, cover, problem, mc, rtol=1e-12):
    return PDDSolve.apply(*(samples[k] for k in NAMES), cover, problem, mc, rtol)
