"""Differentiable compact-multigrid solve.

``u = CMGSolve.apply(kappa, f, opts)`` solves ``-div(kappa grad u) = f``
(``kappa=None``: Poisson) with zero Dirichlet data by the library's FMG and
returns the node solution.  The backward pass runs the library's adjoint
solve ``A lambda = dJ/du`` (``A`` is symmetric, so the same FMG solves it)
and its coefficient-gradient kernel:

* ``dJ/df = lambda`` (zero on the boundary, where ``u`` does not depend on
  ``f``);
* ``dJ/dkappa_c = -h^-2 2^-(d-1) sum over the edges (p, q) of cell c of
  (lambda_q - lambda_p)(u_q - u_p)``, summed over the batch.

This is the discrete adjoint of the linear system that the solver
approximates; the paper's method is used unchanged for both solves.  The
gradients are exact for the discrete system up to the solver's residual, so
for finite-difference checks run the forward and adjoint solves to
convergence (``storage="plain"``, ``vcycle_prec="fp64"`` and a few
``final_iters``).
"""
from __future__ import annotations

import math

import torch

from . import Solver

__all__ = ["CMGSolve", "solve"]


def _shape(kappa, f, dim):
    if kappa is not None:
        dim = kappa.dim()
        ncell = kappa.shape[0]
        if any(s != ncell for s in kappa.shape) or ncell & (ncell - 1):
            raise ValueError("kappa must be a cube of 2**L cells per axis")
        L = int(math.log2(ncell))
    else:
        if dim is None:
            raise ValueError("dim is required for the Poisson operator")
        N = f.shape[-1]
        L = int(math.log2(N - 1))
    N = (1 << L) + 1
    if tuple(f.shape[-dim:]) != (N,) * dim:
        raise ValueError(f"f must end in {dim} axes of {N} nodes")
    batch = f.numel() // N ** dim
    return dim, L, batch


class CMGSolve(torch.autograd.Function):
    """Autograd node around ``cmg_fmg_solve`` / ``cmg_adjoint_solve``."""

    @staticmethod
    def forward(ctx, kappa, f, opts=None, dim=None):
        opts = dict(opts or {})
        dim, L, batch = _shape(kappa, f, dim)
        op = "poisson" if kappa is None else "diffusion"
        kap = None if kappa is None else kappa.detach().to(torch.float64).contiguous()
        solver = Solver(dim, L, op=op, kappa=kap, batch=batch, **opts)
        fd = f.detach().to(torch.float64).contiguous()
        u = solver.solve(fd).reshape(f.shape)
        ctx.solver = solver
        ctx.op = op
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu):
        (u,) = ctx.saved_tensors
        solver = ctx.solver
        want_k = ctx.op == "diffusion" and ctx.needs_input_grad[0]
        lam, gk = solver.adjoint(u, gu.to(torch.float64).contiguous(), want_grad=want_k)
        solver.close()
        ctx.solver = None
        gf = lam.reshape(u.shape) if ctx.needs_input_grad[1] else None
        return (gk if want_k else None), gf, None, None


def solve(f, kappa=None, dim=None, **opts):
    """Differentiable solve; ``opts`` are :func:`paper_2511_19036_amd.options` keys."""
    return CMGSolve.apply(kappa, f, opts, dim)
