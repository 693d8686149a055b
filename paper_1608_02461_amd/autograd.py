"""Differentiable FMM-preconditioned Helmholtz solve.

``HelmholtzSolve.apply(k2, f, solver, restart, rtol, maxit)`` returns
u = A(k2)^{-1} f, where A(k2) = -Laplace_h - diag(k2) is the 5-point operator
of the solver's grid and the solve is the library's right-preconditioned
FGMRES with the FMM-BEM preconditioner (fixed wavenumber k0).

Backward (PyTorch's convention: the incoming gradient is
g = dL/dRe(u) + i dL/dIm(u)).  With dA/dk2_x = -e_x e_x^T,

    A^H mu = g                       (one adjoint solve, same preconditioner)
    dL/dk2 = Re(conj(mu) * u)        dL/df = mu

A is real symmetric for a real k2 field (A^H = A^T = A) and the BEM
preconditioner is complex symmetric, so the adjoint solve is the same FGMRES
run with the transpose flag.  Equivalently lambda = -conj(mu) solves
A^T lambda = -conj(g) and dL/dk2 = -Re(lambda * u).

Both solves must reach rtol (a solve that stops at maxit raises), since a
gradient from an unconverged state is meaningless.  All arithmetic runs in the
library; this module only routes tensors.
"""

import torch

from . import hfmm


class HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, k2, f, solver, restart=200, rtol=1e-10, maxit=5000):
        if k2.dtype != torch.float64 or f.dtype != torch.complex128:
            raise TypeError("k2 must be float64 and f complex128")
        solver.set_k2(k2=k2.detach().contiguous())
        u, info = solver.solve(f.detach(), restart=restart, rtol=rtol, maxit=maxit, strict=True)
        ctx.solver = solver
        ctx.opts = (restart, rtol, maxit)
        ctx.info = info
        ctx.save_for_backward(k2.detach(), u)
        return u

    @staticmethod
    def backward(ctx, g):
        k2, u = ctx.saved_tensors
        restart, rtol, maxit = ctx.opts
        solver = ctx.solver
        solver.set_k2(k2=k2)
        mu, _ = solver.solve(g.contiguous(), restart=restart, rtol=rtol, maxit=maxit, transpose=True, strict=True)
        grad_k2 = (torch.conj(mu) * u).real if ctx.needs_input_grad[0] else None
        grad_f = mu if ctx.needs_input_grad[1] else None
        return grad_k2, grad_f, None, None, None, None


def helmholtz_solve(k2, f, solver, restart=200, rtol=1e-10, maxit=5000):
    return HelmholtzSolve.apply(k2, f, solver, restart, rtol, maxit)


def expand_blocks(kb, n):
    """k2 at the n*n nodes from an (nb, nb) block field (block rows follow y)."""
    nb = kb.shape[0]
    s = n // nb
    return kb.repeat_interleave(s, 0).repeat_interleave(s, 1).reshape(-1)
