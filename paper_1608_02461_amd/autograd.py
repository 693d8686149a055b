"""Differentiable FMM-preconditioned Helmholtz solve.

``HelmholtzSolve.apply(kb, f, solver, restart, rtol, maxit)`` returns
u = A(k2)^{-1} f, where k2 is constant on the square blocks of ``kb``
(nb x nb, block rows following y), A(k2) = -Laplace_h - diag(k2) is the
5-point operator of the solver's grid and the solve is the library's
right-preconditioned FGMRES with the FMM-BEM preconditioner (fixed
wavenumber k0).

Backward (PyTorch's convention: the incoming gradient is
g = dL/dRe(u) + i dL/dIm(u)).  With dA/dk2_x = -e_x e_x^T,

    A^H mu = g                       (one adjoint solve, same preconditioner)
    dL/dkb_b = sum_{x in b} Re(conj(mu_x) u_x)        dL/df = mu

A is real symmetric for a real k2 field (A^H = A^T = A) and the BEM
preconditioner is complex symmetric, so the adjoint solve is the same FGMRES
run with the transpose flag.  Equivalently lambda = -conj(mu) solves
A^T lambda = -conj(g) and dL/dk2 = -Re(lambda * u).

The library expands the block field (``hfmm_solver_set_k2_blocks``) and forms
the gradient product and its block sums (``hfmm_k2_gradient``); this module
only routes tensors.  Both solves must reach rtol (a solve that stops at
maxit raises), since a gradient from an unconverged state is meaningless.
"""

import torch

from . import hfmm


class HelmholtzSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kb, f, solver, restart=200, rtol=1e-10, maxit=5000):
        if kb.dtype != torch.float64 or f.dtype != torch.complex128:
            raise TypeError("kb must be float64 and f complex128")
        if kb.dim() != 2 or kb.shape[0] != kb.shape[1]:
            raise ValueError("kb must be a square (nb, nb) block field")
        kb = kb.detach().contiguous()
        solver.set_k2_blocks(kb)
        u, info = solver.solve(f.detach(), restart=restart, rtol=rtol, maxit=maxit, strict=True)
        ctx.solver = solver
        ctx.opts = (restart, rtol, maxit)
        ctx.info = info
        ctx.save_for_backward(kb, u)
        return u

    @staticmethod
    def backward(ctx, g):
        kb, u = ctx.saved_tensors
        restart, rtol, maxit = ctx.opts
        solver = ctx.solver
        solver.set_k2_blocks(kb)
        mu, _ = solver.solve(g.contiguous(), restart=restart, rtol=rtol, maxit=maxit, transpose=True, strict=True)
        grad_kb = hfmm.hfmm_k2_gradient(solver.n, u, mu, kb.shape[0]) if ctx.needs_input_grad[0] else None
        grad_f = mu if ctx.needs_input_grad[1] else None
        return grad_kb, grad_f, None, None, None, None


def helmholtz_solve(kb, f, solver, restart=200, rtol=1e-10, maxit=5000):
    """u = A(k2(kb))^{-1} f, differentiable in the block field kb and in f."""
    return HelmholtzSolve.apply(kb, f, solver, restart, rtol, maxit)
