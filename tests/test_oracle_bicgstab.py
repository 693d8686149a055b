"""Pins of the CPU BiCGSTAB (oracle.bicgstab): the sparse-direct solution, one iteration
with the exact inverse as preconditioner, a manufactured plane wave with the
BEM preconditioner, and the zero right-hand side."""
import numpy as np
from scipy.sparse.linalg import spsolve, splu

from oracle import bem, bicgstab, fd


def test_against_sparse_direct_unpreconditioned():
    n, k = 10, 2.0
    A = fd.matrix(n, k * k)
    rng = np.random.default_rng(71)
    b = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    x, info = bicgstab.bicgstab(lambda v: A @ v, lambda v: v, b, rtol=1e-10)
    assert info["converged"]
    ref = spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - ref) < 1e-7 * np.linalg.norm(ref)


def test_exact_preconditioner_one_iteration():
    n, k = 14, 11.0
    A = fd.matrix(n, k * k)
    lu = splu(A.tocsc())
    b = np.random.default_rng(2).standard_normal(n * n) + 0j
    x, info = bicgstab.bicgstab(lambda v: A @ v, lu.solve, b, rtol=1e-10)
    assert info["iters"] == 1 and info["converged"]


def test_bem_preconditioned_plane_wave():
    n, k = 20, 14.0
    A = fd.matrix(n, k * k)
    xo = bem.interior_nodes(n)
    u = np.exp(1j * k * (xo[:, 0] * np.cos(0.4) + xo[:, 1] * np.sin(0.4)))
    b = A @ u
    Minv = bem.precond_matrix(n, k)
    x, info = bicgstab.bicgstab(lambda v: A @ v, lambda v: Minv @ v, b, rtol=1e-8)
    assert info["converged"] and info["rel_res"] <= 1e-8
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - u) <= cond * 1e-8 * np.linalg.norm(u)


def test_zero_rhs():
    A = fd.matrix(5, 1.0)
    x, info = bicgstab.bicgstab(lambda v: A @ v, lambda v: v, np.zeros(25, complex))
    assert info["converged"] and np.all(x == 0)
