"""Pins of the CPU FGMRES (oracle.fgmres): the defining property (true relative
residual <= tol), sparse-direct solutions, a manufactured plane wave that
solves the discrete problem exactly, a sine mode with a closed-form
solution, flexibility, and the zero right-hand side."""
import numpy as np
import pytest
from scipy.sparse.linalg import spsolve

from oracle import bem, fd, fgmres


def test_against_sparse_direct_unpreconditioned():
    n, k = 12, 3.0
    A = fd.matrix(n, k * k)
    rng = np.random.default_rng(51)
    b = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    x, info = fgmres.fgmres(lambda v: A @ v, lambda v: v, b, restart=20, rtol=1e-10)
    assert info["converged"]
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    ref = spsolve(A.tocsc(), b)
    assert np.linalg.norm(x - ref) < 1e-7 * np.linalg.norm(ref)


def test_bem_preconditioned_plane_wave():
    n, k = 24, 16.0
    A = fd.matrix(n, k * k)
    xo = bem.interior_nodes(n)
    a = 0.6
    u = np.exp(1j * k * (xo[:, 0] * np.cos(a) + xo[:, 1] * np.sin(a)))
    b = A @ u  # u solves the discrete problem exactly
    Minv = bem.precond_matrix(n, k)
    x, info = fgmres.fgmres(lambda v: A @ v, lambda v: Minv @ v, b, restart=30, rtol=1e-6)
    assert info["converged"] and info["rel_res"] <= 1e-6
    assert info["iters"] < 40
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - u) <= cond * 1e-6 * np.linalg.norm(u)


def test_sine_mode_closed_form():
    n, k = 16, 9.0
    h = 1 / (n + 1)
    xo = bem.interior_nodes(n)
    v = np.sin(np.pi * xo[:, 0]) * np.sin(2 * np.pi * xo[:, 1])
    lam = 4 / h ** 2 * (np.sin(np.pi * h / 2) ** 2 + np.sin(2 * np.pi * h / 2) ** 2) - k * k
    A = fd.matrix(n, k * k)
    x, info = fgmres.fgmres(lambda w: A @ w, lambda w: w, v.astype(complex), restart=5, rtol=1e-12)
    assert np.allclose(x, v / lam, rtol=1e-9, atol=1e-12)
    assert info["iters"] == 1


def test_flexible_preconditioner_changes_between_calls():
    n, k = 14, 12.0
    A = fd.matrix(n, k * k)
    Minv = bem.precond_matrix(n, k)
    calls = {"n": 0}

    def prec(v):
        calls["n"] += 1
        return Minv @ v if calls["n"] % 2 else v

    rng = np.random.default_rng(52)
    b = rng.standard_normal(n * n) + 0j
    x, info = fgmres.fgmres(lambda w: A @ w, prec, b, restart=40, rtol=1e-8)
    assert info["converged"]
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)


def test_zero_rhs():
    A = fd.matrix(4, 1.0)
    x, info = fgmres.fgmres(lambda w: A @ w, lambda w: w, np.zeros(16, complex))
    assert info["converged"] and np.all(x == 0)


def test_restart_counts_cycles():
    n, k = 16, 2.0  # definite: restarted GMRES converges
    A = fd.matrix(n, k * k)
    rng = np.random.default_rng(53)
    b = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    x, info = fgmres.fgmres(lambda w: A @ w, lambda w: w, b, restart=5, rtol=1e-8, maxit=5000)
    assert info["converged"] and info["restarts"] >= 2
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)
