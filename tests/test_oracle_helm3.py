"""Pins of the 3-D model problem's oracle (oracle.helm3): the 7-point
matrix's eigenpairs, closed forms of the cell self term, a brute-force
preconditioner sum, and a preconditioned solve against sparse direct."""

import math

import numpy as np
import scipy.sparse.linalg as spla

from oracle import fgmres, fmm3, helm3


def test_matrix3_eigenpairs_and_one_node():
    n, k = 5, 3.0
    h = 1.0 / (n + 1)
    A = helm3.matrix3(n, k * k)
    xyz = helm3.grid3(n)
    for (a, b, c) in [(1, 1, 1), (2, 3, 1), (5, 4, 2)]:
        v = np.sin(math.pi * a * xyz[:, 0]) * np.sin(math.pi * b * xyz[:, 1]) * np.sin(math.pi * c * xyz[:, 2])
        lam = sum(4.0 / h ** 2 * math.sin(math.pi * m * h / 2) ** 2 for m in (a, b, c)) - k * k
        np.testing.assert_allclose(A @ v, lam * v, rtol=1e-12, atol=1e-10)
    A1 = helm3.matrix3(1, 2.0)
    assert abs(A1[0, 0] - (6.0 / 0.25 - 2.0)) < 1e-12
    # x fastest: node 1 is (2h, h, h)
    np.testing.assert_allclose(xyz[1], [2 * h, h, h])


def test_self_term3_closed_forms():
    # k -> 0: the potential at the centre of a unit-density cube of side h is
    # h^2 (3 ln((sqrt3 + 1)/(sqrt3 - 1)) - pi/2), divided by 4 pi for G
    h = 0.1
    s3 = math.sqrt(3.0)
    c0 = h * h * (3.0 * math.log((s3 + 1) / (s3 - 1)) - math.pi / 2) / (4.0 * math.pi)
    c = helm3.self_term3(1e-7, h)
    assert abs(c.real - c0) <= 1e-12 * c0
    # the imaginary part is the integral of sin(k r) / (4 pi r):
    # k h^3 / (4 pi) - k^3 h^5 / (96 pi) + O(k^5 h^7) (moments of the cube)
    for k in (0.5, 2.0):
        c = helm3.self_term3(k, h)
        im = k * h ** 3 / (4 * math.pi) - k ** 3 * h ** 5 / (96 * math.pi)
        assert abs(c.imag - im) <= 1e-3 * (k * h) ** 4 * k * h ** 3
    # scaling: c(k, h) = h^2 c(k h, 1)
    assert abs(helm3.self_term3(3.0, 0.2) - 0.04 * helm3.self_term3(0.6, 1.0)) < 1e-14


def test_precond3_brute_force():
    n, k = 2, 4.0
    h = 1.0 / 3
    xyz = helm3.grid3(n)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(8) + 1j * rng.standard_normal(8)
    c = helm3.self_term3(k, h)
    ref = np.zeros(8, dtype=complex)
    for i in range(8):
        ref[i] = c * r[i]
        for j in range(8):
            if i != j:
                d = math.dist(xyz[i], xyz[j])
                ref[i] += h ** 3 * r[j] * complex(math.cos(k * d), math.sin(k * d)) / (4 * math.pi * d)
    np.testing.assert_allclose(helm3.precond3_apply(n, k, r), ref, rtol=1e-13)


def test_precond3_fmm_form_matches_dense_and_solve():
    n, k = 7, 3.0
    rng = np.random.default_rng(4)
    r = rng.standard_normal(n ** 3) + 1j * rng.standard_normal(n ** 3)
    zd = helm3.precond3_apply(n, k, r)
    zf = helm3.precond3_apply_fmm(n, k, r, 8, 8)
    assert np.linalg.norm(zf - zd) / np.linalg.norm(zd) < 1e-4
    # the preconditioned solve of A u = -1 reaches the sparse-direct solution
    A = helm3.matrix3(n, k * k)
    b = -np.ones(n ** 3, dtype=complex)
    x, info = fgmres.fgmres(lambda v: A @ v, lambda v: helm3.precond3_apply(n, k, v), b, restart=30, rtol=1e-8)
    xs = spla.spsolve(A.tocsc(), b)
    assert info["converged"] and np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-6
    # and it helps: fewer iterations than without a preconditioner
    _, info0 = fgmres.fgmres(lambda v: A @ v, lambda v: v, b, restart=30, rtol=1e-8)
    assert info["iters"] < info0["iters"]


def test_precond3_at_sampled_nodes_equals_dense():
    n, k = 5, 3.0
    rng = np.random.default_rng(8)
    r = rng.standard_normal(n ** 3) + 1j * rng.standard_normal(n ** 3)
    idx = np.array([0, 7, 62, 124])
    np.testing.assert_allclose(helm3.precond3_apply_at(n, k, r, idx), helm3.precond3_apply(n, k, r)[idx],
                               rtol=1e-14, atol=0)
