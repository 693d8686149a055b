"""Pins of the oracle's kernel and direct sum (oracle.kernel) against values the
mathematics fixes: an independent arbitrary-precision Hankel function
(mpmath), the small-argument series (DLMF 10.8.2), the Wronskian
(DLMF 10.5.2), reciprocity G(x, y) = G(y, x), and brute force."""
import math

import mpmath
import numpy as np
import pytest
from scipy.special import hankel1, jv, yv

from oracle import kernel


@pytest.mark.parametrize("x", [1e-3, 0.05, 0.3125, 2.2, 6.6, 17.7, 54.0, 300.0])
def test_h0_against_mpmath(x):
    ref = complex(mpmath.hankel1(0, x))
    got = complex(hankel1(0, x))
    assert abs(got - ref) <= 1e-12 * abs(ref)


def test_green_is_i_over_4_h0():
    r = np.array([0.01, 0.1, 0.7])
    k = 16.0
    ref = [complex(0.25j * mpmath.hankel1(0, k * t)) for t in r]
    assert np.allclose(kernel.green(r, k), ref, rtol=1e-12, atol=0)


def test_y0_small_argument_series():
    # DLMF 10.8.2: Y0(x) = (2/pi)(ln(x/2) + gamma_E) J0(x) + (2/pi)(x^2/4) + O(x^4 ln x)
    for x in [1e-4, 1e-3, 1e-2]:
        lead = (2 / math.pi) * (math.log(x / 2) + 0.5772156649015329) * jv(0, x)
        assert abs(yv(0, x) - lead - (2 / math.pi) * x * x / 4) < 5 * x ** 4 * (1 + abs(math.log(x)))


def test_wronskian():
    x = np.linspace(0.05, 80, 200)
    w = jv(1, x) * yv(0, x) - jv(0, x) * yv(1, x)
    assert np.allclose(w, 2 / (math.pi * x), rtol=1e-11, atol=0)


def test_direct_sum_brute_force_mpmath():
    rng = np.random.default_rng(11)
    xy = rng.random((9, 2))
    q = rng.standard_normal(9) + 1j * rng.standard_normal(9)
    k = 37.0
    got = kernel.direct_sum(xy, q, k)
    for i in range(9):
        s = mpmath.mpc(0)
        for j in range(9):
            if i == j:
                continue
            r = math.hypot(*(xy[i] - xy[j]))
            s += complex(q[j]) * 0.25j * mpmath.hankel1(0, k * r)
        assert abs(got[i] - complex(s)) <= 1e-12 * abs(complex(s))


def test_reciprocity():
    rng = np.random.default_rng(12)
    xy = rng.random((300, 2))
    a = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    b = rng.standard_normal(300) + 1j * rng.standard_normal(300)
    k = 100.0
    lhs = a @ kernel.direct_sum(xy, b, k)
    rhs = b @ kernel.direct_sum(xy, a, k)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_zero_distance_pairs_add_nothing():
    xy = np.array([[0.2, 0.3], [0.2, 0.3], [0.7, 0.1]])
    q = np.array([1.0, 2.0, 3.0], dtype=complex)
    phi = kernel.direct_sum(xy, q, 5.0)
    g = kernel.green(math.hypot(0.5, 0.2), 5.0)
    assert np.isclose(phi[0], 3.0 * g) and np.isclose(phi[1], 3.0 * g)
    assert np.isclose(phi[2], (1.0 + 2.0) * g)


def test_multirhs_and_targets():
    rng = np.random.default_rng(13)
    xy = rng.random((50, 2))
    q = rng.standard_normal((50, 3)) + 1j * rng.standard_normal((50, 3))
    full = kernel.direct_sum(xy, q, 20.0)
    for c in range(3):
        assert np.allclose(full[:, c], kernel.direct_sum(xy, q[:, c], 20.0), rtol=1e-14)
    tg = rng.random((7, 2))
    sub = kernel.direct_sum(xy, q, 20.0, tgt=tg)
    assert sub.shape == (7, 3)


def test_direct_sum_parallel_equals_serial():
    """The process-pool split over target chunks (which wrote the stored
    2^20 reference) gives the serial sum row by row (to the rounding of the
    BLAS product, whose order depends on the chunk shape); a dropped, repeated
    or misplaced chunk would not."""
    rng = np.random.default_rng(13)
    src = rng.random((700, 2))
    q = rng.standard_normal(700) + 1j * rng.standard_normal(700)
    tgt = rng.random((53, 2))
    ser = kernel.direct_sum(src, q, 41.0, tgt=tgt, chunk=1)
    for workers in (1, 3, 8):
        par = kernel.direct_sum_parallel(src, q, 41.0, tgt, workers=workers)
        assert par.shape == ser.shape
        assert np.allclose(par, ser, rtol=1e-13, atol=0)
    # and one row against arbitrary precision
    s = mpmath.mpc(0)
    for j in range(700):
        r = math.hypot(tgt[5, 0] - src[j, 0], tgt[5, 1] - src[j, 1])
        s += complex(q[j]) * 0.25j * mpmath.hankel1(0, 41.0 * r)
    assert abs(par[5] - complex(s)) <= 1e-12 * abs(complex(s))


@pytest.mark.parametrize("k", [3.0, 40.0])
def test_dgreen_dn_is_the_normal_derivative(k):
    """dG/dn at the source against a central difference of G along n
    (Sec. 5.2): the sign and the factor (i k / 4) H1 follow from dH0/dx = -H1."""
    rng = np.random.default_rng(int(k))
    x = rng.random((20, 2))
    y = rng.random((20, 2)) + 1.5
    a = rng.uniform(0, 2 * np.pi, 20)
    nrm = np.stack([np.cos(a), np.sin(a)], 1)
    eps = 1e-6
    dist = lambda p, q: np.sqrt(((p - q) ** 2).sum(1))
    fdv = (kernel.green(dist(x, y + eps * nrm), k) - kernel.green(dist(x, y - eps * nrm), k)) / (2 * eps)
    got = kernel.dgreen_dn(x, y, nrm, k)
    assert np.allclose(got, fdv, rtol=1e-7, atol=1e-9)
    # mpmath value of one pair
    r = math.hypot(*(x[0] - y[0]))
    ref = complex(0.25j * k * mpmath.hankel1(1, k * r)) * float(((x[0] - y[0]) * nrm[0]).sum()) / r
    assert abs(got[0] - ref) <= 1e-12 * abs(ref)


def test_direct_sum_dipole():
    """The double-layer sum against the derivative of the single-layer sum in
    the source positions, and zero for coincident points."""
    rng = np.random.default_rng(17)
    src = rng.random((40, 2))
    a = rng.uniform(0, 2 * np.pi, 40)
    nrm = np.stack([np.cos(a), np.sin(a)], 1)
    q = rng.standard_normal((40, 2)) + 1j * rng.standard_normal((40, 2))
    tgt = rng.random((15, 2)) + np.array([0.0, 1.2])
    k, eps = 12.0, 1e-6
    fdv = (kernel.direct_sum(src + eps * nrm, q, k, tgt=tgt) - kernel.direct_sum(src - eps * nrm, q, k, tgt=tgt)) / (
        2 * eps)
    got = kernel.direct_sum_dipole(src, q, nrm, k, tgt=tgt)
    assert np.allclose(got, fdv, rtol=1e-6, atol=1e-8)
    # coincident source and target: nothing
    one = kernel.direct_sum_dipole(src[:1], q[:1, 0], nrm[:1], k, tgt=src[:1])
    assert one[0] == 0
