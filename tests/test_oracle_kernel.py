"""Pins of the oracle's kernel and direct sum (O-1) against values the
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
