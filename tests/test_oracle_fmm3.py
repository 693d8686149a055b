"""Pins of the 3-D oracle (oracle.fmm3) to what mathematics fixes: library
3j symbols, quadrature of spherical-harmonic products, the closed-form Green's
function, direct expansions of point sources, brute-force sums and the
partition of the far and near fields over the oct-tree."""

import math

import numpy as np
import pytest

from oracle import fmm3 as f


def test_wigner3j_against_library():
    wigner = pytest.importorskip("sympy.physics.wigner")
    cases = [(1, 1, 0, 0, 0, 0), (2, 1, 1, 1, -1, 0), (3, 2, 1, -2, 1, 1), (4, 4, 2, 2, -1, -1),
             (5, 3, 4, 0, 0, 0), (6, 5, 3, -3, 2, 1), (7, 6, 9, 4, -5, 1), (2, 2, 2, 1, 1, -2)]
    for c in cases:
        assert f.wigner3j(*c) == pytest.approx(float(wigner.wigner_3j(*c)), abs=1e-14)
    assert f.wigner3j(1, 1, 3, 0, 0, 0) == 0.0  # triangle rule
    assert f.wigner3j(2, 2, 2, 1, 1, 1) == 0.0  # m sum


def _sphere_quadrature(nq):
    x, w = np.polynomial.legendre.leggauss(nq)
    th = np.arccos(x)
    ph = 2 * np.pi * np.arange(2 * nq) / (2 * nq)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    W = np.outer(w, np.full(2 * nq, 2 * np.pi / (2 * nq)))
    return TH, PH, W


def test_gaunt_against_quadrature():
    from scipy.special import sph_harm_y
    TH, PH, W = _sphere_quadrature(16)
    for (n1, m1, l, mu, n, m) in [(2, 1, 2, 0, 2, 1), (3, -2, 4, -1, 2, -1), (1, 0, 1, 0, 0, 0),
                                  (4, 3, 5, 2, 3, 1), (5, -5, 7, -3, 4, -2), (3, 1, 1, 1, 2, 0)]:
        ref = np.sum(W * np.conj(sph_harm_y(n1, m1, TH, PH)) * sph_harm_y(l, mu, TH, PH) * sph_harm_y(n, m, TH, PH))
        assert f.gaunt(n1, m1, l, mu, n, m) == pytest.approx(ref.real, abs=1e-13)
        assert abs(ref.imag) < 1e-13
    assert f.gaunt(2, 1, 2, 1, 2, 1) == 0.0  # m' != mu + m


def test_addition_theorem_reproduces_green():
    k = 10.0
    c = np.array([0.1, -0.2, 0.05])
    for x, y in [((0.5, 0.3, -0.2), (0.05, -0.08, 0.1)), ((-0.4, 0.2, 0.6), (0.2, -0.1, 0.0))]:
        x, y = np.asarray(x), np.asarray(y)
        G = f.green3(np.linalg.norm(x - y), k)
        s = 1j * k * f.basis_S(40, (x - c)[None], k)[0] @ np.conj(f.basis_R(40, (y - c)[None], k)[0])
        assert abs(s - G) <= 1e-12 * abs(G)


def test_translations_match_direct_expansions():
    k = 10.0
    # M2M: a source near a child centre, shifted to the parent centre
    cc, cp = np.array([0.1, 0.1, -0.1]), np.zeros(3)
    y = cc + np.array([0.02, -0.03, 0.01])
    Mc = f.p2m(y[None], np.array([1.0 - 0.5j]), cc, k, 20)
    Md = f.p2m(y[None], np.array([1.0 - 0.5j]), cp, k, 6)
    Mp = f.translation(cp - cc, k, 6, 20, "RR") @ Mc
    assert np.abs(Mp - Md).max() <= 1e-12 * np.abs(Md).max()
    # M2L: a well-separated pair of boxes
    cs, ct = np.zeros(3), np.array([0.5, 0.25, -0.25])
    y = cs + np.array([0.03, 0.02, -0.04])
    Ms = f.p2m(y[None], np.array([2.0]), cs, k, 25)
    Lt = f.translation(ct - cs, k, 6, 25, "SR") @ Ms
    Ld = f.p2l(y, 2.0, ct, k, 6)
    assert np.abs(Lt - Ld).max() <= 1e-12 * np.abs(Ld).max()
    # L2L: a local expansion moved to a child centre
    cch = ct + np.array([0.05, -0.05, 0.05])
    Lc = f.translation(cch - ct, k, 6, 25, "RR") @ f.p2l(y, 2.0, ct, k, 25)
    Ld = f.p2l(y, 2.0, cch, k, 6)
    assert np.abs(Lc - Ld).max() <= 1e-10 * np.abs(Ld).max()
    # the multipole and local fields themselves
    x = ct + np.array([0.01, 0.02, 0.0])
    G = 2.0 * f.green3(np.linalg.norm(x - y), k)
    assert abs(f.m2p(Ms, x[None], cs, k, 25)[0] - G) <= 1e-10 * abs(G)
    assert abs(f.l2p(f.p2l(y, 2.0, ct, k, 25), x[None], ct, k, 25)[0] - G) <= 1e-10 * abs(G)


def test_direct_sum3_brute_force():
    rng = np.random.default_rng(5)
    pts = rng.random((7, 3))
    pts[6] = pts[2]  # a coincident pair adds nothing
    q = rng.standard_normal(7) + 1j * rng.standard_normal(7)
    k = 4.0
    ref = np.zeros(7, dtype=complex)
    for i in range(7):
        for j in range(7):
            r = math.dist(pts[i], pts[j])
            if r > 0:
                ref[i] += q[j] * complex(math.cos(k * r), math.sin(k * r)) / (4 * math.pi * r)
    np.testing.assert_allclose(f.direct_sum3(pts, q, k, chunk=3), ref, rtol=1e-14, atol=0)


def test_interaction_lists_partition_the_leaves():
    # every (target leaf, source leaf) pair is covered exactly once: by P2P
    # (neighbours at the leaf level) or by one M2L at the coarsest level where
    # the ancestors are well separated
    L = 3
    nb = 2 ** L
    rng = np.random.default_rng(1)
    for t in [np.array([0, 0, 0]), np.array([7, 3, 4]), rng.integers(0, nb, 3), rng.integers(0, nb, 3)]:
        count = np.zeros((nb, nb, nb), dtype=int)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    s = t + (dx, dy, dz)
                    if np.all(s >= 0) and np.all(s < nb):
                        count[tuple(s)] += 1
        for l in range(2, L + 1):
            tl = t >> (L - l)
            w = 2 ** (L - l)
            for d in f.interaction_offsets(tuple(int(v) for v in tl % 2)):
                s = tl - np.asarray(d)
                if np.any(s < 0) or np.any(s >= 2 ** l):
                    continue
                count[s[0] * w:(s[0] + 1) * w, s[1] * w:(s[1] + 1) * w, s[2] * w:(s[2] + 1) * w] += 1
        assert count.min() == 1 and count.max() == 1
    assert len(f.interaction_offsets((0, 1, 0))) == 189


def test_fmm3_converges_to_direct_sum():
    rng = np.random.default_rng(2)
    N = 1200
    pts = rng.random((N, 3))
    q = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    k = 10.0
    d = f.direct_sum3(pts, q, k)
    errs = []
    for p in (2, 4):
        phi = f.fmm3_apply(pts, q, k, p, leaf=16)
        errs.append(np.linalg.norm(phi - d) / np.linalg.norm(d))
    assert errs[1] < errs[0] / 4 and errs[1] < 3e-4
    # a shifted, scaled root box and a lower wavenumber
    pts2 = 2.0 * rng.random((600, 3)) - 1.0
    q2 = rng.standard_normal(600) + 0j
    d2 = f.direct_sum3(pts2, q2, 3.0)
    phi2 = f.fmm3_apply(pts2, q2, 3.0, 4, leaf=8, origin=(-1.0, -1.0, -1.0), side=2.0)
    assert np.linalg.norm(phi2 - d2) / np.linalg.norm(d2) < 2e-3


def test_fmm3_one_leaf_is_the_direct_sum():
    rng = np.random.default_rng(3)
    pts = rng.random((50, 3))
    q = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    np.testing.assert_allclose(f.fmm3_apply(pts, q, 5.0, 4, leaf=0), f.direct_sum3(pts, q, 5.0), rtol=1e-15)
    assert f.tree_depth3(1000, 16) == 2 and f.tree_depth3(2 ** 20, 64) == 5
    assert f.level_orders3(10.0, 6, 5) == [14, 10, 8, 7, 6, 6]
