"""Pins of the dense BEM preconditioner (oracle.bem): the self terms against
independent quadrature, the boundary geometry, the paper's helm_fixed exact
solution reproduced by z = M^{-1} f as h -> 0, complex symmetry of M^{-1},
and the FMM form of the same preconditioner converging to the dense one."""
import json
import math
import os

import mpmath
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import hankel1

from oracle import bem

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def test_gamma_matches_paper():
    g = GOLD["gamma_exp_euler"]
    assert abs(bem.EULER_GAMMA_EXP - g["value"]) < 10 ** (-(g["digits"] - 1))


def _element_integral(k, w):
    # int_{-w/2}^{w/2} H0(k|s|) ds = 2 int_0^{w/2}; Y0 has a log singularity at 0 (quad 'alg' weight handles it)
    re = 2 * quad(lambda s: hankel1(0, k * s).real, 0, w / 2, epsabs=0, epsrel=1e-13, limit=200)[0]
    im = 2 * quad(lambda s: hankel1(0, k * s).imag, 0, w / 2, epsabs=0, epsrel=1e-12, limit=200)[0]
    return re + 1j * im


@pytest.mark.parametrize("kw,bound", [(0.05, 1e-4), (0.246, 2e-3), (0.3, 2.5e-3), (0.389, 4e-3)])
def test_boundary_self_term_is_small_argument_form(kw, bound):
    """The paper's analytic diagonal is the small-argument integral of H0
    over the element; its error against quadrature shrinks as k w -> 0."""
    k = 16.0
    w = kw / k
    exact = 0.25j * _element_integral(k, w)
    got = bem.boundary_self(k, w)
    assert abs(got - exact) <= bound * abs(exact)


def test_volume_self_term_against_2d_quadrature():
    mpmath.mp.dps = 16
    k, h = 16.0, 1.0 / 65
    f = lambda x, y: mpmath.hankel1(0, k * mpmath.sqrt(x * x + y * y))
    ref = complex(0.25j * 4 * mpmath.quad(f, [0, h / 2], [0, h / 2]))
    assert abs(bem.volume_self(k, h) - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("k,h", [(16.0, 1 / 65), (307.5, 1 / 1025), (100.0, 1 / 257)])
def test_volume_self_term_small_argument(k, h):
    # (i/4) h^2 [1 + i(2/pi)(ln(kh/2) + gamma_E + <ln r> over the unit square)] within 1%
    mean_ln = -1.0611754  # mean of ln|x| over the centred unit square, checked below
    small = 0.25j * h * h * (1 + 1j * (2 / math.pi) * (math.log(k * h / 2) + 0.5772156649015329 + mean_ln))
    got = bem.volume_self(k, h)
    assert abs(got - small) < 1e-2 * abs(got)


def test_mean_log_over_unit_square():
    v = quad(lambda x: quad(lambda y: 0.5 * math.log(x * x + y * y), 0, 0.5)[0], 0, 0.5)[0] * 4
    assert abs(v - (-1.0611754)) < 1e-6


def test_boundary_geometry():
    n = 7
    xg = bem.boundary_nodes(n)
    h = 1 / (n + 1)
    assert xg.shape == (4 * (n + 1), 2)
    corners = np.array([[0, 0], [1, 0], [0, 1], [1, 1]])
    assert np.min(np.linalg.norm(xg[:, None] - corners[None], axis=2)) == pytest.approx(h / 2)
    on_edge = (xg == 0) | (xg == 1)
    assert np.all(on_edge.sum(axis=1) == 1)
    assert len({tuple(p) for p in np.round(xg, 12)}) == xg.shape[0]


def test_interior_nodes_order():
    xo = bem.interior_nodes(3)
    assert np.allclose(xo[:4], [[0.25, 0.25], [0.5, 0.25], [0.75, 0.25], [0.25, 0.5]])


def test_helm_fixed_exact_solution():
    """Sec. 6, first model problem: z = M^{-1} f reproduces sin(pi x) sin(2 pi y)
    to within the discretisation error, which falls as h falls."""
    errs = []
    k = 15.0
    for n in (15, 31):
        xo = bem.interior_nodes(n)
        u = np.sin(np.pi * xo[:, 0]) * np.sin(2 * np.pi * xo[:, 1])
        f = (5 * np.pi ** 2 - k * k) * u
        z = bem.precond_apply(n, k, f)
        errs.append(np.linalg.norm(z - u) / np.linalg.norm(u))
    assert errs[0] < 0.05 and errs[1] < 0.012 and errs[1] < errs[0] / 3


def test_precond_symmetric_and_consistent():
    n, k = 12, 20.0
    Minv = bem.precond_matrix(n, k)
    assert np.abs(Minv - Minv.T).max() < 1e-12 * np.abs(Minv).max()
    rng = np.random.default_rng(31)
    r = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    assert np.allclose(Minv @ r, bem.precond_apply(n, k, r), rtol=1e-11, atol=1e-14)


def test_fmm_form_converges_to_dense():
    n, k = 20, 16.0
    rng = np.random.default_rng(32)
    r = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    ref = bem.precond_apply(n, k, r)
    e = [np.linalg.norm(bem.precond_apply_fmm(n, k, r, p, 8) - ref) / np.linalg.norm(ref) for p in (3, 6, 20)]
    assert e[0] > e[1] > e[2] and e[2] < 1e-10


def _helm2(mu):
    """The paper's inhomogeneous-Dirichlet problem (Sec. 6, eq. helm2) with
    kappa = mu sqrt(2), in the sign convention -Laplace(u) - k^2 u = f (the
    paper's right-hand side negated): exact u = x^2 sin(mu x) cos(mu y)."""
    def u(P):
        return P[:, 0] ** 2 * np.sin(mu * P[:, 0]) * np.cos(mu * P[:, 1])

    def f(P):
        return -(2 * np.sin(mu * P[:, 0]) * np.cos(mu * P[:, 1]) + 4 * mu * P[:, 0] * np.cos(mu * P[:, 0]) *
                 np.cos(mu * P[:, 1]))
    return mu * math.sqrt(2.0), u, f


@pytest.mark.parametrize("mu", [1.0, 4.0])
def test_dirichlet_solve_reproduces_helm2(mu):
    """With f and the boundary values of the exact solution, the boundary
    equation (1/2 delta and double layer) and the interior equation give u
    with an error that falls with h; a wrong sign or a missing double layer
    leaves an O(1) error."""
    k, u, f = _helm2(mu)
    errs = []
    for n in (15, 31):
        xo, xg = bem.interior_nodes(n), bem.boundary_nodes(n)
        us = bem.dirichlet_solve(n, k, f(xo), u(xg))
        errs.append(np.linalg.norm(us - u(xo)) / np.linalg.norm(u(xo)))
    assert errs[1] < 0.5 * errs[0]
    assert errs[1] < (5e-3 if mu == 1.0 else 2e-2)


def test_dirichlet_solve_plane_wave_and_zero_data():
    """f = 0 with the boundary values of a plane wave reproduces the wave
    inside (error falling with h); g = 0 is the preconditioner apply."""
    k, a = 10.0, 0.3
    errs = []
    for n in (15, 31):
        xo, xg = bem.interior_nodes(n), bem.boundary_nodes(n)
        pw = lambda P: np.exp(1j * k * (P[:, 0] * math.cos(a) + P[:, 1] * math.sin(a)))
        us = bem.dirichlet_solve(n, k, np.zeros(n * n), pw(xg))
        errs.append(np.linalg.norm(us - pw(xo)) / np.linalg.norm(pw(xo)))
    assert errs[1] < 0.5 * errs[0] and errs[1] < 0.2
    n = 12
    r = np.random.default_rng(3).standard_normal(n * n) + 0j
    assert np.allclose(bem.dirichlet_solve(n, 9.0, r, np.zeros(4 * (n + 1))), bem.precond_apply(n, 9.0, r),
                       rtol=1e-12, atol=1e-14)


def test_boundary_normals_are_outward():
    n = 7
    xg, nrm = bem.boundary_nodes(n), bem.boundary_normals(n)
    out = xg + 1e-3 * nrm
    assert np.all(((out < 0) | (out > 1)).any(axis=1))


def test_fmm_form_targets_and_dirichlet_data():
    """The FMM form at a subset of targets equals the full FMM form there, and
    with Dirichlet data it converges to the dense solution as p grows."""
    n, k, leaf = 20, 14.0, 8
    rng = np.random.default_rng(12)
    r = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    g = rng.standard_normal(4 * (n + 1)) + 1j * rng.standard_normal(4 * (n + 1))
    tg = np.sort(rng.choice(n * n, 37, replace=False))
    full = bem.precond_apply_fmm(n, k, r, 10, leaf)
    part = bem.precond_apply_fmm(n, k, r, 10, leaf, targets=tg)
    assert np.allclose(part, full[tg], rtol=1e-12, atol=1e-14)
    dense = bem.dirichlet_solve(n, k, r, g)
    errs = [np.linalg.norm(bem.precond_apply_fmm(n, k, r, p, leaf, g=g) - dense) / np.linalg.norm(dense)
            for p in (4, 10, 30)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-12
