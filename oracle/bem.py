"""The BEM-coupled preconditioner, dense closed form (test infrastructure).

Follows Sec. 5.2 (Green's representation with the Cauchy factor, the
Dirichlet boundary equation for du/dn, then the interior equation) and
Sec. 5.3 (piecewise constant elements without nodes at the square's corners,
the block matrix systems, and the analytic singular diagonal of the boundary
matrix).

Readings (where the paper is silent or ambiguous):
* Sign: the representation formula with +int f G and G = (i/4) H0 holds for
  -Laplace(u) - k^2 u = f; that is the equation solved here, and the FD
  operator is -Laplace_h - k^2.
* Geometry: unit square, interior nodes x_ij = (i h, j h), i, j = 1..n,
  h = 1/(n+1), lexicographic order with x fastest.  Each side is cut into n+1
  constant elements of width w = h with collocation at the midpoints, so
  N_Gamma = 4 (n + 1) and no node sits on a corner.
* One-point (midpoint) quadrature off the diagonal, so every element acts as a
  point source of weight w.
* Boundary diagonal: the analytic formula of Sec. 5.3,
      int H0 = w + i (2/pi) w [ln(gamma k w / 4) - 1],  gamma = exp(Euler's const),
  read with the garbled closing parenthesis dropped.
* Volume diagonal (paper silent): the exact integral of G over the node's own
  h x h cell, S_vol = (i/4) int_cell H0(k |x|) dA, evaluated in polar form
      8 int_0^{pi/4} [ R H1(kR)/k + 2i/(pi k^2) ] dtheta,  R = h / (2 cos theta),
  which follows from d/drho [rho H1(k rho)] = k rho H0(k rho).
* The volume integral uses the midpoint rule with weight h^2 per node.
* The boundary system is solved exactly (dense), once per (k, grid).

With u = 0 on Gamma the preconditioner z = M^{-1} r is
    V_Omega = h^2 G_OO r (diagonal S_vol/h^2),  V_Gamma = h^2 G_GO r,
    q = -S^{-1} V_Gamma                 (boundary equation, S = w G_GG),
    z = V_Omega + w G_OG q              (interior equation),
i.e. M^{-1} = h^2 [G_OO - G_OG (S/w)^{-1} G_GO].
"""

import math

import numpy as np
from scipy.integrate import quad
from scipy.special import hankel1

from .kernel import green

EULER_GAMMA_EXP = math.exp(0.57721566490153286061)  # the paper's gamma (Sec. 5.3)


def interior_nodes(n):
    """(n*n, 2) node coordinates, x fastest; h = 1/(n+1)."""
    h = 1.0 / (n + 1)
    i = np.arange(1, n + 1) * h
    X, Y = np.meshgrid(i, i, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def boundary_nodes(n):
    """(4(n+1), 2) element midpoints: bottom, right, top, left sides; width h."""
    h = 1.0 / (n + 1)
    m = (np.arange(n + 1) + 0.5) * h
    z = np.zeros_like(m)
    o = np.ones_like(m)
    return np.concatenate([
        np.stack([m, z], 1),   # y = 0
        np.stack([o, m], 1),   # x = 1
        np.stack([m, o], 1),   # y = 1
        np.stack([z, m], 1),   # x = 0
    ])


def boundary_self(k, w):
    """Diagonal of S = int over the element of G: (i/4) [w + i (2/pi) w (ln(gamma k w/4) - 1)]."""
    return 0.25j * (w + 1j * (2.0 / math.pi) * w * (math.log(EULER_GAMMA_EXP * k * w / 4.0) - 1.0))


def volume_self(k, h):
    """S_vol = (i/4) int_{[-h/2,h/2]^2} H0(k|x|) dA by the polar form (eight triangles)."""

    def f(theta, part):
        R = h / (2.0 * math.cos(theta))
        v = R * hankel1(1, k * R) / k + 2j / (math.pi * k * k)
        return v.real if part == 0 else v.imag

    re = quad(f, 0.0, math.pi / 4, args=(0,), epsabs=0, epsrel=1e-13, limit=200)[0]
    im = quad(f, 0.0, math.pi / 4, args=(1,), epsabs=0, epsrel=1e-13, limit=200)[0]
    return 0.25j * 8.0 * (re + 1j * im)


def _pair_matrix(a, b, k):
    d = a[:, None, :] - b[None, :, :]
    r = np.sqrt(d[..., 0] ** 2 + d[..., 1] ** 2)
    out = np.zeros(r.shape, dtype=np.complex128)
    nz = r > 0
    out[nz] = green(r[nz], k)
    return out


def blocks(n, k):
    """The dense blocks G_OO (with the S_vol/h^2 diagonal), G_OG, G_GO and S/w."""
    h = 1.0 / (n + 1)
    w = h
    xo, xg = interior_nodes(n), boundary_nodes(n)
    Goo = _pair_matrix(xo, xo, k)
    Goo[np.diag_indices_from(Goo)] = volume_self(k, h) / (h * h)
    Gog = _pair_matrix(xo, xg, k)
    Sw = _pair_matrix(xg, xg, k)
    Sw[np.diag_indices_from(Sw)] = boundary_self(k, w) / w
    return Goo, Gog, Sw


def precond_matrix(n, k):
    """M^{-1} = h^2 [G_OO - G_OG (S/w)^{-1} G_GO] as a dense (n^2 x n^2) matrix."""
    h = 1.0 / (n + 1)
    Goo, Gog, Sw = blocks(n, k)
    return h * h * (Goo - Gog @ np.linalg.solve(Sw, Gog.T))


def precond_apply(n, k, r):
    """z = M^{-1} r by the steps of the boundary and interior equations (dense)."""
    h = 1.0 / (n + 1)
    w = h
    Goo, Gog, Sw = blocks(n, k)
    r = np.asarray(r, dtype=np.complex128)
    v_omega = h * h * (Goo @ r)
    v_gamma = h * h * (Gog.T @ r)
    q = -np.linalg.solve(w * Sw, v_gamma)
    return v_omega + w * (Gog @ q)


def boundary_normals(n):
    """Outward unit normals of the elements, in the order of boundary_nodes."""
    m = n + 1
    return np.concatenate([np.tile([0.0, -1.0], (m, 1)), np.tile([1.0, 0.0], (m, 1)),
                           np.tile([0.0, 1.0], (m, 1)), np.tile([-1.0, 0.0], (m, 1))])


def precond_apply_fmm(n, k, r, p, leaf, targets=None, g=None):
    """The same preconditioner with the N-body sums done by the reference FMM.

    Pass 1: sources h^2 r at the interior nodes, targets all nodes (the tree is
    built over interior and boundary nodes together).  Boundary solve.  Pass 2:
    sources w q at the boundary nodes, targets the interior nodes.

    targets : optional interior node indices; z is then computed only there
              (pass 1 at the boundary nodes and those targets, pass 2 at the
              targets), which keeps large grids cheap.
    g       : optional Dirichlet data at the boundary midpoints (Sec. 5.2 with
              u = g on Gamma): pass 1 also carries the double layer
              -w sum_b g_b dG/dn_b, the boundary equation takes the 1/2 delta
              term, S q = g/2 + D_Gamma - V_Gamma, and the interior equation
              keeps -D_Omega (see dirichlet_solve).
    """
    from .fmm import fmm

    h = 1.0 / (n + 1)
    w = h
    xo, xg = interior_nodes(n), boundary_nodes(n)
    pts = np.concatenate([xo, xg])
    no, ng = xo.shape[0], xg.shape[0]
    r = np.asarray(r, dtype=np.complex128)
    squeeze = r.ndim == 1
    if squeeze:
        r = r[:, None]
    tg = np.arange(no) if targets is None else np.asarray(targets, dtype=np.int64)
    t1 = np.concatenate([tg, no + np.arange(ng)])
    src1 = np.zeros((pts.shape[0], r.shape[1]), dtype=np.complex128)
    src1[:no] = h * h * r
    phi1 = fmm(pts, src1, k, p, leaf, targets=t1)
    if g is not None:
        g = np.asarray(g, dtype=np.complex128).reshape(ng, -1)
        nrm = np.zeros((pts.shape[0], 2))
        nrm[no:] = boundary_normals(n)
        srcd = np.zeros_like(src1)
        srcd[no:] = -w * g
        phi1 = phi1 + fmm(pts, srcd, k, p, leaf, targets=t1, normals=nrm)
    v_omega = phi1[:tg.size] + volume_self(k, h) * r[tg]
    v_gamma = phi1[tg.size:]
    Sw = _pair_matrix(xg, xg, k)
    Sw[np.diag_indices_from(Sw)] = boundary_self(k, w) / w
    rhs = -v_gamma if g is None else 0.5 * g - v_gamma
    q = np.linalg.solve(w * Sw, rhs)
    src2 = np.zeros_like(src1)
    src2[no:] = w * q
    phi2 = fmm(pts, src2, k, p, leaf, targets=tg)
    z = v_omega + phi2
    return z[:, 0] if squeeze else z


def double_layer_blocks(n, k):
    """D_OG[i, b] = dG/dn_b(x_i, y_b) and D_GG[a, b] = dG/dn_b(y_a, y_b) (a != b).

    The diagonal of D_GG is zero: on a flat constant element (x - y).n = 0
    for every y of the element, so the element exerts no double-layer field
    on its own midpoint (one-point quadrature elsewhere, as for G).
    """
    from .kernel import dgreen_dn

    xo, xg, nrm = interior_nodes(n), boundary_nodes(n), boundary_normals(n)
    Dog = dgreen_dn(xo[:, None, :], xg[None, :, :], nrm[None, :, :], k)
    X = np.broadcast_to(xg[:, None, :], (xg.shape[0], xg.shape[0], 2))
    Y = np.broadcast_to(xg[None, :, :], X.shape)
    Nn = np.broadcast_to(nrm[None, :, :], X.shape)
    Dgg = np.zeros(X.shape[:2], dtype=np.complex128)
    off = ~np.eye(xg.shape[0], dtype=bool)
    Dgg[off] = dgreen_dn(X[off], Y[off], Nn[off], k)
    return Dog, Dgg


def dirichlet_solve(n, k, f, g):
    """Boundary-element solution with source f and Dirichlet data g (Sec. 5.2), dense.

    Green's representation with the Cauchy factor (1/2 on the smooth boundary
    points, 1 inside) for -Laplace(u) - k^2 u = f:
        eta u = int_Omega f G + int_Gamma (du/dn) G - int_Gamma u dG/dn.
    On the boundary (eq. ubound) the unknown q = du/dn solves
        S q = g/2 + w D_GG g - V_Gamma,     S = w G_GG (analytic diagonal),
    and inside (eq. uinter)
        u = V_Omega + w G_OG q - w D_OG g,
    with V = h^2 G f the volume potential (midpoint rule, exact self cell).
    f : (n*n,) interior values; g : (4(n+1),) values at the element midpoints.
    """
    h = 1.0 / (n + 1)
    w = h
    Goo, Gog, Sw = blocks(n, k)
    Dog, Dgg = double_layer_blocks(n, k)
    f = np.asarray(f, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)
    v_omega = h * h * (Goo @ f)
    v_gamma = h * h * (Gog.T @ f)
    q = np.linalg.solve(w * Sw, 0.5 * g + w * (Dgg @ g) - v_gamma)
    return v_omega + w * (Gog @ q) - w * (Dog @ g)
