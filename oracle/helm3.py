"""The 3-D model problem and a free-space FMM preconditioner for it, plain
numpy / scipy FP64 (test infrastructure only; nothing in the product imports
it).

Sec. 7 poses Laplace(u) + kappa^2 u = f in the unit cube with u = 0 on its
boundary (eq. helm3).  Discretised here like the 2-D system of Sec. 2 by
finite differences, now the 7-point stencil on n^3 interior nodes
(i h, j h, l h), h = 1 / (n + 1), x fastest, ghost values zero:

    (A x)_ijl = (6 x_ijl - sum of the 6 neighbours) / h^2 - k^2 x_ijl,

i.e. -Laplace_h - k^2, whose free-space Green's function is the 3-D G of
Sec. 5.2, G(r) = exp(i k r) / (4 pi r).

Preconditioner (Sec. 4-5 in 3-D, without the boundary-element correction of
Sec. 5.2, which this build does not have for the cube): the volume potential
of the residual,

    z_i = h^3 sum_{j != i} G(|x_i - x_j|) r_j + c_self r_i,
    c_self = integral of G over the cell (a cube of side h centred on the node),

the 3-D analogue of pass 1 of the 2-D preconditioner.  c_self is computed
here by tensor Gauss-Legendre quadrature on the 6 pyramids from the centre
to the faces (the pyramid coordinates remove the 1/r singularity).
"""

import math

import numpy as np
import scipy.sparse as sp

from . import fmm3


def grid3(n):
    """(n^3, 3) interior node coordinates, x fastest, then y, then z."""
    h = 1.0 / (n + 1)
    i = np.arange(1, n + 1) * h
    Z, Y, X = np.meshgrid(i, i, i, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def matrix3(n, k2, h=None):
    """Sparse CSR A = -Laplace_h - k^2 (7-point), k2 a scalar."""
    h = 1.0 / (n + 1) if h is None else h
    e = np.ones(n)
    T = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1])
    I = sp.identity(n)
    lap = (sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)) / (h * h)
    return (lap - k2 * sp.identity(n ** 3)).tocsr().astype(np.complex128)


def self_term3(k, h, nq=24):
    """Integral of exp(i k r) / (4 pi r) over [-h/2, h/2]^3.  On the pyramid
    over the face z = h/2, y = t (a, b, h/2) with (a, b) on the face and t in
    [0, 1]: dV = (h/2) t^2 dt da db and the integrand times dV is
    (h/2) t exp(i k t rho) / (4 pi rho) dt da db, rho = |(a, b, h/2)|."""
    x, w = np.polynomial.legendre.leggauss(nq)
    t, wt = 0.5 * (x + 1.0), 0.5 * w               # [0, 1]
    a, wa = 0.5 * h * x, 0.5 * h * w               # [-h/2, h/2]
    A, B = np.meshgrid(a, a, indexing="ij")
    WAB = np.outer(wa, wa)
    rho = np.sqrt(A * A + B * B + 0.25 * h * h)
    inner = np.zeros_like(rho, dtype=np.complex128)
    for tq, wq in zip(t, wt):
        inner += wq * tq * np.exp(1j * k * tq * rho)
    return 6.0 * np.sum(WAB * (0.5 * h) * inner / (4.0 * math.pi * rho))


def precond3_apply(n, k, r):
    """z = h^3 (direct sum of G over the other nodes) r + c_self r (dense)."""
    h = 1.0 / (n + 1)
    xyz = grid3(n)
    r = np.asarray(r, dtype=np.complex128)
    return h ** 3 * fmm3.direct_sum3(xyz, r, k) + self_term3(k, h) * r


def precond3_apply_fmm(n, k, r, p, leaf):
    """The same with the oracle FMM in place of the direct sum (the tree over
    the nodes in the unit cube)."""
    h = 1.0 / (n + 1)
    xyz = grid3(n)
    r = np.asarray(r, dtype=np.complex128)
    return fmm3.fmm3_apply(xyz, h ** 3 * r, k, p, leaf) + self_term3(k, h) * r


def precond3_apply_at(n, k, r, idx):
    """The dense form at the nodes idx only: h^3 sum_{j != i} G(|x_i - x_j|) r_j
    + c_self r_i for i in idx (the direct sum of the oracle, four targets at a
    time so that a full-size grid fits in memory)."""
    h = 1.0 / (n + 1)
    xyz = grid3(n)
    r = np.asarray(r, dtype=np.complex128)
    idx = np.asarray(idx)
    return h ** 3 * fmm3.direct_sum3(xyz, r, k, targets=xyz[idx], chunk=4) + self_term3(k, h) * r[idx]
