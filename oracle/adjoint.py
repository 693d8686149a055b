"""Adjoint gradient of J(u) = 0.5 ||P u - d||^2 with respect to k^2 (test infrastructure).

u solves A(k^2) u = f with A = -Laplace_h - diag(k^2) (the FD module).  Since
dA/dk^2_x = -e_x e_x^T, the derivative of J is

    dJ/dk^2_x = -Re(lambda_x u_x),   A^T lambda = -conj(P^T (P u - d)),

and for a k^2 that is constant on blocks of nodes the block derivative is the
sum over the block.  All solves here are sparse direct (scipy splu), so this
is the plain definition, not an iteration.
"""

import numpy as np
from scipy.sparse.linalg import splu

from . import fd


def expand_blocks(kb, n):
    """k^2 at the n*n nodes from an (nb, nb) block field (block rows follow y)."""
    nb = kb.shape[0]
    s = n // nb
    return np.kron(kb, np.ones((s, s))).ravel()


def solve(n, k2, f):
    return splu(fd.matrix(n, k2).tocsc()).solve(np.asarray(f, dtype=np.complex128))


def objective(n, kb, f, P, d):
    u = solve(n, expand_blocks(kb, n), f)
    r = u[P] - d
    return 0.5 * float(np.vdot(r, r).real)


def gradient(n, kb, f, P, d):
    """Returns (J, dJ/dkb (nb, nb), u, lambda)."""
    k2 = expand_blocks(kb, n)
    lu = splu(fd.matrix(n, k2).tocsc())
    u = lu.solve(np.asarray(f, dtype=np.complex128))
    r = u[P] - d
    rhs = np.zeros(n * n, dtype=np.complex128)
    np.add.at(rhs, P, r)
    lam = lu.solve(-np.conj(rhs), trans="T")
    g = -np.real(lam * u)
    nb = kb.shape[0]
    s = n // nb
    G = g.reshape(nb, s, nb, s).sum(axis=(1, 3))
    return 0.5 * float(np.vdot(r, r).real), G, u, lam
