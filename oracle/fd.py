"""The 5-point finite-difference Helmholtz matrix (test infrastructure).

The paper's Sec. 2 states that discretising the Helmholtz problem gives a
large sparse complex symmetric system A x = b; the discretisation used here
is the 5-point finite difference on the unit square with zero Dirichlet data:

    (A x)_ij = (4 x_ij - x_{i-1,j} - x_{i+1,j} - x_{i,j-1} - x_{i,j+1}) / h^2 - k2_ij x_ij

with ghost values zero, h = 1/(n+1), lexicographic order with x fastest.
This is -Laplace_h - k^2, the sign that matches the Green's representation
with G = (i/4) H0 (see the BEM module).
"""

import numpy as np
import scipy.sparse as sp


def matrix(n, k2, h=None):
    """Sparse CSR A; k2 is a scalar or an (n*n,) array of k^2 values."""
    h = 1.0 / (n + 1) if h is None else h
    e = np.ones(n)
    T = sp.diags([-e[:-1], 2 * e, -e[:-1]], [-1, 0, 1])
    I = sp.identity(n)
    lap = (sp.kron(I, T) + sp.kron(T, I)) / (h * h)
    k2 = np.broadcast_to(np.asarray(k2, dtype=np.float64), (n * n,))
    return (lap - sp.diags(k2)).tocsr().astype(np.complex128)


def apply(n, k2, x, h=None):
    """y = A x for x of shape (n*n,) or (n*n, nrhs)."""
    return matrix(n, k2, h) @ np.asarray(x, dtype=np.complex128)
