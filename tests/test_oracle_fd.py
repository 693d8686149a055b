"""Pins of the FD matrix (oracle.fd): discrete sine modes are exact eigenvectors
with eigenvalue (4/h^2)(sin^2(m pi h/2) + sin^2(l pi h/2)) - k^2."""
import numpy as np
import pytest

from oracle import bem, fd


@pytest.mark.parametrize("m,l", [(1, 1), (1, 2), (5, 3), (9, 9)])
def test_sine_modes(m, l):
    n, k = 9, 7.0
    h = 1 / (n + 1)
    xo = bem.interior_nodes(n)
    v = np.sin(m * np.pi * xo[:, 0]) * np.sin(l * np.pi * xo[:, 1])
    lam = 4 / h ** 2 * (np.sin(m * np.pi * h / 2) ** 2 + np.sin(l * np.pi * h / 2) ** 2) - k * k
    assert np.allclose(fd.apply(n, k * k, v), lam * v, atol=1e-9 * abs(lam))


def test_variable_k2_and_symmetry():
    n = 6
    rng = np.random.default_rng(41)
    k2 = rng.uniform(10, 20, n * n)
    A = fd.matrix(n, k2).toarray()
    assert np.allclose(A, A.T)
    assert np.allclose(np.diag(A), 4 * (n + 1) ** 2 - k2)
    # second node in the first row couples to its x-neighbours and the node above
    assert np.allclose([A[1, 0], A[1, 2], A[1, 1 + n]], -(n + 1) ** 2) and A[1, 3] == 0
