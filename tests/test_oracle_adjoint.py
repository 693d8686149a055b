"""Pin of the adjoint gradient (oracle.adjoint) against central finite differences of
J on the block values of k^2."""
import numpy as np

from oracle import adjoint


def test_adjoint_matches_central_differences():
    n, nb = 32, 4
    rng = np.random.default_rng(61)
    kb = rng.uniform(0.8, 1.2, (nb, nb)) * 400.0
    f = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    P = rng.choice(n * n, 60, replace=False)
    d = adjoint.solve(n, 400.0, f)[P]
    J, G, u, lam = adjoint.gradient(n, kb, f, P, d)
    assert J > 0
    for (i, j) in [(0, 0), (1, 2), (3, 3), (2, 1)]:
        dk = 1e-4 * kb[i, j]
        kp, km = kb.copy(), kb.copy()
        kp[i, j] += dk
        km[i, j] -= dk
        fdv = (adjoint.objective(n, kp, f, P, d) - adjoint.objective(n, km, f, P, d)) / (2 * dk)
        assert abs(fdv - G[i, j]) <= 1e-5 * abs(G).max()


def test_block_expansion_layout():
    kb = np.arange(4.0).reshape(2, 2)
    k2 = adjoint.expand_blocks(kb, 4).reshape(4, 4)  # rows follow y
    assert k2[0, 0] == 0 and k2[0, 3] == 1 and k2[3, 0] == 2 and k2[3, 3] == 3
