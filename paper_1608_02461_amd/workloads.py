"""Seeded synthetic inputs shaped like the paper's model problems.

This module holds only random-number recipes and problem sizes: none of the
method's arithmetic.  The same arrays feed the HIP path and the CPU oracle.
All generators are numpy PCG64 (``numpy.random.default_rng(seed)``).

Workloads (the paper runs its own synthetic PDE model problems, Sec. 6; no
dataset is involved):

* ``solve_64``   64 x 64 interior grid, h = 1/65, k = 16, f complex N(0,1).
* ``fmm_2p20``     N = 2^20 uniform points in the unit square, complex N(0,1)
                 charges, k = 100, 2048 sampled targets.
* ``solve_1024``   1024 x 1024 grid, k = 0.3/h, Gaussian bump
                 f = exp(-|x - x0|^2 / 0.01) with x0 uniform in [0.25, 0.75]^2.
* ``batch_16x4``   16 problems, k uniform in [20, 300], n from {128,256,384,512}
                 with k h <= 0.6, 4 right-hand sides each, complex64 N(0,1).
* ``adjoint_256`` 256 x 256 grid, k^2 constant on 16 x 16 blocks with values in
                 [0.8, 1.2] * 100^2, 512 sampled nodes, f complex N(0,1).
* ``fmm3_2p20``  the 3-D apply: N = 2^20 uniform points in the unit cube,
                 complex N(0,1) charges, k = 10, p = 6, leaf 64 (8^5 leaves of
                 32 points on average), 256 sampled targets.
"""

import numpy as np


def grid_h(n):
    return 1.0 / (n + 1)


def interior_xy(n):
    """(n*n, 2) interior node coordinates (i h, j h), x fastest."""
    h = grid_h(n)
    i = np.arange(1, n + 1) * h
    X, Y = np.meshgrid(i, i, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def complex_normal(rng, shape, dtype=np.complex128):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


def solve_64(n=64, k=16.0, seed=1):
    rng = np.random.default_rng(seed)
    f = complex_normal(rng, n * n)
    return {"n": n, "h": grid_h(n), "k": k, "f": f, "p": 6, "leaf": 32, "restart": 30, "rtol": 1e-6}


def fmm_2p20(N=1 << 20, k=100.0, seed=2, n_samples=2048, nrhs=1):
    rng = np.random.default_rng(seed)
    xy = rng.random((N, 2))
    q = complex_normal(rng, (N, nrhs) if nrhs > 1 else N)
    samples = rng.choice(N, min(n_samples, N), replace=False)
    return {"xy": xy, "q": q, "k": k, "samples": np.sort(samples), "leaf": 64}


def solve_1024(n=1024, kh=0.3, seed=3):
    rng = np.random.default_rng(seed)
    h = grid_h(n)
    x0 = rng.uniform(0.25, 0.75, 2)
    xy = interior_xy(n)
    r2 = (xy[:, 0] - x0[0]) ** 2 + (xy[:, 1] - x0[1]) ** 2
    f = np.exp(-r2 / 0.01).astype(np.complex128)
    return {"n": n, "h": h, "k": kh / h, "f": f, "x0": x0, "leaf": 32, "restart": 50, "rtol": 1e-6}


def batch_16x4(seed=4, n_problems=16, nrhs=4, sizes=(128, 256, 384, 512), kh_max=0.6):
    rng = np.random.default_rng(seed)
    probs = []
    for _ in range(n_problems):
        k = float(rng.uniform(20.0, 300.0))
        ok = [s for s in sizes if k / (s + 1) <= kh_max]
        n = int(rng.choice(ok))
        f = complex_normal(rng, (n * n, nrhs), np.complex64)
        probs.append({"n": n, "h": grid_h(n), "k": k, "f": f})
    return {"problems": probs, "p": 6, "leaf": 32, "restart": 200, "rtol": 1e-6}


def adjoint_256(n=256, nb=16, k0=100.0, n_obs=512, seed=5):
    rng = np.random.default_rng(seed)
    kb = rng.uniform(0.8, 1.2, (nb, nb)) * k0 * k0
    P = np.sort(rng.choice(n * n, n_obs, replace=False))
    f = complex_normal(rng, n * n)
    return {"n": n, "h": grid_h(n), "kb": kb, "P": P, "f": f, "k0": k0, "k2_ref": k0 * k0,
            "p": 6, "leaf": 32, "restart": 200}


def random_cloud(N, seed, nrhs=1, dtype=np.complex128):
    """Uniform points in the unit square with complex N(0,1) charges (parity cases)."""
    rng = np.random.default_rng(seed)
    xy = rng.random((N, 2))
    q = complex_normal(rng, (N, nrhs), dtype)
    return xy, q


def fmm3_2p20(N=1 << 20, k=10.0, p=6, seed=6, n_samples=256):
    rng = np.random.default_rng(seed)
    xyz = rng.random((N, 3))
    q = complex_normal(rng, N)
    samples = np.sort(rng.choice(N, min(n_samples, N), replace=False))
    return {"xyz": xyz, "q": q, "k": k, "p": p, "leaf": 64, "samples": samples}


def random_cloud3(N, seed, dtype=np.complex128):
    """Uniform points in the unit cube with complex N(0,1) charges (parity cases)."""
    rng = np.random.default_rng(seed)
    xyz = rng.random((N, 3))
    q = complex_normal(rng, N, dtype)
    return xyz, q


def helm3_cube(n, k=10.0):
    """The 3-D model problem (Sec. 7, eq. helm3) on n^3 interior nodes of the
    unit cube: source 1 (negated for -Laplace - k^2, as in 2-D), u = 0 on the
    faces.  The paper sets kappa = 0; the Helmholtz kernel needs k > 0."""
    return {"n": n, "k": k, "b": -np.ones(n ** 3, dtype=np.complex128), "p": 6, "leaf": 64}
