"""Writes pass_1024_reference.npz: the first FMM pass of the preconditioner on the
1024 x 1024 grid (k h = 0.3, Gaussian-bump source), as the direct N-body sum
(oracle.kernel) at 2048 seeded targets, and the reference FMM's own relative
error there for p = 4, 6, 8 (oracle.fmm, leaf 32).

The pass sums the sources h^2 f at the interior nodes over the tree of
interior nodes and boundary element midpoints (Sec. 5.3: the volume term is
the dominant N_Omega x N_Omega product), so the targets are drawn from all
nodes of that tree.  Calls only oracle/ and the seeded input recipe.  Run from
the repository root:  python tests/golden/make_pass_1024_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import bem, fmm, kernel  # noqa: E402
from paper_1608_02461_amd import workloads  # noqa: E402

N_SAMPLES = 2048
SEED = 33


def main():
    w = workloads.solve_1024()
    n, k, h = w["n"], w["k"], w["h"]
    pts = np.concatenate([bem.interior_nodes(n), bem.boundary_nodes(n)])
    q = np.zeros(pts.shape[0], dtype=np.complex128)
    q[: n * n] = h * h * w["f"]
    samples = np.sort(np.random.default_rng(SEED).choice(pts.shape[0], N_SAMPLES, replace=False))
    t = time.time()
    direct = kernel.direct_sum_parallel(pts, q, k, pts[samples])
    print(f"direct sum at {samples.size} targets: {time.time() - t:.1f} s", flush=True)
    out = {"samples": samples, "direct": direct, "k": k, "leaf": w["leaf"], "seed": SEED}
    for p in (4, 6, 8):
        t = time.time()
        f = fmm.fmm(pts, q, k, p, w["leaf"], targets=samples)
        err = np.linalg.norm(f - direct) / np.linalg.norm(direct)
        out[f"eps_oracle_p{p}"] = err
        print(f"oracle FMM p={p}: rel err {err:.3e} ({time.time() - t:.1f} s)", flush=True)
    np.savez(os.path.join(os.path.dirname(os.path.abspath(__file__)), "pass_1024_reference.npz"), **out)


if __name__ == "__main__":
    main()
