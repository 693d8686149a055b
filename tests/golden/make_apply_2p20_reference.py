"""Writes apply_2p20_reference.npz: the direct N-body sum (oracle.kernel) at sampled
targets of the N = 2^20, k = 100 workload, and the reference FMM's own
relative error there for p = 4, 8, 12 (oracle.fmm, leaf 64).

Calls only oracle/ and the seeded input recipe.  Run from the repository
root:  python tests/golden/make_apply_2p20_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fmm, kernel  # noqa: E402
from paper_1608_02461_amd import workloads  # noqa: E402

N_SAMPLES = 2048


def main():
    w = workloads.fmm_2p20()
    xy, q, k = w["xy"], w["q"], w["k"]
    samples = w["samples"][:N_SAMPLES]
    t = time.time()
    direct = kernel.direct_sum_parallel(xy, q, k, xy[samples])
    print(f"direct sum at {samples.size} targets: {time.time() - t:.1f} s", flush=True)
    out = {"samples": samples, "direct": direct, "k": k, "leaf": w["leaf"]}
    for p in (4, 8, 12):
        t = time.time()
        f = fmm.fmm(xy, q, k, p, w["leaf"], targets=samples)
        err = np.linalg.norm(f - direct) / np.linalg.norm(direct)
        out[f"eps_oracle_p{p}"] = err
        print(f"oracle FMM p={p}: rel err {err:.3e} ({time.time() - t:.1f} s)", flush=True)
    np.savez(os.path.join(os.path.dirname(os.path.abspath(__file__)), "apply_2p20_reference.npz"), **out)


if __name__ == "__main__":
    main()
