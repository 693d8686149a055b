"""The no-allocation FMM apply (hfmm_fmm_apply_noalloc, through the C-ABI)
against the allocating apply on the same inputs: the N = 2^20 workload
(two-stream schedule), then a smaller tree with two columns and a
single-leaf tree, so each call follows a larger one in the same fixed work
array; plus the size limit and the missing-plan error."""
import numpy as np
import pytest

from paper_1608_02461_amd import hfmm, workloads
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,dt,tol", [(hfmm.FP64, np.complex128, 1e-12), (hfmm.FP32, np.complex64, 1e-6)])
def test_noalloc_matches_apply(prec, dt, tol):
    cap = hfmm.hfmm_fmm_noalloc_capacity()
    assert cap == 64 << 20
    cases = []
    w = workloads.fmm_2p20()
    cases.append(("N=2^20 leaf 64", w["xy"], w["q"][:, None], 64, w["k"], 8))
    xy, q = workloads.random_cloud(3000, seed=91, nrhs=2)
    cases.append(("N=3000 leaf 16, 2 columns", xy, q, 16, 40.0, 10))
    xy, q = workloads.random_cloud(500, seed=92)
    cases.append(("N=500 single leaf", xy, q, 0, 20.0, 6))
    for name, xy, q, leaf, k, p in cases:
        say(f"noalloc prec={prec} {name}")
        t = hfmm.Tree(to_dev(xy), leaf_size=leaf)
        hfmm.hfmm_fmm_plan_info(t, k, p, prec)  # makes the plan
        qd = to_dev(np.ascontiguousarray(q).astype(dt))
        ref = to_np(hfmm.hfmm_fmm_apply(t, k, p, qd, prec=prec))
        for rep in range(2):  # two calls in a row on the same array
            got = to_np(hfmm.hfmm_fmm_apply_noalloc(t, k, p, qd, prec=prec))
            e = rel(got, ref)
            say(f"  call {rep}: rel diff {e:.3e} bitwise {np.array_equal(got, ref)}")
            assert np.all(np.isfinite(got))
            assert e <= tol


def test_noalloc_limits():
    w = workloads.fmm_2p20()
    t = hfmm.Tree(to_dev(w["xy"]), leaf_size=64)
    q2 = to_dev(np.repeat(w["q"][:, None], 2, axis=1))
    hfmm.hfmm_fmm_plan_info(t, w["k"], 8, hfmm.FP64)
    with pytest.raises(hfmm.HFMMError) as e:  # 2 columns of complex128 at 2^20 points exceed 64 MiB
        hfmm.hfmm_fmm_apply_noalloc(t, w["k"], 8, q2, prec=hfmm.FP64)
    assert e.value.status == -1 and "bytes of work memory" in str(e.value)
    with pytest.raises(hfmm.HFMMError) as e:  # no plan for this k
        hfmm.hfmm_fmm_apply_noalloc(t, 50.0, 8, q2[:, 0].contiguous(), prec=hfmm.FP64)
    assert e.value.status == -4
