"""GPU parity of the 3-D oct-tree FMM (hfmm3_*) against the oracle
(oracle.fmm3): the oracle FMM with the same tree, orders and translations
element by element on small clouds (trees of depth 2 and 3, both
precisions), clustered clouds with empty leaves, points on the cube's faces
and coincident points; and, at the full 2^20-point size in the configuration
the benchmark times, sampled targets against the oracle's direct sum (Sec.
5.1, the N-body sum with the 3-D G of Sec. 5.2)."""
import numpy as np
import pytest

from oracle import fmm3 as o3
from paper_1608_02461_amd import hfmm, workloads
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def maxrel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def both(t, xyz, q, k, p):
    f64 = to_np(hfmm.hfmm3_fmm_apply(t, k, p, to_dev(q), prec=hfmm.FP64))
    f32 = to_np(hfmm.hfmm3_fmm_apply(t, k, p, to_dev(q.astype(np.complex64)), prec=hfmm.FP32))
    return f64, f32


# the FP64 near field: library sincos in the first two cases; the Taylor form
# with 13, 10 and 7 terms in the last three (k times twice the leaf diagonal
# 1.73, 1.08, 0.39)
@pytest.mark.parametrize("N,leaf,k,p", [(700, 16, 10.0, 4), (3000, 8, 6.0, 3), (3000, 8, 4.0, 4),
                                        (3000, 8, 2.5, 4), (3000, 8, 0.9, 3)])
def test_fmm3_matches_oracle_fmm(N, leaf, k, p):
    say(f"fmm3 parity N={N} leaf={leaf} k={k} p={p}")
    xyz, q = workloads.random_cloud3(N, 40 + N)
    t = hfmm.Tree3(to_dev(xyz), leaf_size=leaf)
    L = t.info()["levels"]
    assert L == o3.tree_depth3(N, leaf)
    assert t.orders(k, p) == o3.level_orders3(k, p, L)
    ref = o3.fmm3_apply(xyz, q, k, p, leaf)
    f64, f32 = both(t, xyz, q, k, p)
    say(f"  L={L} fp64 {rel(f64, ref):.2e} (max {maxrel(f64, ref):.2e}) fp32 {rel(f32, ref):.2e}")
    assert maxrel(f64, ref) <= 1e-11
    assert rel(f32, ref) <= 2e-5 and maxrel(f32, ref) <= 2e-4


def test_fmm3_clustered_faces_and_coincident_points():
    rng = np.random.default_rng(77)
    N = 1500
    centres = rng.uniform(0.2, 0.8, (3, 3))
    xyz = centres[rng.integers(0, 3, N)] + 0.02 * rng.standard_normal((N, 3))
    xyz = np.clip(xyz, 0.0, 1.0)
    xyz[:20] = rng.random((20, 3))
    xyz[20:30, 0] = 1.0  # on the far faces
    xyz[30:40, 1] = 1.0
    xyz[40:50, 2] = 1.0
    xyz[50:55] = 0.0     # the near corner
    xyz[60:70] = xyz[70:80]  # coincident distinct points
    q = workloads.complex_normal(rng, N)
    k, p, leaf = 8.0, 4, 8
    say(f"fmm3 clustered N={N}")
    t = hfmm.Tree3(to_dev(xyz), leaf_size=leaf)
    info = t.info()
    assert info["levels"] == 3 and info["max_leaf_count"] > 50
    ref = o3.fmm3_apply(xyz, q, k, p, leaf)
    f64, f32 = both(t, xyz, q, k, p)
    say(f"  fp64 {maxrel(f64, ref):.2e} fp32 {rel(f32, ref):.2e}")
    assert maxrel(f64, ref) <= 1e-11
    assert rel(f32, ref) <= 2e-5
    assert np.all(np.isfinite(f64)) and np.all(np.isfinite(f32))


def test_fmm3_errors_and_tree_checks():
    xyz, q = workloads.random_cloud3(500, 5)
    bad = xyz.copy()
    bad[3, 2] = 1.5
    with pytest.raises(hfmm.HFMMError):
        hfmm.Tree3(to_dev(bad), leaf_size=16)
    t = hfmm.Tree3(to_dev(xyz), leaf_size=16)
    with pytest.raises(hfmm.HFMMError):
        hfmm.hfmm3_fmm_apply(t, 0.0, 4, to_dev(q))          # k <= 0
    with pytest.raises(hfmm.HFMMError):
        hfmm.hfmm3_fmm_apply(t, 10.0, 21, to_dev(q))        # p above 20
    with pytest.raises(hfmm.HFMMError):
        hfmm.hfmm3_fmm_apply(t, 200.0, 4, to_dev(q))        # k times the leaf half-diagonal above 6
    phi = hfmm.hfmm3_fmm_apply(t, 10.0, 4, to_dev(q))
    assert phi.shape == (500,)


def test_fmm3_full_size_sampled():
    w = workloads.fmm3_2p20()
    xyz, q, k, p, smp = w["xyz"], w["q"], w["k"], w["p"], w["samples"]
    say(f"fmm3 full size N={len(xyz)} k={k} p={p}")
    t = hfmm.Tree3(to_dev(xyz), leaf_size=w["leaf"])
    assert t.info()["levels"] == 5
    ref = o3.direct_sum3(xyz, q, k, targets=xyz[smp], chunk=8)
    f64, f32 = both(t, xyz, q, k, p)
    e64, e32 = rel(f64[smp], ref), rel(f32[smp], ref)
    # the truncation error of this order with one-box separation: the oracle
    # FMM's own error on a cloud with the same leaf boxes (side 1/32, a cube
    # of side 1/4 at depth 3) and the same leaf orders
    c, qc = workloads.random_cloud3(4000, 9)
    c *= 0.25
    eps = rel(o3.fmm3_apply(c, qc, k, p, 8, side=0.25), o3.direct_sum3(c, qc, k))
    say(f"  fp64 {e64:.3e} fp32 {e32:.3e}  fp32 vs fp64 {rel(f32, f64):.3e}  oracle FMM error {eps:.3e}")
    assert e64 <= 2.0 * eps
    assert e32 <= 2.0 * eps and rel(f32, f64) <= 3e-5


def test_fmm3_overlapped_equals_serial_timed_apply():
    # the plain apply runs the far-field chain on the tree's second stream
    # beside the P2P; the timed apply runs the stages one after another
    xyz, q = workloads.random_cloud3(20000, 91)
    t = hfmm.Tree3(to_dev(xyz), leaf_size=16)
    say("fmm3 overlapped vs serial N=20000")
    for prec, dt in ((hfmm.FP64, np.complex128), (hfmm.FP32, np.complex64)):
        qd = to_dev(q.astype(dt))
        a = to_np(hfmm.hfmm3_fmm_apply(t, 12.0, 5, qd, prec=prec))
        b, ms = hfmm.hfmm3_fmm_apply_timed(t, 12.0, 5, qd, prec=prec)
        assert np.array_equal(a, to_np(b))
        assert set(ms) == set(hfmm.STAGES3) and ms["total"] > 0
