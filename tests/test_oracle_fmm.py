"""Pins of the reference FMM (oracle.fmm): brute force on small N, error falling
with the order p down to round-off (Graf's addition theorem is exact in the
limit), the stage identities on a two-particle chain, the tree depth rule
and reciprocity within the FMM error."""
import numpy as np
import pytest

from oracle import fmm, kernel


@pytest.fixture(scope="module")
def cloud():
    rng = np.random.default_rng(21)
    xy = rng.random((900, 2))
    q = rng.standard_normal(900) + 1j * rng.standard_normal(900)
    return xy, q


@pytest.mark.parametrize("k", [16.0, 100.0])
def test_error_falls_with_p(cloud, k):
    xy, q = cloud
    ref = kernel.direct_sum(xy, q, k)
    errs = []
    for p in (2, 4, 6, 8, 12, 20, 30):
        f = fmm.fmm(xy, q, k, p, leaf=16)
        errs.append(np.linalg.norm(f - ref) / np.linalg.norm(ref))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-12
    assert errs[2] < 2e-3  # p = 6


def test_two_particle_chain_is_exact_at_high_order():
    # source in leaf (0,0), target in leaf (3,3) at L = 2: only the far field
    xy = np.array([[0.07, 0.11], [0.91, 0.83]])
    q = np.array([1.0 + 0.5j, 0.0])
    k = 9.0
    f = fmm.fmm(xy, q, k, 30, leaf=1)
    ref = kernel.direct_sum(xy, q, k)
    assert abs(f[1] - ref[1]) < 1e-13 * abs(ref[1])


def test_stage_identities():
    """P2M then the far-field sum (i/4) sum_n M_n out_n equals the direct field
    outside the box; L2P of the local expansion equals the far part."""
    from scipy.special import hankel1, jv
    rng = np.random.default_rng(22)
    xy = rng.random((40, 2)) * 0.25  # all in the first level-2 box
    q = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    k = 12.0
    _, st = fmm.fmm(xy, q, k, 25, leaf=64, return_stages=True)
    L = st["L"]
    assert L == 2
    M = st["M"][2][0, 0, :, 0]
    P = st["orders"][2]
    c = 0.125 + 0.125j
    x = 0.8 + 0.6j
    n = np.arange(-P, P + 1)
    far = 0.25j * np.sum(M * hankel1(n, k * abs(x - c)) * np.exp(1j * n * np.angle(x - c)))
    ref = kernel.direct_sum(xy, q, k, tgt=np.array([[x.real, x.imag]]))[0]
    assert abs(far - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("n,leaf,L", [(4356, 32, 4), (1048576, 64, 7), (1052676, 32, 8),
                                      (16900, 32, 5), (66564, 32, 6), (264196, 32, 7), (10, 0, 0), (5, 32, 2)])
def test_tree_depth_rule(n, leaf, L):
    assert fmm.tree_depth(n, leaf) == L


def test_level_orders():
    # p_l = p + floor(k d_l / 2), d_l = sqrt(2) 2^-l
    o = fmm.level_orders(100.0, 4, 7, 1.0)
    assert o[7] == 4 and o[6] == 5 and o[2] == 4 + 17


def test_targets_subset(cloud):
    xy, q = cloud
    full = fmm.fmm(xy, q, 30.0, 6, leaf=16)
    idx = np.array([0, 5, 17, 300, 899])
    sub = fmm.fmm(xy, q, 30.0, 6, leaf=16, targets=idx)
    assert np.allclose(sub, full[idx], rtol=1e-13, atol=1e-15)


def test_reciprocity_within_fmm_error(cloud):
    xy, _ = cloud
    rng = np.random.default_rng(23)
    a = rng.standard_normal(900) + 1j * rng.standard_normal(900)
    b = rng.standard_normal(900) + 1j * rng.standard_normal(900)
    lhs = a @ fmm.fmm(xy, b, 40.0, 12, leaf=16)
    rhs = b @ fmm.fmm(xy, a, 40.0, 12, leaf=16)
    assert abs(lhs - rhs) < 1e-6 * abs(lhs)


def test_all_pairs_mode_is_direct(cloud):
    xy, q = cloud
    f = fmm.fmm(xy[:200], q[:200], 50.0, 4, leaf=0)
    ref = kernel.direct_sum(xy[:200], q[:200], 50.0)
    assert np.allclose(f, ref, rtol=1e-13)


@pytest.mark.parametrize("k", [16.0, 60.0])
def test_dipole_error_falls_with_p(cloud, k):
    """Dipole sources (the double layer): the P2M of a dipole is the exact
    derivative of the monopole expansion, so the FMM error against the direct
    dG/dn sum falls with p to round-off, as for G."""
    xy, q = cloud
    rng = np.random.default_rng(5)
    a = rng.uniform(0, 2 * np.pi, xy.shape[0])
    nrm = np.stack([np.cos(a), np.sin(a)], 1)
    ref = kernel.direct_sum_dipole(xy, q, nrm, k)
    errs = []
    for p in (2, 4, 8, 14, 24):
        f = fmm.fmm(xy, q, k, p, leaf=16, normals=nrm)
        errs.append(np.linalg.norm(f - ref) / np.linalg.norm(ref))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-11
    # targets give the same values
    t = np.arange(0, xy.shape[0], 7)
    ft = fmm.fmm(xy, q, k, 14, leaf=16, normals=nrm, targets=t)
    assert np.allclose(ft, fmm.fmm(xy, q, k, 14, leaf=16, normals=nrm)[t], rtol=1e-13, atol=1e-13)
