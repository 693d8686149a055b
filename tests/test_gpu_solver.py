"""GPU parity of the FD operator, the FMM-BEM preconditioner and FGMRES
(through the C-ABI) against the CPU oracle."""
import numpy as np
import pytest
import torch

from oracle import bem, fd, fgmres
from paper_1608_02461_amd import hfmm, workloads
from gpu_util import rel, say, to_dev, to_np

pytestmark = pytest.mark.gpu


def inv_norm_A(n, k2):
    """||A^{-1}||_2 for the FD operator with constant k^2 (discrete sine spectrum)."""
    h = 1.0 / (n + 1)
    s = 4 / h ** 2 * np.sin(np.arange(1, n + 1) * np.pi * h / 2) ** 2
    lam = s[:, None] + s[None, :] - k2
    return 1.0 / np.abs(lam).min()


@pytest.mark.parametrize("n,nrhs,field", [(1, 1, False), (7, 1, False), (64, 2, True), (129, 3, False)])
def test_fd_matvec(n, nrhs, field):
    say(f"fd n={n} nrhs={nrhs} field={field}")
    rng = np.random.default_rng(n)
    x = workloads.complex_normal(rng, (n * n, nrhs))
    k2 = rng.uniform(100, 200, n * n) if field else 150.0
    ref = fd.apply(n, k2, x)
    y = to_np(hfmm.hfmm_fd_helmholtz_matvec(n, 1.0 / (n + 1), to_dev(x), k2=to_dev(k2) if field else None,
                                            k2_const=0.0 if field else k2))
    assert rel(y, ref) <= 1e-14


@pytest.mark.parametrize("n,k,p,leaf", [(20, 16.0, 6, 8), (31, 30.0, 8, 16), (64, 16.0, 6, 32)])
def test_precond_fp64_matches_oracle(n, k, p, leaf):
    say(f"precond fp64 n={n} k={k} p={p} leaf={leaf}")
    rng = np.random.default_rng(n + p)
    r = workloads.complex_normal(rng, n * n)
    ref_fmm = bem.precond_apply_fmm(n, k, r, p, leaf)
    s = hfmm.Solver(n, k, p=p, leaf_size=leaf, prec=hfmm.FP64)
    z = to_np(s.precond_apply(to_dev(r)))
    say(f"  vs oracle FMM form: {rel(z, ref_fmm):.3e}  cond(S)={s.info()['cond_S']:.3e}")
    assert rel(z, ref_fmm) <= 1e-9
    if n <= 31:
        ref = bem.precond_apply(n, k, r)
        eps = rel(ref_fmm, ref)
        assert rel(z, ref) <= eps + 1e-6


@pytest.mark.parametrize("n,k,p,leaf", [(20, 16.0, 6, 8), (64, 16.0, 6, 32)])
def test_precond_fp32(n, k, p, leaf):
    say(f"precond fp32 n={n}")
    rng = np.random.default_rng(3 * n)
    r = workloads.complex_normal(rng, n * n)
    ref_fmm = bem.precond_apply_fmm(n, k, r, p, leaf)
    s = hfmm.Solver(n, k, p=p, leaf_size=leaf, prec=hfmm.FP32)
    z = to_np(s.precond_apply(to_dev(r)))
    say(f"  fp32 vs oracle FMM form: {rel(z, ref_fmm):.3e}")
    assert rel(z, ref_fmm) <= 1e-4


def test_solve_64_fp64():
    """64 x 64, k = 16, FGMRES(30), p = 6, leaf 32: true residual <= 1e-6 and
    the error bound ||x - x*|| <= ||A^-1|| ||b - A x|| against sparse direct."""
    w = workloads.solve_64()
    n, k = w["n"], w["k"]
    s = hfmm.Solver(n, k, p=w["p"], leaf_size=w["leaf"], prec=hfmm.FP64)
    x, info = s.solve(to_dev(w["f"]), restart=w["restart"], rtol=w["rtol"])
    x = to_np(x)
    A = fd.matrix(n, k * k)
    res = np.linalg.norm(w["f"] - A @ x) / np.linalg.norm(w["f"])
    say(f"  64^2 fp64: iters={info['iters']} restarts={info['restarts']} rel_res={res:.3e} (reported {info['rel_res_true']:.3e})")
    assert info["converged"] == 1
    assert res <= 1e-6
    assert abs(res - info["rel_res_true"]) <= 1e-9
    from scipy.sparse.linalg import spsolve
    xs = spsolve(A.tocsc(), w["f"])
    bound = inv_norm_A(n, k * k) * np.linalg.norm(w["f"] - A @ x)
    assert np.linalg.norm(x - xs) <= bound * (1 + 1e-6)
    # the oracle FGMRES with the exact dense preconditioner: report both counts
    Minv = bem.precond_matrix(n, k)
    xo, io = fgmres.fgmres(lambda v: A @ v, lambda v: Minv @ v, w["f"], restart=30, rtol=1e-6)
    say(f"  oracle dense-preconditioner iterations {io['iters']}, GPU FMM p=6 iterations {info['iters']}")
    assert abs(info["iters"] - io["iters"]) <= 5


def test_solve_64_fp32_preconditioner():
    w = workloads.solve_64()
    n, k = w["n"], w["k"]
    s = hfmm.Solver(n, k, p=w["p"], leaf_size=w["leaf"], prec=hfmm.FP32)
    x, info = s.solve(to_dev(w["f"]), restart=w["restart"], rtol=w["rtol"])
    A = fd.matrix(n, k * k)
    res = np.linalg.norm(w["f"] - A @ to_np(x)) / np.linalg.norm(w["f"])
    say(f"  64^2 fp32-precond: iters={info['iters']} rel_res={res:.3e}")
    assert info["converged"] == 1 and res <= 1e-6


def test_plane_wave_manufactured():
    n, k = 48, 20.0
    xo = bem.interior_nodes(n)
    u = np.exp(1j * k * (xo[:, 0] * np.cos(0.7) + xo[:, 1] * np.sin(0.7)))
    A = fd.matrix(n, k * k)
    b = A @ u
    s = hfmm.Solver(n, k, p=6, leaf_size=16, prec=hfmm.FP64)
    x, info = s.solve(to_dev(b), restart=30, rtol=1e-8)
    x = to_np(x)
    r = np.linalg.norm(b - A @ x)
    assert r <= 1e-8 * np.linalg.norm(b)
    assert np.linalg.norm(x - u) <= inv_norm_A(n, k * k) * r * (1 + 1e-6)


def test_multi_rhs_solve_and_zero_column():
    n, k = 32, 12.0
    rng = np.random.default_rng(9)
    b = workloads.complex_normal(rng, (n * n, 3))
    b[:, 1] = 0
    s = hfmm.Solver(n, k, p=6, leaf_size=16, prec=hfmm.FP64, nrhs=3)
    x, info = s.solve(to_dev(b), restart=20, rtol=1e-7)
    x = to_np(x)
    A = fd.matrix(n, k * k)
    assert np.all(x[:, 1] == 0)
    for c in (0, 2):
        assert np.linalg.norm(b[:, c] - A @ x[:, c]) <= 1e-7 * np.linalg.norm(b[:, c])
    assert info["converged"] == 1


def test_maxit_reports_not_converged():
    n, k = 24, 16.0
    rng = np.random.default_rng(2)
    b = workloads.complex_normal(rng, n * n)
    s = hfmm.Solver(n, k, p=6, leaf_size=16)
    x, info = s.solve(to_dev(b), restart=10, maxit=2, rtol=1e-12)
    assert info["converged"] == 0 and info["iters"] == 2
    with pytest.raises(hfmm.HFMMError) as e:
        s.solve(to_dev(b), restart=10, maxit=2, rtol=1e-12, strict=True)
    assert e.value.status == 1


def test_k2_field_and_set_k2():
    n = 32
    rng = np.random.default_rng(4)
    k2 = rng.uniform(0.8, 1.2, n * n) * 400.0
    b = workloads.complex_normal(rng, n * n)
    s = hfmm.Solver(n, 20.0, k2=to_dev(k2), p=6, leaf_size=16)
    x, info = s.solve(to_dev(b), restart=30, rtol=1e-8)
    A = fd.matrix(n, k2)
    assert np.linalg.norm(b - A @ to_np(x)) <= 1e-8 * np.linalg.norm(b)
    s.set_k2(k2_const=400.0)
    x2, _ = s.solve(to_dev(b), restart=30, rtol=1e-8)
    assert np.linalg.norm(b - fd.matrix(n, 400.0) @ to_np(x2)) <= 1e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_equals_individual(use_graph):
    probs = [(32, 14.0, 2), (48, 25.0, 1), (40, 9.0, 3)]
    solvers, bs, refs = [], [], []
    for i, (n, k, nr) in enumerate(probs):
        rng = np.random.default_rng(70 + i)
        b = workloads.complex_normal(rng, (n * n, nr))
        s = hfmm.Solver(n, k, p=6, leaf_size=16, prec=hfmm.FP32, nrhs=nr)
        solvers.append(s)
        bs.append(to_dev(b))
        refs.append(to_np(s.solve(to_dev(b), restart=20, rtol=1e-7)[0]))
    xs, infos = hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=20, rtol=1e-7, use_graph=use_graph)
    for (n, k, nr), x, ref, b, inf in zip(probs, xs, refs, bs, infos):
        x = to_np(x)
        assert inf["converged"] == 1
        assert np.array_equal(x, ref)
        A = fd.matrix(n, k * k)
        bb = to_np(b)
        for c in range(nr):
            assert np.linalg.norm(bb[:, c] - A @ x[:, c]) <= 1e-7 * np.linalg.norm(bb[:, c])


def test_solver_invalid_arguments():
    for kw in [dict(n=1, k0=5.0), dict(n=16, k0=0.0), dict(n=16, k0=5.0, p=0), dict(n=16, k0=5.0, leaf_size=-1)]:
        n = kw.pop("n")
        k0 = kw.pop("k0")
        with pytest.raises(hfmm.HFMMError):
            hfmm.Solver(n, k0, **kw)


def test_matched_wavenumber_and_fewer_iterations():
    k, h = 100.0, 1.0 / 257
    ref = 0.5 * (2 / h * np.arcsin(k * h / 2) + 2 * np.sqrt(2) / h * np.arcsin(k * h / (2 * np.sqrt(2))))
    assert abs(hfmm.hfmm_matched_wavenumber(k, h) - ref) <= 1e-12 * ref
    with pytest.raises(hfmm.HFMMError):
        hfmm.hfmm_matched_wavenumber(600.0, 1.0 / 257)  # k h >= 2
    n = 256
    rng = np.random.default_rng(91)
    b = workloads.complex_normal(rng, n * n)
    its = {}
    for name, k0 in (("k", k), ("matched", ref)):
        s = hfmm.Solver(n, k0, k2_const=k * k, p=6, leaf_size=32, prec=hfmm.FP32)
        x, info = s.solve(to_dev(b), restart=50, rtol=1e-6, maxit=2000)
        A = fd.matrix(n, k * k)
        assert np.linalg.norm(b - A @ to_np(x)) <= 1e-6 * np.linalg.norm(b)
        its[name] = info["iters"]
    say(f"  iterations k0=k: {its['k']}, matched: {its['matched']}")
    assert its["matched"] < its["k"]


def test_first_graph_solve_equals_eager():
    """The first solve after creation (graph mode on a private stream) must see
    a zeroed workspace and the caller's inputs: compare with a later eager solve."""
    solvers, bs = [], []
    for i, (n, k) in enumerate([(128, 60.0), (96, 40.0), (64, 30.0)]):
        rng = np.random.default_rng(100 + i)
        solvers.append(hfmm.Solver(n, hfmm.hfmm_matched_wavenumber(k, 1 / (n + 1)), k2_const=k * k, p=6,
                                   leaf_size=32, prec=hfmm.FP32, nrhs=2))
        bs.append(to_dev(workloads.complex_normal(rng, (n * n, 2))))
    xg, ig = hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=60, rtol=1e-6, use_graph=True)
    xe, ie = hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=60, rtol=1e-6, use_graph=False)
    for a, b, p, q in zip(xg, xe, ig, ie):
        assert p["iters"] == q["iters"]
        assert np.array_equal(to_np(a), to_np(b))


def test_graph_kept_across_solves_and_dropped_on_change():
    """The captured Arnoldi step is kept from one batched solve to the next
    (same restart, maxit, rtol) and captured again after a new restart or a
    change of k^2: every graph solve equals the eager one bit for bit."""
    probs = [(96, 40.0), (64, 30.0)]
    solvers = [hfmm.Solver(n, hfmm.hfmm_matched_wavenumber(k, 1 / (n + 1)), k2_const=k * k, p=6, leaf_size=32,
                           prec=hfmm.FP32, nrhs=2) for n, k in probs]
    rng = np.random.default_rng(120)

    def rhs():
        return [to_dev(workloads.complex_normal(rng, (n * n, 2))) for n, _ in probs]

    def check(bs, restart):
        xg, ig = hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=restart, rtol=1e-6, use_graph=True)
        xe, ie = hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=restart, rtol=1e-6, use_graph=False)
        for a, b, p, q in zip(xg, xe, ig, ie):
            assert p["converged"] == 1 and p["iters"] == q["iters"]
            assert np.array_equal(to_np(a), to_np(b))

    check(rhs(), 60)
    bs = rhs()
    check(bs, 60)  # the kept graphs
    check(bs, 40)  # captured again: new restart
    for s, (n, k) in zip(solvers, probs):
        s.set_k2(k2_const=(1.05 * k) ** 2)
    check(bs, 40)  # captured again: new k^2


def test_leaf_size_autotune():
    """leaf_size = 0 times the candidate trees and keeps one; the solve still meets rtol."""
    w = workloads.solve_64()
    n, k = w["n"], w["k"]
    s = hfmm.Solver(n, k, p=6, leaf_size=0, prec=hfmm.FP32)
    inf = s.info()
    say(f"  chosen leaf {inf['leaf_size']} (levels {inf['levels']})")
    assert inf["leaf_size"] in (16, 32, 64)
    x, info = s.solve(to_dev(w["f"]), restart=30, rtol=1e-6)
    A = fd.matrix(n, k * k)
    assert info["converged"] == 1
    assert np.linalg.norm(w["f"] - A @ to_np(x)) <= 1e-6 * np.linalg.norm(w["f"])


def test_solve_with_bf16_m2l_converges():
    """The preconditioner with its M2L operands rounded to BF16 still takes
    the 64 x 64 solve to the true residual 1e-6 (Sec. 6.1: the
    preconditioner need not be accurate)."""
    w = workloads.solve_64()
    s = hfmm.Solver(w["n"], w["k"], p=w["p"], leaf_size=w["leaf"], prec=hfmm.FP32)
    _, base = s.solve(to_dev(w["f"]), restart=w["restart"], rtol=w["rtol"])
    s.set_m2l_input_rounding("bf16")
    _, info = s.solve(to_dev(w["f"]), restart=w["restart"], rtol=w["rtol"])
    say(f"  iterations fp32 {base['iters']} bf16 {info['iters']}")
    assert info["converged"] == 1 and info["rel_res_true"] <= 1e-6
    assert info["iters"] <= base["iters"] + 5
