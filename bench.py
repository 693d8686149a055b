"""Benchmark: the 2-D Helmholtz FMM apply (and FMM-BEM preconditioned solves) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--p 8] [--no-extras] [--no-cpu]

Headline workload (one step = one FMM apply, inputs resident in HBM, tree
built beforehand and timed separately): N = 2^20 uniform points in the unit
square, complex N(0,1) charges, k = 100, leaf 64, complex64 arithmetic, order
p (default 8).  value = N / (time per apply) in Mpts/s.

Also reported on the same JSON line:
* the same apply in complex128 and at p = 4, 8, 12, with relative errors on
  the 2048 seeded targets against the stored direct sum, and the FP64 near
  field's roofline;
* the 1024 x 1024 grid, k h = 0.3, Gaussian bump, to 1e-6: complex64 FMM
  inside FP64 FGMRES(50) vs all-FP64 at p = 4, 6, 8 (k0 = k) and with the
  dispersion-matched k0 at p = 6; the first FMM pass's error on 2048 samples
  against the stored direct sum;
* the batched solve of 16 problems x 4 right-hand sides (k in [20, 300], n in
  {128, 256, 384, 512}): matched k0 with FGMRES(200), graph vs eager, and the
  survey's settings (k0 = k, FGMRES(50), non-convergence reported);
* the M2L with its operands rounded to FP16 / BF16 (accuracy experiment):
  the N = 2^20 apply's error and the 1024 x 1024 solve's iterations;
* forward + backward of the block-k^2 adjoint gradient on 256 x 256, checked
  against the CPU oracle's sparse-direct adjoint gradient;
* the 64 x 64 solve; the paper's helm2 family (inhomogeneous Dirichlet data)
  on FD; BiCGSTAB vs FGMRES on helm1; iterations against p in both
  precisions; the FD matvec's HBM rate;
* `roofline` for the dominant kernel of the apply (the near field), from
  hipEvents recorded on its launch stream around it, over the same number of
  applies as the timed steps;
* `cpu_baseline`: the CPU oracle's direct N-body sum on a bounded sample of
  targets, scaled to Mpts/s of the full sum; `cpu_baselines_extra`: the
  oracle's 64 x 64 solve, a sparse-direct 1024 x 1024 solve and the oracle
  adjoint gradient on the host.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FMM-preconditioned Helmholtz solves/s to 1e-6 res; FMM Mpts/s FP32-mixed vs FP64"
PEAK_FP32_ALU = 78.6   # TFLOP/s: 256 CU x 64 FP32 FMA lanes x 2 flop x 2.4 GHz (packed FP32 off)
PEAK_FP64_ALU = 78.6
PEAK_HBM = 8000.0       # GB/s


PMC_SUMMARY = os.path.join(ROOT, "profiles", "p2p_fmm_n1m_k100_p8_fp32_pmc.md")
M2L_SUMMARY = os.path.join(ROOT, "profiles", "m2l_mfma_fmm_n1m_and_n1024_counters.md")
FMM3_SUMMARY = os.path.join(ROOT, "profiles", "fmm3_apply_n1m_k10_p6_kernels.md")
PEAK_FP32_MFMA = 157.3  # TFLOP/s, dense FP32 matrix cores
PEAK_FP64_MFMA = 78.6


def profile_record(path, kernel):
    """The JSON record of a committed counter summary, or None when the
    summary is absent, is for another kernel, or a source file it names has
    changed since the counters were taken (SHA-256 of `source`, or of each
    file in `sources` against `sources_sha256`)."""
    import hashlib
    import re
    try:
        txt = open(path).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", txt, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec["kernel"] != kernel:
        return None
    pairs = (zip(rec["sources"], rec["sources_sha256"]) if "sources" in rec
             else [(rec["source"], rec["source_sha256"])])
    for src, sha in pairs:
        if hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest() != sha:
            return None
    return rec


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading on
    a plain device copy of known size), or None when the summary is absent,
    is for another kernel, or the near-field source has changed since."""
    rec = profile_record(PMC_SUMMARY, kernel)
    return None if rec is None else rec["bytes_per_launch"]


def _deinterleave(v):
    v = v & 0x55555555
    v = (v | (v >> 1)) & 0x33333333
    v = (v | (v >> 2)) & 0x0F0F0F0F
    v = (v | (v >> 4)) & 0x00FF00FF
    return (v | (v >> 8)) & 0x0000FFFF


def m2l_translations(tree):
    """Interaction-list translations per level (Sec. 5.1.2): pairs of
    non-empty boxes of one level whose parents are neighbours (or the same)
    while they are not neighbours themselves, counted from the tree's leaf
    occupancy (Morton order, parents occupied when a child is)."""
    _, off = tree.export()
    occ = np.diff(off.cpu().numpy()) > 0
    L = tree.info()["levels"]
    out = {}
    for lev in range(L, 1, -1):
        side = 1 << lev
        idx = np.arange(side * side)
        grid = np.zeros((side, side), bool)
        grid[_deinterleave(idx), _deinterleave(idx >> 1)] = occ
        X, Y = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
        c = 0
        for dx in range(-3, 4):
            for dy in range(-3, 4):
                if max(abs(dx), abs(dy)) <= 1:
                    continue
                sx, sy = X + dx, Y + dy
                ok = (sx >= 0) & (sx < side) & (sy >= 0) & (sy < side) & grid
                ok &= (np.abs(sx // 2 - X // 2) <= 1) & (np.abs(sy // 2 - Y // 2) <= 1)
                c += int(grid[sx[ok], sy[ok]].sum())
        out[lev] = c
        occ = occ.reshape(-1, 4).any(1)
    return out


def m2l_algorithmic_flops(tree, orders, nrhs=1):
    """Real flops of the M2L as dense complex products: a translation at
    level l maps 2 p_l + 1 coefficients to 2 p_l + 1, each complex
    multiply-add 8 flops."""
    return sum(c * 8 * (2 * orders[lev] + 1) ** 2 * nrhs for lev, c in m2l_translations(tree).items())


def m2l_roofline(tree, orders, ms, prec_name, counters_key=None):
    """M2L rate from the launch's hipEvent time on its own stream (`ms`)
    against the MFMA peak of its precision; the executed-to-algorithmic
    ratio comes from the committed MFMA counter summary when it matches the
    current source."""
    fl = m2l_algorithmic_flops(tree, orders)
    peak = PEAK_FP32_MFMA if prec_name == "fp32" else PEAK_FP64_MFMA
    ach = fl / (ms * 1e-3) / 1e12
    out = {"bound": "mfma", "kernel": f"k_m2l_mfma<{'float' if prec_name == 'fp32' else 'double'}>",
           "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
           "algorithmic_flops_per_launch": fl, "ms_per_launch": round(ms, 5),
           "translations_per_level": m2l_translations(tree)}
    rec = profile_record(M2L_SUMMARY, "k_m2l_mfma") if counters_key else None
    if rec is not None and counters_key in rec["executed_flops"]:
        out["executed_over_algorithmic"] = round(rec["executed_flops"][counters_key] / fl, 3)
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def p2p_flops_per_pair(deg, nrhs=1, plain_below=9):
    """FP32 fast-path P2P flops per pair, counted from the kernel source
    (FMA = 2): dx, dy (2); t = fma(dx, dx, dy*dy) (3); the centred variable
    u = fma(t, ua, ub) (2), only for coefficient counts of 9 and more (the
    lower ones are polynomials in t itself); two Horner chains of deg-1 FMAs
    (4 (deg-1)); Y = fma(Jc, log2 t, Yf) (2); 4 FMAs per right-hand side into
    the accumulators (8 nrhs).  The log2 per pair is a transcendental and is
    not counted."""
    return 2 + 3 + (0 if deg < plain_below else 2) + 4 * (deg - 1) + 2 + 8 * nrhs


def timed_solves(s, f, reps, **kw):
    """Warm solve, then the mean wall time of `reps` solves (host clock, stream synchronised)."""
    import torch
    s.solve(f, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        x, info = s.solve(f, **kw)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, x, info


def p2p_flops_per_pair_fp64(deg, nrhs=1):
    """FP64 fast-path P2P flops per pair (as p2p_flops_per_pair; the centred
    variable is used from 12 coefficients up; the FP64 log2 is not counted)."""
    return p2p_flops_per_pair(deg, nrhs, plain_below=12)


def bench_fmm_orders(tree, k, N, q32, q64, gold, smp, hfmm, torch, plan32):
    """The 2^20-point apply at p = 4, 8, 12 in both precisions, errors on the stored samples,
    and the near-field roofline of the FP64 apply at p = 8."""
    fmm_tab = {}
    for pp in (4, 8, 12):
        row = {"eps_oracle": float(gold[f"eps_oracle_p{pp}"])}
        for name, q, prec in (("fp32", q32, hfmm.FP32), ("fp64", q64, hfmm.FP64)):
            hfmm.hfmm_fmm_apply(tree, k, pp, q, prec=prec)
            torch.cuda.synchronize()
            reps = 5
            t0 = time.perf_counter()
            for _ in range(reps):
                out = hfmm.hfmm_fmm_apply(tree, k, pp, q, prec=prec)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            o = out.cpu().numpy()[smp]
            row[name] = {"mpts_s": round(N / dt / 1e6, 2), "ms": round(dt * 1e3, 4),
                         "rel_err": float(np.linalg.norm(o - gold["direct"]) / np.linalg.norm(gold["direct"]))}
        fmm_tab[f"p{pp}"] = row
        log(f"2^20 apply p={pp}: {row}")
    # FP64 near-field roofline (p = 8): duration from the stage-timed applies
    plan64 = hfmm.hfmm_fmm_plan_info(tree, k, 8, hfmm.FP64)
    st = {s_: 0.0 for s_ in hfmm.STAGES}
    for _ in range(5):
        _, ms = hfmm.hfmm_fmm_apply_timed(tree, k, 8, q64, prec=hfmm.FP64)
        for s_ in st:
            st[s_] += ms[s_] / 5
    fl = plan64["pairs"] * p2p_flops_per_pair_fp64(plan64["near_deg"])
    ach = fl / (st["p2p"] * 1e-3) / 1e12
    fmm_tab["fp64_p8_stage_ms"] = {s_: round(v, 4) for s_, v in st.items()}
    fmm_tab["fp64_p8_roofline"] = {
        "bound": "alu", "kernel": f"k_p2p4<double,1,{plan64['near_deg']},true,{plan64['lanes_per_target']}>",
        "achieved": round(ach, 3), "peak": PEAK_FP64_ALU, "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_ALU, 4),
        "algorithmic_flops_per_launch": fl, "ms_per_launch": round(st["p2p"], 5), "near_deg": plan64["near_deg"],
        "note": "the per-pair FP64 log2 is counted as 0 flops"}
    fmm_tab["fp64_p8_m2l_roofline"] = m2l_roofline(tree, plan64["orders"], st["m2l"], "fp64", "apply_2p20_p8_fp64")
    log(f"2^20 apply fp64 p=8 stages {fmm_tab['fp64_p8_stage_ms']} roofline {fmm_tab['fp64_p8_roofline']['frac']} "
        f"M2L {fmm_tab['fp64_p8_m2l_roofline']['frac']}")
    return fmm_tab


def solver_tree_points(n):
    """Interior nodes then boundary element midpoints (bottom, right, top, left), as the solver's tree."""
    h = 1.0 / (n + 1)
    m = (np.arange(n + 1) + 0.5) * h
    z, o = np.zeros_like(m), np.ones_like(m)
    from paper_1608_02461_amd import workloads
    return np.concatenate([workloads.interior_xy(n), np.stack([m, z], 1), np.stack([o, m], 1),
                           np.stack([m, o], 1), np.stack([z, m], 1)])


def bench_solve_1024(dev, hfmm, workloads, torch):
    """1024 x 1024, k h = 0.3: mixed vs FP64 FGMRES(50) at p = 4, 6, 8 (k0 = k), the
    dispersion-matched k0 at p = 6, the first pass's FMM error on 2048 samples
    against the stored direct sum, and per-stage times of one pass."""
    w1024 = workloads.solve_1024()
    n3, k3 = w1024["n"], w1024["k"]
    f = torch.from_numpy(w1024["f"]).to(dev)
    out = {"k": k3, "leaf": w1024["leaf"], "restart": 50}
    k3m = hfmm.hfmm_matched_wavenumber(k3, 1.0 / (n3 + 1))
    lf = w1024["leaf"]
    runs = [(f"p{pp}_{name}", pp, prec, k3, lf) for pp in (4, 6, 8)
            for name, prec in (("mixed", hfmm.FP32), ("fp64", hfmm.FP64))]
    runs += [("p6_mixed_matched_k0", 6, hfmm.FP32, k3m, lf), ("p6_fp64_matched_k0", 6, hfmm.FP64, k3m, lf)]
    # the leaf size chosen by the solver's own timing of its two passes (16, 32 or 64)
    runs += [("p6_mixed_leaf_auto", 6, hfmm.FP32, k3, 0), ("p6_fp64_leaf_auto", 6, hfmm.FP64, k3, 0)]
    for name, pp, prec, k0, leaf in runs:
        t0 = time.perf_counter()
        s = hfmm.Solver(n3, k0, k2_const=k3 ** 2, p=pp, leaf_size=leaf, prec=prec)
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        dt, x, info = timed_solves(s, f, 2, restart=50, rtol=1e-6, maxit=3000)
        out[name] = {"k0": round(k0, 4), "solves_s": round(1 / dt, 4), "s_per_solve": round(dt, 4),
                     "iters": info["iters"], "rel_res_true": info["rel_res_true"], "converged": info["converged"],
                     "ms_precond_per_iter": round(info["ms_precond"] / max(1, info["iters"]), 4),
                     "ms_krylov_per_iter": round(info["ms_krylov"] / max(1, info["iters"]), 4),
                     "setup_s": round(setup, 3), "levels": s.info()["levels"], "leaf": s.info()["leaf_size"]}
        log(f"1024^2 solve {name}: {out[name]}")
        del s
    for pp in (4, 6, 8):
        out[f"p{pp}_mixed_over_fp64_speedup"] = round(out[f"p{pp}_fp64"]["s_per_solve"] /
                                                      out[f"p{pp}_mixed"]["s_per_solve"], 3)
    out["p6_mixed_over_fp64_speedup_matched_k0"] = round(
        out["p6_fp64_matched_k0"]["s_per_solve"] / out["p6_mixed_matched_k0"]["s_per_solve"], 3)
    # the first FMM pass (sources h^2 f at the interior nodes) against the stored direct sum
    pts = solver_tree_points(n3)
    t3 = hfmm.Tree(torch.from_numpy(pts).to(dev), leaf_size=w1024["leaf"])
    g3 = np.load(os.path.join(ROOT, "tests", "golden", "pass_1024_reference.npz"))
    q = np.zeros(len(pts), dtype=np.complex128)
    q[: n3 * n3] = w1024["h"] ** 2 * w1024["f"]
    err = {}
    for pp in (4, 6, 8):
        row = {"eps_oracle": float(g3[f"eps_oracle_p{pp}"])}
        for name, prec, dt_ in (("fp32", hfmm.FP32, np.complex64), ("fp64", hfmm.FP64, np.complex128)):
            phi = hfmm.hfmm_fmm_apply(t3, k3, pp, torch.from_numpy(q.astype(dt_)).to(dev), prec=prec)
            o = phi.cpu().numpy()[g3["samples"]]
            row[name] = float(np.linalg.norm(o - g3["direct"]) / np.linalg.norm(g3["direct"]))
        err[f"p{pp}"] = row
    out["pass1_rel_err_2048_samples"] = err
    log(f"1024^2 pass-1 errors: {err}")
    qq = torch.ones(len(pts), dtype=torch.complex64, device=dev)
    for name, prec, qv in (("fp32", hfmm.FP32, qq), ("fp64", hfmm.FP64, qq.to(torch.complex128))):
        hfmm.hfmm_fmm_apply_timed(t3, k3, 6, qv, prec=prec)
        _, ms = hfmm.hfmm_fmm_apply_timed(t3, k3, 6, qv, prec=prec)
        out[f"fmm_pass_stage_ms_{name}"] = {s_: round(v, 4) for s_, v in ms.items()}
        orders = hfmm.hfmm_fmm_plan_info(t3, k3, 6, prec)["orders"]
        out[f"fmm_pass_m2l_roofline_{name}"] = m2l_roofline(t3, orders, ms["m2l"], name, f"pass_1024_p6_{name}")
    out["orders_p6"] = hfmm.hfmm_fmm_plan_info(t3, k3, 6, hfmm.FP32)["orders"]
    log(f"1024^2 pass stages: {out['fmm_pass_stage_ms_fp32']}")
    return out


def bench_batch_16x4(dev, hfmm, workloads, torch):
    """16 problems x 4 right-hand sides: the dispersion-matched variant
    (FGMRES(200)) graph vs eager, and the survey's settings (k0 = k,
    FGMRES(50), non-convergence reported)."""
    wb = workloads.batch_16x4()
    out = {"problems": [(pr["n"], round(pr["k"], 2)) for pr in wb["problems"]]}
    bs = [torch.from_numpy(pr["f"].astype(np.complex128)).to(dev) for pr in wb["problems"]]
    for variant, matched, restart, maxit in (("matched_k0_restart200", True, 200, 3000),
                                            ("k0_eq_k_restart50", False, 50, 1500)):
        t0 = time.perf_counter()
        solvers = []
        for pr in wb["problems"]:
            k0 = hfmm.hfmm_matched_wavenumber(pr["k"], pr["h"]) if matched else pr["k"]
            solvers.append(hfmm.Solver(pr["n"], k0, k2_const=pr["k"] ** 2, p=wb["p"], leaf_size=wb["leaf"],
                                       prec=hfmm.FP32, nrhs=4))
        torch.cuda.synchronize()
        row = {"setup_s": round(time.perf_counter() - t0, 3), "restart": restart, "maxit": maxit,
               "k0": "matched" if matched else "k"}
        modes = (("graph", True), ("eager", False)) if matched else (("graph", True),)
        if matched:  # one untimed batch per mode: first-use costs (the graph capture, workspace) stay out
            for _, graph in modes:
                hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=restart, rtol=wb["rtol"], maxit=maxit,
                                               use_graph=graph)
            torch.cuda.synchronize()
        for mode, graph in modes:
            t0 = time.perf_counter()
            xs, infos = hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=restart, rtol=wb["rtol"], maxit=maxit,
                                                       use_graph=graph)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            row[mode] = {"solves_s": round(64 / dt, 3), "t_batch_s": round(dt, 4),
                         "converged": sum(i["converged"] for i in infos), "iters": [i["iters"] for i in infos],
                         "max_rel_res": max(i["rel_res_true"] for i in infos)}
            log(f"16x4 batch {variant} {mode}: {row[mode]}")
        if "eager" in row:
            row["graph_over_eager_speedup"] = round(row["eager"]["t_batch_s"] / row["graph"]["t_batch_s"], 3)
        out[variant] = row
        del solvers
    return out


def bench_batch_small(dev, hfmm, workloads, torch):
    """16 small problems (64 x 64 grids, k = 8..23, one right-hand side each,
    FGMRES(30) to 1e-6): graph vs eager where launches, not the FMM's work,
    set the pace of an Arnoldi step."""
    n = 64
    rng = np.random.default_rng(11)
    ks = [8.0 + i for i in range(16)]
    solvers = [hfmm.Solver(n, k, p=6, leaf_size=32, prec=hfmm.FP32) for k in ks]
    bs = [torch.from_numpy(workloads.complex_normal(rng, n * n)).to(dev) for _ in ks]
    torch.cuda.synchronize()
    out = {"problems": len(ks), "n": n, "k": [ks[0], ks[-1]]}
    for _, graph in (("graph", True), ("eager", False)):  # untimed first batch per mode
        hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=30, rtol=1e-6, use_graph=graph)
    torch.cuda.synchronize()
    for mode, graph in (("graph", True), ("eager", False)):
        reps = 3
        t0 = time.perf_counter()
        for _ in range(reps):
            _, infos = hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=30, rtol=1e-6, use_graph=graph)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[mode] = {"t_batch_s": round(dt, 5), "solves_s": round(len(ks) / dt, 2),
                     "converged": sum(i["converged"] for i in infos), "iters": [i["iters"] for i in infos]}
        log(f"16 x 64^2 batch {mode}: {out[mode]}")
    out["graph_over_eager_speedup"] = round(out["eager"]["t_batch_s"] / out["graph"]["t_batch_s"], 3)
    del solvers
    return out


def bench_adjoint_256(dev, hfmm, workloads, torch):
    from oracle import adjoint as oadj
    from paper_1608_02461_amd.autograd import helmholtz_solve
    wa = workloads.adjoint_256()
    n5 = wa["n"]
    s5 = hfmm.Solver(n5, wa["k0"], p=wa["p"], leaf_size=wa["leaf"], prec=hfmm.FP32)
    d5 = hfmm.Solver(n5, wa["k0"], p=wa["p"], leaf_size=wa["leaf"], prec=hfmm.FP32)
    f5 = torch.from_numpy(wa["f"]).to(dev)
    ud, _ = d5.solve(f5, restart=200, rtol=1e-10, strict=True)
    P5 = torch.from_numpy(wa["P"]).to(dev)
    dd = ud[P5]
    del d5

    def fwd_bwd(rtol):
        kbt = torch.from_numpy(wa["kb"]).to(dev).requires_grad_(True)
        u = helmholtz_solve(kbt, f5, s5, restart=200, rtol=rtol)
        r = u[P5] - dd
        J = 0.5 * (r.real ** 2 + r.imag ** 2).sum()
        J.backward()
        return J.item(), kbt.grad.cpu().numpy()

    fwd_bwd(1e-10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J5, g5 = fwd_bwd(1e-10)
    torch.cuda.synchronize()
    t_fb = time.perf_counter() - t0
    t0 = time.perf_counter()
    J6, g6 = fwd_bwd(1e-6)
    torch.cuda.synchronize()
    t_fb6 = time.perf_counter() - t0
    Jo, Go, _, _ = oadj.gradient(n5, wa["kb"], wa["f"], wa["P"], dd.cpu().numpy())
    out = {"fwd_bwd_s_rtol1e-10": round(t_fb, 4), "fwd_bwd_s_rtol1e-6": round(t_fb6, 4),
           "grad_rel_err_vs_oracle_rtol1e-10": float(np.linalg.norm(g5 - Go) / np.linalg.norm(Go)),
           "grad_rel_err_vs_oracle_rtol1e-6": float(np.linalg.norm(g6 - Go) / np.linalg.norm(Go)),
           "J_rel_err": abs(J5 - Jo) / abs(Jo)}
    log(f"256^2 adjoint: {out}")
    return out


def bench_solve_64(dev, hfmm, workloads, torch):
    w64 = workloads.solve_64()
    s = hfmm.Solver(w64["n"], w64["k"], p=6, leaf_size=32, prec=hfmm.FP64)
    f1 = torch.from_numpy(w64["f"]).to(dev)
    dt, x, info = timed_solves(s, f1, 5, restart=30, rtol=1e-6)
    out = {"solves_s": round(1 / dt, 3), "iters": info["iters"], "rel_res_true": info["rel_res_true"],
           "setup_ms": round(info["ms_setup"], 3)}
    # the same solve in graph mode (the batched entry point with one problem):
    # its Arnoldi step replayed from a captured graph, flags read every 4 steps
    hfmm.hfmm_fgmres_solve_batched([s], [f1], restart=30, rtol=1e-6, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        _, ig = hfmm.hfmm_fgmres_solve_batched([s], [f1], restart=30, rtol=1e-6, use_graph=True)
    torch.cuda.synchronize()
    dg = (time.perf_counter() - t0) / 5
    out["graph"] = {"solves_s": round(1 / dg, 3), "iters": ig[0]["iters"], "rel_res_true": ig[0]["rel_res_true"]}
    log(f"64^2 solve: {out}")
    return out


def helm2_problem(mu, n):
    """Sec. 6, eq. helm2 on the unit square with kappa = mu sqrt(2), right-hand side
    negated (-Laplace(u) - k^2 u = f): exact u = x^2 sin(mu x) cos(mu y).  Returns
    k, the exact solution at the interior nodes, f, the boundary data at the
    element midpoints and the FD right-hand side with the Dirichlet ghosts."""
    from paper_1608_02461_amd import workloads
    h = 1.0 / (n + 1)
    xo = workloads.interior_xy(n)
    ue = lambda X, Y: X ** 2 * np.sin(mu * X) * np.cos(mu * Y)
    f = -(2 * np.sin(mu * xo[:, 0]) * np.cos(mu * xo[:, 1]) +
          4 * mu * xo[:, 0] * np.cos(mu * xo[:, 0]) * np.cos(mu * xo[:, 1])) + 0j
    m = (np.arange(n + 1) + 0.5) * h
    z, o = np.zeros_like(m), np.ones_like(m)
    g = np.concatenate([ue(m, z), ue(o, m), ue(m, o), ue(z, m)]) + 0j
    b = f.copy()
    ix, iy = np.arange(n * n) % n, np.arange(n * n) // n
    for dx, dy in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ghost = (ix + dx < 0) | (ix + dx >= n) | (iy + dy < 0) | (iy + dy >= n)
        b[ghost] += ue((ix[ghost] + 1 + dx) * h, (iy[ghost] + 1 + dy) * h) / h ** 2
    return mu * np.sqrt(2.0), ue(xo[:, 0], xo[:, 1]) + 0j, f, g, b


def bench_helm2(dev, hfmm, torch):
    """The paper's inhomogeneous-Dirichlet family (Sec. 6, eq. helm2, Table t:p3)
    on the FD grid: FGMRES(30) iterations from x0 = 0 (the paper's setting) and
    from the boundary-element solution with the Dirichlet data (double layer
    and 1/2 delta), the error of both against the exact solution, p = 6, FP64
    preconditioner.  Table t:p3 is FEM with a degraded direct sum: context."""
    paper_fmm = {1: (7, 6, 6), 4: (7, 6, 6), 6: (6, 6, 6), 8: (7, 7, 6)}
    out = {}
    for mu in (1, 4, 6, 8):
        for hi, n in enumerate((31, 63, 127)):
            k, ue, f, g, b = helm2_problem(float(mu), n)
            s = hfmm.Solver(n, k, p=6, leaf_size=16, prec=hfmm.FP64)
            ft, gt, bt = (torch.from_numpy(a).to(dev) for a in (f, g, b))
            ub = s.dirichlet_apply(ft, gt)
            x0, i0 = s.solve(bt, restart=30, rtol=1e-6)
            x1, i1 = s.solve(bt, x0=ub, restart=30, rtol=1e-6)
            rel = lambda a: float(np.linalg.norm(a.cpu().numpy() - ue) / np.linalg.norm(ue))
            out[f"mu{mu}_h2^-{hi + 5}"] = {
                "n": n, "k": round(k, 4), "iters_x0_zero": i0["iters"], "iters_x0_bem": i1["iters"],
                "converged": i0["converged"] and i1["converged"], "bem_solution_rel_err": rel(ub),
                "fd_solution_rel_err": rel(x0), "paper_fmm_iters_fem": paper_fmm[mu][hi]}
            del s
        log(f"helm2 mu={mu}: {[out[f'mu{mu}_h2^-{e}'] for e in (5, 6, 7)]}")
    return out


def helm1_problem(kappa, n):
    """Sec. 6, eq. helm1 on [-1, 1]^2 mapped to the unit square (x = 2x' - 1):
    k' = 2 kappa, f' = -4 exp(-10((y - 1)^2 + (x - 0.5)^2)) (negated), zero
    Dirichlet data; h = 2^-5 on [-1, 1]^2 is n = 63 here."""
    from paper_1608_02461_amd import workloads
    xo = workloads.interior_xy(n)
    X, Y = 2 * xo[:, 0] - 1, 2 * xo[:, 1] - 1
    return 2.0 * kappa, -4.0 * np.exp(-10 * ((Y - 1) ** 2 + (X - 0.5) ** 2)) + 0j


def bench_bicgstab(dev, hfmm, torch):
    """Sec. 3 (Fig. gmres_bigcstab): FMM-preconditioned GMRES vs BiCGSTAB iterations
    to 1e-6 on helm1, h = 2^-5 (n = 63 on the unit square), p = 6, FP64.  A BiCGSTAB
    iteration costs two preconditioner applies."""
    out = {}
    for kappa in (2.0, 5.0, 7.0, 10.0, 15.0):
        k, f = helm1_problem(kappa, 63)
        s = hfmm.Solver(63, k, p=6, leaf_size=16, prec=hfmm.FP64)
        ft = torch.from_numpy(f).to(dev)
        _, ig = s.solve(ft, restart=30, rtol=1e-6)
        _, ib = s.bicgstab(ft, rtol=1e-6)
        out[f"kappa{kappa:g}"] = {"fgmres_iters": ig["iters"], "bicgstab_iters": ib["iters"],
                                  "fgmres_precond_applies": ig["iters"], "bicgstab_precond_applies": 2 * ib["iters"],
                                  "converged": ig["converged"] and ib["converged"],
                                  "fgmres_ms": round(ig["ms_total"], 3), "bicgstab_ms": round(ib["ms_total"], 3)}
        del s
    log(f"BiCGSTAB vs FGMRES: {out}")
    return out


def bench_pstudy(dev, hfmm, workloads, torch):
    """Sec. 6.1 (Fig. convergence): FGMRES(30) iterations against the expansion
    order p in FP64 and FP32, on helm1 (kappa = 7, h = 2^-5) and the 64 x 64
    workload, with the preconditioner apply's error against the oracle's dense
    M^-1 for each (p, precision)."""
    from oracle import bem
    out = {}
    cases = {"helm1_kappa7": helm1_problem(7.0, 63) + (63,)}
    w64 = workloads.solve_64()
    cases["solve_64"] = (w64["k"], w64["f"], w64["n"])
    for cname, (k, f, n) in cases.items():
        ref = bem.precond_apply(n, k, f)
        ft = torch.from_numpy(f).to(dev)
        for pp in (2, 4, 6, 8, 12):
            for pname, prec in (("fp64", hfmm.FP64), ("fp32", hfmm.FP32)):
                s = hfmm.Solver(n, k, p=pp, leaf_size=16, prec=prec)
                z = s.precond_apply(ft).cpu().numpy()
                _, info = s.solve(ft, restart=30, rtol=1e-6)
                out[f"{cname}_p{pp}_{pname}"] = {
                    "iters": info["iters"], "converged": info["converged"],
                    "precond_rel_err_vs_dense": float(np.linalg.norm(z - ref) / np.linalg.norm(ref))}
                if pname == "fp32" and pp in (4, 6, 8):
                    # M2L operands rounded to 16-bit formats (FP32 products)
                    for rname in ("fp16", "bf16"):
                        s.set_m2l_input_rounding(rname)
                        z = s.precond_apply(ft).cpu().numpy()
                        _, info = s.solve(ft, restart=30, rtol=1e-6, maxit=1000)
                        out[f"{cname}_p{pp}_fp32_m2l_{rname}"] = {
                            "iters": info["iters"], "converged": info["converged"],
                            "precond_rel_err_vs_dense": float(np.linalg.norm(z - ref) / np.linalg.norm(ref))}
                del s
        log(f"p study {cname}: " + ", ".join(f"{kk}: {v['iters']}" for kk, v in out.items() if kk.startswith(cname)))
    return out


def bench_m2l_rounding(dev, hfmm, workloads, torch, tree, gold, smp):
    """The 16-bit M2L experiment at scale: the N = 2^20 apply's error on the
    stored samples with the M2L operands rounded to FP16 / BF16 (p = 4, 8,
    12), and the 1024 x 1024 solve (matched k0, p = 6) with each."""
    w = workloads.fmm_2p20()
    q32 = torch.from_numpy(w["q"].astype(np.complex64)).to(dev)
    out = {}
    for rname in ("none", "fp16", "bf16"):
        tree.set_m2l_input_rounding(rname)
        for pp in (4, 8, 12):
            phi = hfmm.hfmm_fmm_apply(tree, w["k"], pp, q32, prec=hfmm.FP32).cpu().numpy()[smp]
            out[f"apply_2p20_p{pp}_{rname}_rel_err"] = float(np.linalg.norm(phi - gold["direct"]) /
                                                    np.linalg.norm(gold["direct"]))
    tree.set_m2l_input_rounding("none")
    w1024 = workloads.solve_1024()
    n3, k3 = w1024["n"], w1024["k"]
    k0 = hfmm.hfmm_matched_wavenumber(k3, 1.0 / (n3 + 1))
    f = torch.from_numpy(w1024["f"]).to(dev)
    s = hfmm.Solver(n3, k0, k2_const=k3 ** 2, p=6, leaf_size=w1024["leaf"], prec=hfmm.FP32)
    for rname in ("none", "fp16", "bf16"):
        s.set_m2l_input_rounding(rname)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = s.solve(f, restart=50, rtol=1e-6, maxit=600)
        torch.cuda.synchronize()
        out[f"solve_1024_matched_p6_{rname}"] = {"iters": info["iters"], "converged": info["converged"],
                                                 "rel_res_true": info["rel_res_true"],
                                                 "s": round(time.perf_counter() - t0, 4), "maxit": 600}
    del s
    log(f"M2L rounding: {out}")
    return out


def bench_hbm(dev, hfmm, workloads, torch, xy_2p20):
    """HBM-bound parts timed with hipEvents on the launch stream: the FD matvec on
    1024 x 1024 (32 algorithmic bytes per point: x read once, y written once,
    complex128; neighbours come from cache) and the tree build of the 2^20 apply points
    (a rough 40 bytes per point per pass, several passes)."""
    n = 1024
    x = torch.randn(n * n, dtype=torch.complex128, device=dev)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    y = hfmm.hfmm_fd_helmholtz_matvec(n, 1.0 / (n + 1), x, k2_const=1e4)
    torch.cuda.synchronize()
    reps = 50
    e0.record(st)
    for _ in range(reps):
        y = hfmm.hfmm_fd_helmholtz_matvec(n, 1.0 / (n + 1), x, k2_const=1e4)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out = {"fd_matvec_1024": {"ms": round(ms, 5), "algorithmic_bytes": 32 * n * n,
                              "gb_s": round(32 * n * n / (ms * 1e-3) / 1e9, 1), "peak_gb_s": PEAK_HBM,
                              "note": "includes the binding's output allocation and column-major copy"}}
    log(f"HBM: {out}")
    return out


def cpu_direct_sum_baseline(w, smp, k, N):
    """The oracle's direct N-body sum on a bounded target sample, scaled by
    linearity to Mpts/s of the full N x N sum."""
    from concurrent.futures import ThreadPoolExecutor

    from threadpoolctl import threadpool_limits

    from oracle import kernel

    avail = len(os.sched_getaffinity(0))
    # one oracle call per thread; the GPU machine's CPU share is 16 threads
    nthr = max(1, min(16, avail))
    n_t = 64 * nthr
    tg = w["xy"][smp[:n_t]] if n_t <= len(smp) else w["xy"][:n_t]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(nthr) as ex:
            list(ex.map(lambda i: kernel.direct_sum(w["xy"], w["q"], k, tgt=tg[i::nthr]), range(nthr)))
        dt = time.perf_counter() - t0
    full = dt / n_t * N
    return {"value": round(N / full / 1e6, 6), "unit": "Mpts/s", "cores": nthr, "kind": "oracle",
            "sample": f"oracle direct N-body sum (scipy hankel1, FP64) from all {N} sources to {n_t} of the "
                      f"seeded targets ({dt:.1f} s on {nthr} threads, one oracle call per thread); Mpts/s of "
                      f"the full N x N sum by linearity",
            "pairs_per_s": round(n_t * N / dt, 1), "sched_getaffinity_cores": avail, "cpu_model": cpu_model(),
            "blas_threads_per_call": 1}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_extra_baselines(workloads):
    """The oracle on the host for the other workloads: the 64 x 64 solve
    (dense M^-1 formed from the paper's equations, then FGMRES(30)), the
    1024 x 1024 system by sparse LU (scipy splu: a different method, the CPU
    reference solution), and the adjoint gradient on 256 x 256 (sparse direct)."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import adjoint as oadj
    from oracle import bem, fd, fgmres
    out = {"blas": [{"api": i.get("internal_api"), "threads": i.get("num_threads")} for i in threadpool_info()],
           "threads_cap": 16}
    with threadpool_limits(16):
        w64 = workloads.solve_64()
        A = fd.matrix(w64["n"], w64["k"] ** 2)
        t0 = time.perf_counter()
        Minv = bem.precond_matrix(w64["n"], w64["k"])
        t1 = time.perf_counter()
        x, info = fgmres.fgmres(lambda v: A @ v, lambda v: Minv @ v, w64["f"], restart=30, rtol=1e-6)
        t2 = time.perf_counter()
        out["solve_64_oracle_dense_fgmres"] = {"form_Minv_s": round(t1 - t0, 3), "fgmres_s": round(t2 - t1, 4),
                                               "solves_s": round(1 / (t2 - t0), 4), "iters": info["iters"]}
        log(f"CPU 64^2 solve: {out['solve_64_oracle_dense_fgmres']}")
        w1024 = workloads.solve_1024()
        from scipy.sparse.linalg import splu
        A3 = fd.matrix(w1024["n"], w1024["k"] ** 2).tocsc()
        t0 = time.perf_counter()
        lu = splu(A3)
        t1 = time.perf_counter()
        x3 = lu.solve(w1024["f"])
        t2 = time.perf_counter()
        out["solve_1024_cpu_sparse_direct_reference"] = {
            "factor_s": round(t1 - t0, 2), "solve_s": round(t2 - t1, 3), "solves_s": round(1 / (t2 - t0), 5),
            "rel_res": float(np.linalg.norm(w1024["f"] - A3 @ x3) / np.linalg.norm(w1024["f"])),
            "label": "CPU sparse-direct reference (different method)"}
        log(f"CPU 1024^2 solve: {out['solve_1024_cpu_sparse_direct_reference']}")
        del lu
        wa = workloads.adjoint_256()
        u_ref = oadj.solve(wa["n"], wa["k2_ref"], wa["f"])
        d = u_ref[wa["P"]]
        t0 = time.perf_counter()
        oadj.gradient(wa["n"], wa["kb"], wa["f"], wa["P"], d)
        out["adjoint_256_oracle_gradient_s"] = round(time.perf_counter() - t0, 3)
        # the 3-D apply: the oracle's direct sum from all 2^20 sources to 64
        # sampled targets (Mpts/s of the full N x N sum by linearity)
        from oracle import fmm3 as ofmm3
        w3 = workloads.fmm3_2p20()
        tg = w3["samples"][:64]
        t0 = time.perf_counter()
        ofmm3.direct_sum3(w3["xyz"], w3["q"], w3["k"], targets=w3["xyz"][tg], chunk=8)
        dt = time.perf_counter() - t0
        n3 = len(w3["xyz"])
        out["fmm3_2p20_oracle_direct_sum"] = {
            "sample": f"all {n3} sources to 64 sampled targets, numpy FP64, {round(dt, 2)} s",
            "pairs_per_s": round(64 * n3 / dt, 1), "Mpts_per_s_full_sum": round(64 / dt / 1e6, 9)}
        log(f"CPU 3-D direct sum: {out['fmm3_2p20_oracle_direct_sum']}")
    return out


def m2l3_flops(L, orders):
    """The 3-D M2L per apply: algorithmic flops (8 P^4 per (target, source)
    pair of the interaction lists inside the cube, P^2 = (p_l + 1)^2
    coefficients; a complex multiply-add is 8 real flops) and the MFMA flops
    the kernel executes: a wave of 32 class members (columns) runs the real
    2P^2 x 2P^2 product, rows padded to a multiple of 16 and k to one of 4,
    for every offset of its class for which one of its members has a source."""
    alg, exe = 0, 0
    for l in range(2, L + 1):
        nb, h = 2 ** l, 2 ** (l - 1)
        P2 = (orders[l] + 1) ** 2
        kp = (2 * P2 + 15) // 16 * 16
        ke = (2 * P2 + 3) // 4 * 4  # the k extent the kernel multiplies (K padding skipped)
        m = np.arange(h ** 3)
        wave = m // 32
        nw = int(wave.max()) + 1
        for par in range(8):
            px, py, pz = par & 1, (par >> 1) & 1, (par >> 2) & 1
            tx, ty, tz = 2 * (m % h) + px, 2 * ((m // h) % h) + py, 2 * (m // (h * h)) + pz
            for dx in range(px - 3, px + 3):
                for dy in range(py - 3, py + 3):
                    for dz in range(pz - 3, pz + 3):
                        if max(abs(dx), abs(dy), abs(dz)) <= 1:
                            continue
                        sx, sy, sz = tx - dx, ty - dy, tz - dz
                        ok = (sx >= 0) & (sx < nb) & (sy >= 0) & (sy < nb) & (sz >= 0) & (sz < nb)
                        alg += int(np.count_nonzero(ok)) * 8 * P2 * P2
                        waves_on = np.count_nonzero(np.bincount(wave[ok], minlength=nw))
                        exe += int(waves_on) * 32 * 2 * kp * ke
    return alg, exe


def p2p3_pairs(xyz, L):
    """Near-field pairs of the oct-tree (27 neighbouring leaves, self pairs excluded)."""
    nb = 2 ** L
    ib = np.clip(np.floor(xyz * nb).astype(np.int64), 0, nb - 1)
    cnt = np.zeros((nb, nb, nb), dtype=np.int64)
    np.add.at(cnt, (ib[:, 0], ib[:, 1], ib[:, 2]), 1)
    pad = np.pad(cnt, 1)
    nsum = np.zeros_like(cnt)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                nsum += pad[1 + dx:1 + dx + nb, 1 + dy:1 + dy + nb, 1 + dz:1 + dz + nb]
    return int((cnt * nsum).sum() - len(xyz))


P2P3_FLOPS_PER_PAIR = 23  # difference 3 + offset 3, r^2 5, sqrt 1, 1/r 1, k r 1, cos and sin 2, G 2, complex MAC 4 + 1 scale


def bench_fmm3(dev, hfmm, workloads, torch, runs=10):
    """The 3-D oct-tree apply (N = 2^20 uniform in the unit cube, k = 10, p = 6,
    leaf 64): tree build, throughput and per-stage device times in both
    precisions, the M2L against the MFMA peak of its precision and the P2P
    pair rate."""
    w = workloads.fmm3_2p20()
    xyz = torch.from_numpy(w["xyz"]).to(dev)
    N, k, p = len(w["xyz"]), w["k"], w["p"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tree = hfmm.Tree3(xyz, leaf_size=w["leaf"])
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    tree2 = hfmm.Tree3(xyz, leaf_size=w["leaf"])
    torch.cuda.synchronize()
    t_second = time.perf_counter() - t0
    tree2.close()
    info = tree.info()
    L = info["levels"]
    orders = tree.orders(k, p)
    alg, exe = m2l3_flops(L, orders)
    pairs = p2p3_pairs(w["xyz"], L)
    out = {"workload": f"3-D FMM apply, N=2^20 uniform points in the unit cube, complex N(0,1) charges, k={k}, "
                       f"leaf {w['leaf']}, p={p}", "levels": L, "orders": orders,
           "max_leaf": info["max_leaf_count"], "tree_build_first_ms": round(t_first * 1e3, 3),
           "tree_build_ms": round(t_second * 1e3, 3), "m2l_algorithmic_flops": alg, "m2l_executed_flops": exe,
           "p2p_pairs": pairs}
    # calibrated HBM bytes of the M2L stage from the committed counters
    rec3 = profile_record(FMM3_SUMMARY, "k3_trans")
    phis = {}
    for name, prec, dt, peak in (("fp32", hfmm.FP32, torch.complex64, 157.3), ("fp64", hfmm.FP64, torch.complex128, 78.6)):
        q = torch.from_numpy(w["q"]).to(dt).to(dev)
        t0 = time.perf_counter()
        hfmm.hfmm3_fmm_apply(tree, k, p, q, prec=prec)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        for _ in range(2):
            hfmm.hfmm3_fmm_apply(tree, k, p, q, prec=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(runs):
            phi = hfmm.hfmm3_fmm_apply(tree, k, p, q, prec=prec)
        torch.cuda.synchronize()
        dt_s = (time.perf_counter() - t0) / runs
        st = {s: 0.0 for s in hfmm.STAGES3}
        for _ in range(runs):
            _, ms = hfmm.hfmm3_fmm_apply_timed(tree, k, p, q, prec=prec)
            for s_ in st:
                st[s_] += ms[s_] / runs
        phis[name] = phi.to(torch.complex128).cpu().numpy()
        m2l_s = st["m2l"] * 1e-3
        out[name] = {
            "ms_per_apply": round(dt_s * 1e3, 4), "Mpts_per_s": round(N / dt_s / 1e6, 2),
            "first_apply_with_plan_s": round(t_plan, 3),
            "stage_ms": {s_: round(v, 4) for s_, v in st.items()},
            "m2l_roofline": {"bound": "mfma", "achieved": round(alg / m2l_s / 1e12, 3), "peak": peak,
                             "unit": "TFLOP/s", "frac": round(alg / m2l_s / 1e12 / peak, 4),
                             "traffic": (rec3["m2l_stage_traffic_bytes_fp32"] if rec3 and name == "fp32" else None),
                             "executed_TFLOP_s": round(exe / m2l_s / 1e12, 3),
                             "executed_over_algorithmic": round(exe / alg, 3)},
            "p2p_pairs_per_s": round(pairs / (st["p2p"] * 1e-3), 1),
            "p2p_alu_TFLOP_s": round(pairs * P2P3_FLOPS_PER_PAIR / (st["p2p"] * 1e-3) / 1e12, 3),
        }
        log(f"3-D apply {name}: {out[name]}")
    out["fp32_vs_fp64_rel"] = float(np.linalg.norm(phis["fp32"] - phis["fp64"]) / np.linalg.norm(phis["fp64"]))
    tree.close()
    return out


def bench_helm3(dev, hfmm, workloads, torch):
    """The 3-D model problem (7-point grid, n^3 unknowns, k = 10): FGMRES(30)
    to 1e-6 with the oct-tree FMM volume potential as the preconditioner, in
    FP32 and FP64, for n = 63 and 127 at p = 6, and at n = 127 also p = 3
    (a cheaper, less accurate preconditioner)."""
    out = {}
    for n, p in ((63, 6), (127, 6), (127, 3)):
        w = workloads.helm3_cube(n)
        b = torch.from_numpy(w["b"]).to(dev)
        row = {"unknowns": n ** 3, "p": p}
        for name, prec in (("fp32", hfmm.FP32), ("fp64", hfmm.FP64)):
            t0 = time.perf_counter()
            s = hfmm.Solver3(n, w["k"], p=p, leaf_size=w["leaf"], prec=prec)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            s.solve(b, restart=30, rtol=1e-6)  # untimed: first-use costs
            torch.cuda.synchronize()
            reps = 2
            t0 = time.perf_counter()
            for _ in range(reps):
                x, info = s.solve(b, restart=30, rtol=1e-6)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            row[name] = {"s_per_solve": round(dt, 4), "iters": info["iters"], "converged": info["converged"],
                         "rel_res_true": info["rel_res_true"], "ms_precond_per_iter":
                         round(info["ms_precond"] / max(1, info["iters"]), 3),
                         "ms_krylov_total": round(info["ms_krylov"], 2), "setup_s": round(t_setup, 3),
                         "levels": s.info()["levels"]}
            log(f"3-D model problem n={n} p={p} {name}: {row[name]}")
            s.close()
        row["mixed_over_fp64"] = round(row["fp64"]["s_per_solve"] / row["fp32"]["s_per_solve"], 3)
        out[f"n{n}" if p == 6 else f"n{n}_p{p}"] = row
    return out


PROFILE_CASES = ("apply-2p20-fp64", "pass-1024-fp32", "pass-1024-fp64", "solve-1024", "apply3-2p20-fp32",
                 "apply3-2p20-fp64", "solve3-127-fp32")


def copy_probe(torch, dev):
    """One device-to-device copy of 64 Mi doubles (512 MiB read, 512 MiB
    written): the calibration of the HBM byte counters."""
    src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def profile_case(name, steps, warmup, probe):
    """One workload alone, for a profiler (no JSON line):
    apply-2p20-fp64        the headline apply in complex128 (N = 2^20, k = 100, leaf 64, p = 8);
    pass-1024-fp32   the first FMM pass of the 1024 x 1024 preconditioner (sources
    pass-1024-fp64   h^2 f at the interior nodes, k h = 0.3, leaf 32, p = 6);
    solve-1024       solver set-up (tree, boundary inverse, plans) then `steps`
                   complex64-preconditioned FGMRES(50) solves of that system with
                   the dispersion-matched k0, p = 6;
    apply3-2p20-fp32 the 3-D oct-tree apply (N = 2^20 in the unit cube, k = 10,
    apply3-2p20-fp64 leaf 64, p = 6), its stages one after another;
    solve3-127-fp32  the 3-D model problem on 127^3 nodes (k = 10, p = 6,
                   leaf 64): set-up, then `steps` FGMRES(30) solves to 1e-6
                   with the complex64 volume-potential preconditioner."""
    import torch
    from paper_1608_02461_amd import hfmm, workloads
    dev = torch.device("cuda:0")
    if name == "apply-2p20-fp64":
        w = workloads.fmm_2p20()
        tree = hfmm.Tree(torch.from_numpy(w["xy"]).to(dev), leaf_size=w["leaf"])
        q = torch.from_numpy(w["q"]).to(dev)
        run = lambda: hfmm.hfmm_fmm_apply(tree, w["k"], 8, q, prec=hfmm.FP64)
    elif name.startswith("pass-1024"):
        w1024 = workloads.solve_1024()
        n3 = w1024["n"]
        pts = solver_tree_points(n3)
        tree = hfmm.Tree(torch.from_numpy(pts).to(dev), leaf_size=w1024["leaf"])
        q = np.zeros(len(pts), dtype=np.complex128)
        q[: n3 * n3] = w1024["h"] ** 2 * w1024["f"]
        prec, dt = (hfmm.FP32, np.complex64) if name.endswith("fp32") else (hfmm.FP64, np.complex128)
        qd = torch.from_numpy(q.astype(dt)).to(dev)
        run = lambda: hfmm.hfmm_fmm_apply(tree, w1024["k"], 6, qd, prec=prec)
    elif name == "solve-1024":
        w1024 = workloads.solve_1024()
        n3, k3 = w1024["n"], w1024["k"]
        k0 = hfmm.hfmm_matched_wavenumber(k3, 1.0 / (n3 + 1))
        f = torch.from_numpy(w1024["f"]).to(dev)
        s = hfmm.Solver(n3, k0, k2_const=k3 ** 2, p=6, leaf_size=w1024["leaf"], prec=hfmm.FP32)
        warmup = 0
        run = lambda: s.solve(f, restart=50, rtol=1e-6, maxit=3000)
    elif name.startswith("apply3-2p20"):
        w = workloads.fmm3_2p20()
        tree = hfmm.Tree3(torch.from_numpy(w["xyz"]).to(dev), leaf_size=w["leaf"])
        prec, dt = (hfmm.FP32, torch.complex64) if name.endswith("fp32") else (hfmm.FP64, torch.complex128)
        q = torch.from_numpy(w["q"]).to(dt).to(dev)
        # the timed apply: its stages run one after another, as the benchmark's
        # per-stage times (and its M2L roofline) see them
        run = lambda: hfmm.hfmm3_fmm_apply_timed(tree, w["k"], w["p"], q, prec=prec)[0]
    elif name == "solve3-127-fp32":
        w = workloads.helm3_cube(127)
        b3 = torch.from_numpy(w["b"]).to(dev)
        s3 = hfmm.Solver3(w["n"], w["k"], p=w["p"], leaf_size=w["leaf"], prec=hfmm.FP32)
        warmup = 0
        run = lambda: s3.solve(b3, restart=30, rtol=1e-6)
    else:
        raise SystemExit(f"unknown profile case {name}; one of {PROFILE_CASES}")
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    log(f"profile {name}: {steps} runs")
    for _ in range(steps):
        out = run()
    torch.cuda.synchronize()
    if name in ("solve-1024", "solve3-127-fp32"):
        log(f"profile {name}: {out[1]}")
    if probe:
        copy_probe(torch, dev)
    print(f"profile {name} done", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed applies, copy 512 MiB device to device once (counter calibration)")
    ap.add_argument("--profile", choices=PROFILE_CASES,
                    help="run one workload alone for a profiler (steps after warmup) and print no JSON line")
    args = ap.parse_args()
    if args.profile:
        profile_case(args.profile, args.steps, args.warmup, args.copy_probe)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU path "
              "is a design only and is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1608_02461_amd import hfmm, workloads

    dev = torch.device("cuda:0")
    w = workloads.fmm_2p20()
    N, k, leaf, p = len(w["xy"]), w["k"], w["leaf"], args.p
    xy = torch.from_numpy(w["xy"]).to(dev)
    q32 = torch.from_numpy(w["q"].astype(np.complex64)).to(dev)
    q64 = torch.from_numpy(w["q"]).to(dev)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    tree = hfmm.Tree(xy, leaf_size=leaf)
    torch.cuda.synchronize()
    t_tree_first = time.perf_counter() - t0
    # build time of a tree (the trees stay alive, so no teardown is timed)
    t0 = time.perf_counter()
    trees_b = [hfmm.Tree(xy, leaf_size=leaf) for _ in range(5)]
    torch.cuda.synchronize()
    t_tree = (time.perf_counter() - t0) / 5
    del trees_b
    plan = hfmm.hfmm_fmm_plan_info(tree, k, p, hfmm.FP32)
    stream = torch.cuda.current_stream()

    # ---------------- timed region: K FP32 applies
    for _ in range(args.warmup):
        phi = hfmm.hfmm_fmm_apply(tree, k, p, q32, prec=hfmm.FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        phi = hfmm.hfmm_fmm_apply(tree, k, p, q32, prec=hfmm.FP32)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed / args.steps * 1e3
    value = N / (elapsed / args.steps) / 1e6

    if args.copy_probe:
        copy_probe(torch, dev)

    # ---------------- per-stage device times (hipEvents on the launch stream), same applies
    stages = {s: 0.0 for s in hfmm.STAGES}
    for _ in range(args.steps):
        _, ms = hfmm.hfmm_fmm_apply_timed(tree, k, p, q32, prec=hfmm.FP32)
        for s in stages:
            stages[s] += ms[s] / args.steps
    # the dominant kernel is the near field (P2P): about 70% of the kernel
    # time of an apply; it runs beside the far-field chain, so its duration
    # here includes that contention, as in the timed loop above
    fl = plan["pairs"] * p2p_flops_per_pair(plan["near_deg"])
    roof_kernel = f"k_p2p4<float,1,{plan['near_deg']},true,{plan['lanes_per_target']}>"
    ms_p2p = stages["p2p"]
    achieved = fl / (ms_p2p * 1e-3) / 1e12
    L = tree.info()["levels"]
    roofline = {"bound": "alu", "kernel": roof_kernel, "achieved": round(achieved, 3), "peak": PEAK_FP32_ALU,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_ALU, 4),
                "traffic": measured_traffic(roof_kernel),
                "algorithmic_flops_per_launch": fl, "ms_per_launch": round(ms_p2p, 5),
                # positions, sorted charges and the permutation read once, potentials
                # written once (in caller order)
                "algorithmic_bytes_per_launch": (8 + 8 + 4 + 8) * N,
                "pairs_per_s": round(plan["pairs"] / (ms_p2p * 1e-3), 1)}

    gold = np.load(os.path.join(ROOT, "tests", "golden", "apply_2p20_reference.npz"))
    smp = gold["samples"]
    phi_np = phi.cpu().numpy()[smp]
    err32 = float(np.linalg.norm(phi_np - gold["direct"]) / np.linalg.norm(gold["direct"]))

    result = {
        "metric": METRIC, "value": round(value, 3), "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64", "data": "synthetic",
        "config": {"workload": f"FMM apply, N=2^20 uniform points in the unit square, complex N(0,1) charges, "
                               f"k=100, leaf 64, p={p}, complex64", "N": N, "k": k, "p": p, "leaf": leaf,
                   "levels": tree.info()["levels"], "orders": plan["orders"]},
        "stage_ms": {s: round(v, 5) for s, v in stages.items()},
        "tree_build_ms": round(t_tree * 1e3, 4), "tree_build_first_ms": round(t_tree_first * 1e3, 3),
        "rel_err_2048_samples": err32,
        "roofline": roofline,
        # the M2L launch on the far-field chain's stream (beside the near field)
        "m2l_roofline": m2l_roofline(tree, plan["orders"], stages["m2l"], "fp32", f"apply_2p20_p{p}_fp32"),
    }

    if not args.no_extras:
        result["fmm_2p20"] = bench_fmm_orders(tree, k, N, q32, q64, gold, smp, hfmm, torch, plan)
        result["solve_1024"] = bench_solve_1024(dev, hfmm, workloads, torch)
        result["batch_16x4"] = bench_batch_16x4(dev, hfmm, workloads, torch)
        result["batch_16_small"] = bench_batch_small(dev, hfmm, workloads, torch)
        result["adjoint_256"] = bench_adjoint_256(dev, hfmm, workloads, torch)
        result["solve_64"] = bench_solve_64(dev, hfmm, workloads, torch)
        result["helm2_dirichlet"] = bench_helm2(dev, hfmm, torch)
        result["bicgstab_vs_fgmres"] = bench_bicgstab(dev, hfmm, torch)
        result["precond_accuracy_study"] = bench_pstudy(dev, hfmm, workloads, torch)
        result["m2l_16bit_inputs"] = bench_m2l_rounding(dev, hfmm, workloads, torch, tree, gold, smp)
        result["hbm_kernels"] = bench_hbm(dev, hfmm, workloads, torch, xy)
        result["fmm3_2p20"] = bench_fmm3(dev, hfmm, workloads, torch)
        result["helm3_solve"] = bench_helm3(dev, hfmm, workloads, torch)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_direct_sum_baseline(w, smp, k, N)
        if not args.no_extras:
            result["cpu_baselines_extra"] = cpu_extra_baselines(workloads)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
