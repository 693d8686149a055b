"""Benchmark: the 2-D Helmholtz FMM apply (and FMM-BEM preconditioned solves) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--p 8] [--no-extras] [--no-cpu]

Headline workload (one step = one FMM apply, inputs resident in HBM, tree
built beforehand and timed separately): N = 2^20 uniform points in the unit
square, complex N(0,1) charges, k = 100, leaf 64, complex64 arithmetic, order
p (default 8).  value = N / (time per apply) in Mpts/s.

Also reported on the same JSON line:
* the same apply in complex128 and at p = 4, 8, 12, with relative errors on
  the 2048 seeded targets against the stored direct sum;
* the mixed-precision (complex64 FMM inside FP64 FGMRES(50)) and all-FP64
  solves of the 1024 x 1024 grid, k h = 0.3, Gaussian bump, to 1e-6;
* the 64 x 64, k = 16, FP64 FGMRES(30) solve;
* the batched solve of 16 problems x 4 right-hand sides (k in [20, 300], n in
  {128, 256, 384, 512}), one hipGraph-captured Arnoldi step vs eager;
* forward + backward of the block-k^2 adjoint gradient on 256 x 256, checked
  against the CPU oracle's sparse-direct adjoint gradient;
* `roofline` for the dominant kernel of the apply (the near field), from
  hipEvents recorded on its launch stream around it, over the same number of
  applies as the timed steps;
* `cpu_baseline`: the CPU oracle's direct N-body sum on a bounded sample of
  targets, scaled to Mpts/s of the full sum.
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


PMC_SUMMARY = os.path.join(ROOT, "profiles", "p2p_fmm_c2_n1m_k100_p8_fp32_pmc.md")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's reading on
    a plain device copy of known size), or None when the summary is absent,
    is for another kernel, or the near-field source has changed since."""
    import hashlib
    import re
    try:
        txt = open(PMC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", txt, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    src = open(os.path.join(ROOT, rec["source"]), "rb").read()
    if rec["kernel"] != kernel or hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    return rec["bytes_per_launch"]


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
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU design is "
              "described in DESIGN.md and not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1608_02461_amd import hfmm, workloads

    dev = torch.device("cuda:0")
    w = workloads.fmm_c2()
    N, k, leaf, p = len(w["xy"]), w["k"], w["leaf"], args.p
    xy = torch.from_numpy(w["xy"]).to(dev)
    q32 = torch.from_numpy(w["q"].astype(np.complex64)).to(dev)
    q64 = torch.from_numpy(w["q"]).to(dev)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    tree = hfmm.Tree(xy, leaf_size=leaf)
    torch.cuda.synchronize()
    t_tree_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(5):
        tree_b = hfmm.Tree(xy, leaf_size=leaf)
    torch.cuda.synchronize()
    t_tree = (time.perf_counter() - t0) / 5
    del tree_b
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
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

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

    gold = np.load(os.path.join(ROOT, "tests", "golden", "c2_reference.npz"))
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
    }

    if not args.no_extras:
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
            log(f"C2 p={pp}: {row}")
        result["fmm_c2"] = fmm_tab

        # 1024 x 1024 solve, mixed vs FP64
        c3 = workloads.solve_c3()
        f = torch.from_numpy(c3["f"]).to(dev)
        solves = {}
        k3m = hfmm.hfmm_matched_wavenumber(c3["k"], 1.0 / (c3["n"] + 1))
        for name, prec, k0 in (("mixed", hfmm.FP32, c3["k"]), ("fp64", hfmm.FP64, c3["k"]),
                               ("mixed_matched_k0", hfmm.FP32, k3m), ("fp64_matched_k0", hfmm.FP64, k3m)):
            t0 = time.perf_counter()
            s = hfmm.Solver(c3["n"], k0, k2_const=c3["k"] ** 2, p=6, leaf_size=c3["leaf"], prec=prec)
            torch.cuda.synchronize()
            setup = time.perf_counter() - t0
            s.solve(f, restart=50, rtol=1e-6)  # warm
            torch.cuda.synchronize()
            reps = 2
            t0 = time.perf_counter()
            for _ in range(reps):
                x, info = s.solve(f, restart=50, rtol=1e-6)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            solves[name] = {"k0": round(k0, 4), "solves_s": round(1 / dt, 4), "s_per_solve": round(dt, 4),
                            "iters": info["iters"],
                            "rel_res_true": info["rel_res_true"], "converged": info["converged"],
                            "ms_precond_per_iter": round(info["ms_precond"] / max(1, info["iters"]), 4),
                            "setup_s": round(setup, 3)}
            log(f"C3 {name}: {solves[name]}")
            del s
        solves["mixed_over_fp64_speedup"] = round(solves["fp64"]["s_per_solve"] / solves["mixed"]["s_per_solve"], 3)
        solves["mixed_over_fp64_speedup_matched_k0"] = round(
            solves["fp64_matched_k0"]["s_per_solve"] / solves["mixed_matched_k0"]["s_per_solve"], 3)
        # stage times of one FMM pass on the same point set (interior nodes + boundary midpoints)
        n3 = c3["n"]
        h3 = 1.0 / (n3 + 1)
        m = (np.arange(n3 + 1) + 0.5) * h3
        z, o = np.zeros_like(m), np.ones_like(m)
        pts = np.concatenate([workloads.interior_xy(n3), np.stack([m, z], 1), np.stack([o, m], 1),
                              np.stack([m, o], 1), np.stack([z, m], 1)])
        t3 = hfmm.Tree(torch.from_numpy(pts).to(dev), leaf_size=c3["leaf"])
        qq = torch.ones(len(pts), dtype=torch.complex64, device=dev)
        for name, prec, qv in (("fp32", hfmm.FP32, qq), ("fp64", hfmm.FP64, qq.to(torch.complex128))):
            hfmm.hfmm_fmm_apply_timed(t3, c3["k"], 6, qv, prec=prec)
            _, ms = hfmm.hfmm_fmm_apply_timed(t3, c3["k"], 6, qv, prec=prec)
            solves[f"fmm_pass_stage_ms_{name}"] = {s_: round(v, 4) for s_, v in ms.items()}
        solves["orders"] = hfmm.hfmm_fmm_plan_info(t3, c3["k"], 6, hfmm.FP32)["orders"]
        log(f"C3 FMM stages: {solves['fmm_pass_stage_ms_fp32']}")
        result["solve_1024"] = solves

        # batched: 16 problems x 4 right-hand sides, one captured Arnoldi step for all
        c4 = workloads.batch_c4()
        t0 = time.perf_counter()
        solvers, bs = [], []
        for pr in c4["problems"]:
            k0 = hfmm.hfmm_matched_wavenumber(pr["k"], pr["h"])
            solvers.append(hfmm.Solver(pr["n"], k0, k2_const=pr["k"] ** 2, p=c4["p"], leaf_size=c4["leaf"],
                                       prec=hfmm.FP32, nrhs=4))
            bs.append(torch.from_numpy(pr["f"].astype(np.complex128)).to(dev))
        torch.cuda.synchronize()
        setup4 = time.perf_counter() - t0
        maxit4, restart4 = 3000, 200
        batch = {"setup_s": round(setup4, 3), "k0": "matched", "maxit": maxit4, "restart": restart4,
                 "problems": [(pr["n"], round(pr["k"], 2)) for pr in c4["problems"]]}
        log(f"C4 setup {setup4:.2f} s")
        for mode, graph in (("graph", True), ("eager", False)):
            t0 = time.perf_counter()
            xs, infos = hfmm.hfmm_fgmres_solve_batched(solvers, bs, restart=restart4, rtol=c4["rtol"],
                                                       maxit=maxit4, use_graph=graph)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            batch[mode] = {"solves_s": round(64 / dt, 3), "t_batch_s": round(dt, 4),
                           "converged": sum(i["converged"] for i in infos),
                           "iters": [i["iters"] for i in infos],
                           "max_rel_res": max(i["rel_res_true"] for i in infos)}
            log(f"C4 {mode}: {batch[mode]}")
        result["batch_16x4"] = batch
        del solvers, bs, xs

        # adjoint: block k^2 field on 256 x 256, forward + backward through the autograd wrapper
        from oracle import adjoint as oadj
        from paper_1608_02461_amd.autograd import expand_blocks, helmholtz_solve
        c5 = workloads.adjoint_c5()
        n5 = c5["n"]
        s5 = hfmm.Solver(n5, c5["k0"], p=c5["p"], leaf_size=c5["leaf"], prec=hfmm.FP32)
        d5 = hfmm.Solver(n5, c5["k0"], p=c5["p"], leaf_size=c5["leaf"], prec=hfmm.FP32)
        f5 = torch.from_numpy(c5["f"]).to(dev)
        ud, _ = d5.solve(f5, restart=200, rtol=1e-10, strict=True)
        P5 = torch.from_numpy(c5["P"]).to(dev)
        dd = ud[P5]
        del d5

        def fwd_bwd(rtol):
            kbt = torch.from_numpy(c5["kb"]).to(dev).requires_grad_(True)
            u = helmholtz_solve(expand_blocks(kbt, n5), f5, s5, restart=200, rtol=rtol)
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
        Jo, Go, _, _ = oadj.gradient(n5, c5["kb"], c5["f"], c5["P"], dd.cpu().numpy())
        result["adjoint_256"] = {
            "fwd_bwd_s_rtol1e-10": round(t_fb, 4), "fwd_bwd_s_rtol1e-6": round(t_fb6, 4),
            "grad_rel_err_vs_oracle_rtol1e-10": float(np.linalg.norm(g5 - Go) / np.linalg.norm(Go)),
            "grad_rel_err_vs_oracle_rtol1e-6": float(np.linalg.norm(g6 - Go) / np.linalg.norm(Go)),
            "J_rel_err": abs(J5 - Jo) / abs(Jo)}
        log(f"C5: {result['adjoint_256']}")
        del s5

        c1 = workloads.solve_c1()
        s = hfmm.Solver(c1["n"], c1["k"], p=6, leaf_size=32, prec=hfmm.FP64)
        f1 = torch.from_numpy(c1["f"]).to(dev)
        s.solve(f1, restart=30)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            x, info = s.solve(f1, restart=30, rtol=1e-6)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        result["solve_64"] = {"solves_s": round(1 / dt, 3), "iters": info["iters"],
                              "rel_res_true": info["rel_res_true"]}
        log(f"C1: {result['solve_64']}")

    if not args.no_cpu:
        from concurrent.futures import ThreadPoolExecutor

        from threadpoolctl import threadpool_limits

        from oracle import kernel

        # one oracle call per thread on its own targets; numpy and scipy release
        # the GIL in the pairwise work, so the threads run in parallel
        nthr = max(1, min(16, len(os.sched_getaffinity(0))))
        n_t = 64 * nthr
        tg = w["xy"][smp[:n_t]] if n_t <= len(smp) else w["xy"][:n_t]
        with threadpool_limits(1):
            t0 = time.perf_counter()
            with ThreadPoolExecutor(nthr) as ex:
                list(ex.map(lambda i: kernel.direct_sum(w["xy"], w["q"], k, tgt=tg[i::nthr]), range(nthr)))
            dt = time.perf_counter() - t0
        # full N x N direct sum time by linearity in the number of targets
        full = dt / n_t * N
        result["cpu_baseline"] = {
            "value": round(N / full / 1e6, 6), "unit": "Mpts/s", "cores": nthr, "kind": "oracle",
            "sample": f"oracle direct N-body sum (scipy hankel1, FP64) from all {N} sources to {n_t} of the "
                      f"seeded targets ({dt:.1f} s on {nthr} threads, one oracle call per thread); Mpts/s of "
                      f"the full N x N sum by linearity",
            "pairs_per_s": round(n_t * N / dt, 1)}

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
