#!/usr/bin/env python3
"""Benchmark of the bivariate Matern log-likelihood hot path on one MI355X.

One step = one likelihood evaluation l(theta) of the dense FP64 workload
(N = 25,600 Morton-ordered jittered-grid locations, 51,200 x 51,200
covariance: tile generation, tiled Cholesky, log-determinant, triangular
solve) plus cokriging of 100 held-out locations on the resident factor.
Inputs are synthetic and resident in HBM before the timed region.

Prints one JSON line: evals/s, the Cholesky TFLOP/s, the roofline of the
dominant kernel (trailing-update GEMM/SYRK on FP64 MFMA) from HIP events on
the stream each launch runs on, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json

import numpy as np
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6


def measured_traffic(kernel: str, workload_tag: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (profiles/*_hbm_traffic.md), or None when no summary exists for
    this workload or the kernel source changed since the counters were taken."""
    import glob
    import hashlib
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_hbm_traffic.md")):
        for line in open(path):
            if not line.startswith("traffic_json:"):
                continue
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel") != kernel or rec.get("workload") != workload_tag:
                continue
            src = os.path.join(ROOT, rec["source"])
            if not os.path.exists(src):
                return None
            if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
                return None
            return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return None


def cpu_baseline(n_full, sample_n, theta, seed):
    """Oracle (as is) on the leading sample_n locations of the same workload,
    scaled to evals/s at n_full by the O(n^3) cost of the factorisation."""
    import numpy as np

    import oracle
    import synthetic
    x, y = synthetic.jittered_grid(n_full, seed)
    p = oracle.morton_order(x, y)
    x, y = x[p][:sample_n], y[p][:sample_n]
    z = synthetic.normal_eps(2 * sample_n, seed)
    t0 = time.perf_counter()
    oracle.loglik(x, y, z, theta)
    dt = time.perf_counter() - t0
    scale = (sample_n / n_full) ** 3
    return {"value": scale / dt, "unit": "evals/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "one oracle loglik at N=%d (first %d Morton-ordered locations of the "
                      "N=%d workload) took %.2f s; scaled by (%d/%d)^3" %
                      (sample_n, sample_n, n_full, dt, sample_n, n_full)}


FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0


def run_variants(mvg, xs, ys, z, th, args, ref_loglik, reps=2):
    """Mixed-precision evaluations of the same inputs beside the FP64 result:
    evals/s, relative delta loglik and delta log|Sigma| against FP64, the
    refinement sweeps, and the off-band GEMM rate on its own MFMA peak."""
    import torch
    out = {}
    ref = mvg.loglik(xs, ys, z, th, {"nb": args.nb})
    for name, prec, peak, band in (
            ("mixed_fp32", mvg.MVG_MIXED_FP32, FP32_MFMA_PEAK_TFLOPS, args.band),
            ("mixed_fp32_band%d" % args.wide_band, mvg.MVG_MIXED_FP32, FP32_MFMA_PEAK_TFLOPS,
             args.wide_band),
            ("mixed_bf16", mvg.MVG_MIXED_BF16, BF16_MFMA_PEAK_TFLOPS, args.band),
            ("mixed_fp32x", mvg.MVG_MIXED_FP32X, FP32_MFMA_PEAK_TFLOPS, args.band)):
        o = {"nb": args.nb, "precision": prec, "band_tiles": band}
        mvg.loglik(xs, ys, z, th, o)  # warm-up
        torch.cuda.synchronize()
        mvg.mvg_prof_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            res = mvg.loglik(xs, ys, z, th, o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        prof = {k: mvg.mvg_prof_read(k) for k in ("trailing", "lowp", "potrf", "ir", "gen")}
        mvg.mvg_prof_enable(False)
        ir = mvg.mvg_ir_stats(0)
        N = 2 * args.n
        lp = prof["lowp"]
        lp_tf = lp["flops"] / (lp["ms"] * 1e-3) / 1e12 if lp["ms"] > 0 else None
        potrf_ms = prof["potrf"]["ms"] / max(1, prof["potrf"]["launches"])
        out[name] = {
            "evals_per_s": 1.0 / dt,
            "status": int(res["status"][0]),
            "rel_dloglik_vs_fp64": abs(res["loglik"][0] - ref["loglik"][0]) / abs(ref["loglik"][0]),
            "dlogdet_vs_fp64": float(res["logdet"][0] - ref["logdet"][0]),
            "rel_dquad_vs_fp64": abs(res["quad"][0] - ref["quad"][0]) / abs(ref["quad"][0]),
            "ir": ir,
            "band_tiles": band,
            "cholesky_tflops_equiv": (N ** 3 / 3.0) / (potrf_ms * 1e-3) / 1e12,
            "phases_ms_per_eval": {k: prof[k]["ms"] / reps for k in ("gen", "potrf", "ir")},
            "offband_gemm": {"achieved": lp_tf, "peak": peak, "unit": "TFLOP/s",
                             "frac": lp_tf / peak if lp_tf else None},
            "band_gemm_tflops": (prof["trailing"]["flops"] / (prof["trailing"]["ms"] * 1e-3) / 1e12
                                 if prof["trailing"]["ms"] > 0 else None),
        }
    # Diagonal Super Tile (tiles far from the diagonal annihilated), at the
    # workload's range and at weak dependence (a = 0.03) on the same data
    th_weak = (th[0], th[1], 0.03) + tuple(th[3:])
    ref_weak = mvg.loglik(xs, ys, z, th_weak, {"nb": args.nb})
    for tag, t, r in (("", th, ref), ("_a0.03", th_weak, ref_weak)):
        for name, keep in (("dst_40_60", 0.4), ("dst_70_30", 0.7)):
            w = mvg.mvg_dst_band(args.n, args.nb, keep)
            o = {"nb": args.nb, "precision": mvg.MVG_DST, "band_tiles": w}
            mvg.loglik(xs, ys, z, t, o)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                res = mvg.loglik(xs, ys, z, t, o)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            ok = int(res["status"][0]) == 0
            out[name + tag] = {
                "evals_per_s": 1.0 / dt, "status": int(res["status"][0]), "band_tiles": w,
                "a": t[2],
                "rel_dloglik_vs_fp64": (abs(res["loglik"][0] - r["loglik"][0]) /
                                        abs(r["loglik"][0]) if ok else None),
            }
    return out


def _step(msg):
    """Progress of a long workload (stderr; the JSON line stays alone on stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _line(metric, value, unit, steps, warmup, ms, dtype, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out), flush=True)


def run_tlr(args, mvg, dev, synthetic, torch):
    """TLR likelihood on the N = 100,000 workload (200,000 x 200,000, tile
    1200), beside one dense FP64 evaluation of the same inputs."""
    n, nb = args.n, 1200
    th = (1.0, 1.0, args.a, 0.5, 1.0, 0.5)
    xr, yr = synthetic.jittered_grid(n, args.seed)
    _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
    # Z = L eps at the true theta from the FP64 factor (setup; 160 GB resident)
    _step("tlr: Z = L eps from the FP64 factor, n=%d" % n)
    A = mvg.cov_generate(xs, ys, th, {"nb": 1024})
    if mvg.potrf_tiled(A):
        raise SystemExit("Sigma(theta) not positive definite")
    z = mvg.mvg_trmv(A, dev(synthetic.normal_eps(2 * n, args.seed)))
    del A
    ref = None
    dense = {}
    if not args.no_dense_ref:
        _step("tlr: dense FP64 reference evaluation")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ref = mvg.loglik(xs, ys, z, th, {"nb": 1024})
        torch.cuda.synchronize()
        dense = {"evals_per_s": 1.0 / (time.perf_counter() - t0), "loglik": float(ref["loglik"][0])}
    accs = [float(a) for a in args.accs.split(",")]
    res = {}
    for acc in accs:
        o = {"nb": nb, "precision": mvg.MVG_TLR, "tlr_acc": acc, "tlr_max_rank": 300}
        _step("tlr: acc %g, %d evaluation(s)" % (acc, max(1, args.steps)))
        mvg.mvg_prof_enable(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(max(1, args.steps)):
            r = mvg.loglik(xs, ys, z, th, o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / max(1, args.steps)
        pr = {k: mvg.mvg_prof_read(k) for k in ("gen", "potrf", "solve", "trailing")}
        mvg.mvg_prof_enable(False)
        rec = {"evals_per_s": 1.0 / dt, "s_per_eval": dt, "status": int(r["status"][0]),
               "loglik": float(r["loglik"][0]),
               "phases_ms_per_eval": {"compress": pr["gen"]["ms"] / max(1, args.steps),
                                      "factor": pr["potrf"]["ms"] / max(1, args.steps),
                                      "solve": pr["solve"]["ms"] / max(1, args.steps)},
               "update_gemm_tflops": (pr["trailing"]["flops"] / (pr["trailing"]["ms"] * 1e-3) / 1e12
                                      if pr["trailing"]["ms"] > 0 else None)}
        if ref is not None:
            rec["rel_dloglik_vs_fp64"] = abs(r["loglik"][0] - ref["loglik"][0]) / abs(ref["loglik"][0])
        res["acc%g" % acc] = rec
    simplex = None
    if not args.no_simplex:  # the 7 points of a Nelder-Mead step in one call
        pts = synthetic.nelder_mead_simplex(th)
        _step("tlr: %d simplex points in one call" % len(pts))
        o = {"nb": nb, "precision": mvg.MVG_TLR, "tlr_acc": accs[0], "tlr_max_rank": 300}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r7 = mvg.loglik(xs, ys, z, pts, o)
        torch.cuda.synchronize()
        dt7 = time.perf_counter() - t0
        simplex = {"points": len(pts), "seconds": dt7, "evals_per_s": len(pts) / dt7,
                   "vs_one_at_a_time": (len(pts) / dt7) / res["acc%g" % accs[0]]["evals_per_s"],
                   "failed": int((r7["status"] != 0).sum())}
    _, ranks = mvg.tlr_compress(xs, ys, th, {"nb": nb, "tlr_acc": accs[0], "tlr_max_rank": 300})
    T = ranks.shape[0]
    low = ranks[np.tril_indices(T, -1)]
    head = res["acc%g" % accs[0]]
    _line("loglik evals/s + Cholesky TFLOP/s (FP64 vs mixed/TLR at |dl|<=1e-6); p99 latency",
          head["evals_per_s"], "evals/s", max(1, args.steps), 0, 1e3 * head["s_per_eval"], "f64",
          {"workload": "TLR bivariate Matern loglik, N=%d locations (%dx%d), tile %d, acc %s, "
                       "max rank 300, theta=(1,1,%g,0.5,1,0.5)" % (n, 2 * n, 2 * n, nb, args.accs,
                                                                   args.a),
           "n_loc": n, "nb": nb, "precision": "tlr"},
          tlr=res, dense_fp64=dense, simplex7=simplex,
          ranks={"acc": accs[0], "median_offset1": int(np.median(np.diag(ranks, -1))),
                 "median_all": int(np.median(low[low >= 0])) if (low >= 0).any() else None,
                 "dense_tiles": int((low < 0).sum()), "tiles": int(low.size)})


def run_batched(args, mvg, dev, synthetic, torch):
    """Many theta on the N = 400 workload (800 x 800) in one persistent launch."""
    n = 400
    th0 = synthetic.THETA_CFG0
    xr, yr = synthetic.jittered_grid(n, args.seed)
    _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
    A = mvg.cov_generate(xs, ys, th0, {"nb": 128})   # Z = L eps at the true theta (setup)
    if mvg.potrf_tiled(A):
        raise SystemExit("Sigma(theta) not positive definite")
    z = mvg.mvg_trmv(A, dev(synthetic.normal_eps(2 * n, args.seed)))
    del A
    ths = synthetic.jittered_thetas(args.batch, args.seed + 1)
    warm = max(1, args.warmup)   # the full batch: its workspace is sized then
    for _ in range(warm):
        mvg.loglik(xs, ys, z, ths, {"nb": 128})
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = mvg.loglik(xs, ys, z, ths, {"nb": 128})
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    # the same evaluations one call at a time (tiled path), on a subset
    k = min(32, args.batch)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for t in ths[:k]:
        mvg.loglik(xs, ys, z, t, {"nb": 128})
    torch.cuda.synchronize()
    single = k / (time.perf_counter() - t1)
    simplex = synthetic.nelder_mead_simplex(th0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    mvg.loglik(xs, ys, z, simplex, {"nb": 128})
    torch.cuda.synchronize()
    _line("loglik evals/s + Cholesky TFLOP/s (FP64 vs mixed/TLR at |dl|<=1e-6); p99 latency",
          args.batch / dt, "evals/s", args.steps, warm, 1e3 * dt, "f64",
          {"workload": "batched FP64 loglik, %d theta (+-20%% around (1,1,0.1,0.5,1,0.5)) on "
                       "N=%d locations (%dx%d), one persistent launch" % (args.batch, n, 2 * n, 2 * n),
           "n_loc": n, "batch": args.batch, "precision": "fp64"},
          single_call_evals_per_s=single, speedup_vs_single_calls=(args.batch / dt) / single,
          simplex7_ms=1e3 * (time.perf_counter() - t2), failed=int((r["status"] != 0).sum()))


def run_mloe(args, mvg, dev, synthetic, torch):
    """Prediction efficiency (Section 5.4, Algorithm 1) of an approximate
    model's theta_a against the true theta on the N = 25,600 workload with
    100 targets: two covariance generations, two FP64 Cholesky
    factorisations, the multi-right-hand-side solves and the traces."""
    n, m = args.n, args.targets
    th = (1.0, 1.0, args.a, 0.5, 1.0, 0.5)
    tha = (0.97, 1.04, 1.08 * args.a, 0.52, 0.96, 0.47)
    xr, yr = synthetic.jittered_grid(n, args.seed)
    _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
    x0r, y0r = synthetic.uniform_targets(m, args.seed)
    x0, y0 = dev(x0r), dev(y0r)
    o = {"nb": args.nb}
    for _ in range(args.warmup):
        mvg.mloe_mmom(xs, ys, th, tha, x0, y0, o)
    torch.cuda.synchronize()
    mvg.mvg_prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = mvg.mloe_mmom(xs, ys, th, tha, x0, y0, o)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    mvg.mvg_prof_enable(False)
    gen, fac, sol = (mvg.mvg_prof_read(k) for k in ("gen", "potrf", "solve"))
    per = lambda p: p["ms"] / args.steps   # noqa: E731
    _line("loglik evals/s + Cholesky TFLOP/s (FP64 vs mixed/TLR at |dl|<=1e-6); p99 latency",
          1.0 / dt, "MLOE/MMOM evals/s", args.steps, args.warmup, 1e3 * dt, "f64",
          {"workload": "multivariate MLOE/MMOM, N=%d locations (%dx%d), %d targets, nb %d, "
                       "theta_a = theta perturbed by 3-8%%" % (n, 2 * n, 2 * n, m, args.nb),
           "n_loc": n, "targets": m, "precision": "fp64"},
          mloe=r["mloe"], mmom=r["mmom"], status=r["status"],
          gen_ms=per(gen), fact_ms=per(fac), comp_ms=per(sol),
          fact_tflops=fac["flops"] / (fac["ms"] * 1e9) if fac["ms"] else None,
          comp_tflops=sol["flops"] / (sol["ms"] * 1e9) if sol["ms"] else None)


def run_trivariate(args, mvg, dev, synthetic, torch):
    """The p = 3 model (the trivariate application's form, Section 6.4.2) at
    the dense workload's matrix order: n = 17,066 locations, 51,198 x 51,198,
    Eq. (1) and the profile likelihood of Section 5.2 (three univariate
    17,066 x 17,066 factorisations, then Eq. (1))."""
    n = args.n
    th = {"sigma_sq": [1.0, 1.0, 1.0], "a": args.a, "nu": [0.5, 1.0, 1.5],
          "beta": [[1.0, 0.5, -0.3], [0.5, 1.0, -0.2], [-0.3, -0.2, 1.0]]}
    xr, yr = synthetic.jittered_grid(n, args.seed)
    _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
    o = {"nb": args.nb}
    A = mvg.cov_generate_p(xs, ys, th, o)       # Z = L eps at the true theta (setup)
    if mvg.potrf_tiled(A):
        raise SystemExit("trivariate Sigma(theta) not positive definite")
    z = mvg.mvg_trmv(A, dev(synthetic.normal_eps(3 * n, args.seed)))
    del A
    for _ in range(args.warmup):
        mvg.loglik_p(xs, ys, z, th, o)
    torch.cuda.synchronize()
    mvg.mvg_prof_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = mvg.loglik_p(xs, ys, z, th, o)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    prof = {k: mvg.mvg_prof_read(k) for k in ("gen", "potrf")}
    mvg.mvg_prof_enable(False)
    N = 3 * n
    potrf_ms = prof["potrf"]["ms"] / max(1, prof["potrf"]["launches"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof_ll = mvg.profile_loglik_p(xs, ys, z, th, o)
    torch.cuda.synchronize()
    _line("loglik evals/s + Cholesky TFLOP/s (FP64 vs mixed/TLR at |dl|<=1e-6); p99 latency",
          1.0 / dt, "evals/s", args.steps, args.warmup, 1e3 * dt, "f64",
          {"workload": "trivariate parsimonious Matern loglik, N=%d locations (%dx%d), nb %d"
                       % (n, N, N, args.nb), "n_loc": n, "p": 3, "precision": "fp64"},
          loglik=float(r["loglik"][0]), status=int(r["status"][0]),
          cholesky_tflops=(N ** 3 / 3.0) / (potrf_ms * 1e-3) / 1e12,
          gen_ms=prof["gen"]["ms"] / max(1, prof["gen"]["launches"]),
          profile_loglik={"seconds": time.perf_counter() - t1, "loglik": prof_ll["loglik"],
                          "sigma_sq": [float(v) for v in prof_ll["sigma_sq"]]})


def run_mle(args, mvg, dev, synthetic, torch):
    """Maximum likelihood at the shape of the synthetic estimation study
    (Section 6.4.1, Experiment 2: 22,464 sampled locations, a = 0.09, nu11 =
    0.5, nu22 = 1): Nelder-Mead from a perturbed start, a bounded number of
    exact FP64 evaluations (one fit needs a few hundred)."""
    n = args.n
    th = (1.0, 1.0, 0.09, 0.5, 1.0, 0.5)
    start = (1.2, 0.8, 0.12, 0.6, 0.9, 0.3)
    xr, yr = synthetic.jittered_grid(n, args.seed)
    _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
    A = mvg.cov_generate(xs, ys, th, {"nb": args.nb})
    if mvg.potrf_tiled(A):
        raise SystemExit("Sigma(theta) not positive definite")
    z = mvg.mvg_trmv(A, dev(synthetic.normal_eps(2 * n, args.seed)))
    del A
    o = {"nb": args.nb}
    l_true = float(mvg.loglik(xs, ys, z, th, o)["loglik"][0])
    l_start = float(mvg.loglik(xs, ys, z, start, o)["loglik"][0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fit = mvg.mle_fit(xs, ys, z, start, o, max_evals=args.max_evals)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _line("loglik evals/s + Cholesky TFLOP/s (FP64 vs mixed/TLR at |dl|<=1e-6); p99 latency",
          fit["evals"] / dt, "evals/s", fit["evals"], 0, 1e3 * dt / fit["evals"], "f64",
          {"workload": "Nelder-Mead MLE, N=%d locations (%dx%d), nb %d, FP64, %d evaluations"
                       % (n, 2 * n, 2 * n, args.nb, args.max_evals), "n_loc": n,
           "precision": "fp64"},
          fit_seconds=dt, theta_start=start, theta_true=th, theta_hat=fit["theta"],
          loglik_start=l_start, loglik_true=l_true, loglik_hat=fit["loglik"],
          converged=fit["converged"], iterations=fit["iters"])


def serve_stream(args, mvg, dev, synthetic, torch, rate, nreq):
    """One Poisson stream through a fresh server; returns its summary."""
    import threading
    reqs, sizes = synthetic.serving_stream(nreq, args.seed, rate_hz=rate)
    data = []
    for d, n in enumerate(sizes):
        x, y = synthetic.jittered_grid(int(n), args.seed + 100 + d)
        _, xs, ys = mvg.morton_order(dev(x), dev(y), sorted_xy=True)
        data.append((xs, ys, dev(synthetic.normal_eps(2 * int(n), args.seed + 100 + d))))
    x0r, y0r = synthetic.uniform_targets(100, args.seed)
    x0, y0 = dev(x0r), dev(y0r)
    S = mvg.Server(int(args.budget_gb * (1 << 30)), args.workers, {"nb": 512})
    ids = [S.add_dataset(*t) for t in data]
    torch.cuda.synchronize()
    last = None
    plan = []
    for q in reqs:   # a cokriging request refers to the latest likelihood's (dataset, theta)
        if q.kind == "cokrige" and last is not None:
            plan.append((mvg.REQ_COKRIGE, last[0], last[1], q.arrival_s))
        else:
            plan.append((mvg.REQ_LOGLIK, q.dataset, q.theta, q.arrival_s))
            last = (q.dataset, q.theta)
    zh = [torch.empty(200, dtype=torch.float64, device="cuda") for _ in plan]
    t_base = S.clock()

    def feeder():
        for i, (kind, d, th, ta) in enumerate(plan):
            wait = t_base + ta - S.clock()
            if wait > 0:
                time.sleep(wait)
            if kind == mvg.REQ_COKRIGE:
                S.submit(kind, ids[d], th, x0, y0, zh[i], t_arrive=t_base + ta)
            else:
                S.submit(kind, ids[d], th, t_arrive=t_base + ta)

    th_feed = threading.Thread(target=feeder)
    th_feed.start()
    done = []
    while len(done) < len(plan):
        done += S.poll(256, 200)
    th_feed.join()
    stats = S.stats()
    S.close()
    lat = np.array([r.t_end - r.t_arrive for r in done])
    span = max(r.t_end for r in done) - t_base
    ok = [r for r in done if r.status == 0]
    return {"achieved_rate": len(ok) / span, "offered_rate": len(plan) / (plan[-1][3] or 1.0),
            "requests": len(plan), "makespan_s": span,
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "rejected": int(sum(1 for r in done if r.status < 0)),
            "failed": int(sum(1 for r in done if r.status > 0)), "cache": stats,
            "mean_batch": float(np.mean([r.batch for r in done])), "datasets": len(sizes)}


def run_serving(args, mvg, dev, synthetic, torch):
    """The 50 req/s stream (above the FP64 capacity: the queue grows) and a
    stream below capacity (bounded latency), same request mix."""
    hot = serve_stream(args, mvg, dev, synthetic, torch, args.rate, args.requests)
    calm = serve_stream(args, mvg, dev, synthetic, torch, args.sustain_rate, args.requests)
    _line("loglik evals/s + Cholesky TFLOP/s (FP64 vs mixed/TLR at |dl|<=1e-6); p99 latency",
          hot["achieved_rate"], "requests/s", hot["requests"], 0,
          1e3 * hot["makespan_s"] / hot["requests"], "f64",
          {"workload": "serving: %d requests, Poisson %.0f req/s, %d datasets n~U[1000,20000], "
                       "10%% cokriging (100 targets) on the latest likelihood's factor, theta +-20%%"
                       % (hot["requests"], args.rate, hot["datasets"]),
           "requests": hot["requests"], "rate_hz": args.rate, "workers": args.workers,
           "budget_gb": args.budget_gb, "precision": "fp64"},
          offered_rate=hot["offered_rate"], p50_latency_s=hot["p50_latency_s"],
          p99_latency_s=hot["p99_latency_s"], rejected=hot["rejected"], failed=hot["failed"],
          cache=hot["cache"], mean_batch=hot["mean_batch"],
          below_capacity={"rate_hz": args.sustain_rate, **calm})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None,
                    help="locations (default 25,600; 100,000 for --workload tlr)")
    ap.add_argument("--a", type=float, default=0.1)
    ap.add_argument("--nb", type=int, default=0,
                    help="tile size (0: dense workload autotunes among 256/512/768/1024; "
                         "mloe / trivariate / mle use 1024)")
    ap.add_argument("--targets", type=int, default=100)
    ap.add_argument("--cpu-sample-n", type=int, default=2400)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the mixed-precision evaluations of the same inputs")
    ap.add_argument("--band", type=int, default=2, help="FP64 band width in tiles (mixed)")
    ap.add_argument("--wide-band", type=int, default=16,
                    help="second, wider FP64 band for the FP32 variant")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="dense", choices=["dense", "tlr", "batched", "serving", "mloe", "trivariate", "mle"],
                    help="dense: N=25,600 FP64 (+ mixed variants); tlr: N=100,000 TLR; batched: "
                         "many theta at N=400 in one launch; serving: request stream; mloe: "
                         "MLOE/MMOM at N=25,600 with 100 targets; trivariate: p = 3 at N=17,066; mle: Nelder-Mead at N=22,464")
    ap.add_argument("--accs", default="1e-7", help="TLR accuracies (first one is the value)")
    ap.add_argument("--no-dense-ref", action="store_true")
    ap.add_argument("--no-simplex", action="store_true",
                    help="TLR: skip the 7-point simplex evaluated in one call")
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--max-evals", type=int, default=40, help="MLE: likelihood evaluations")
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--sustain-rate", type=float, default=6.0)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--budget-gb", type=float, default=200.0)
    ap.add_argument("--copy-calibration", type=float, default=0.0,
                    help="only run a plain device copy of this many GiB (to scale HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2008_07437_amd as mvg
    import synthetic

    torch.cuda.set_device(0)
    if args.copy_calibration > 0:
        nbytes = int(args.copy_calibration * (1 << 30))
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes}), flush=True)
        return
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()  # noqa
    tune_nb = args.workload == "dense" and args.nb == 0
    args.nb = args.nb or 1024   # the size the autotuner picks at n = 25,600
    if args.workload == "tlr":
        args.n = args.n or 100000
        return run_tlr(args, mvg, dev, synthetic, torch)
    args.n = args.n or 25600
    if args.workload == "batched":
        return run_batched(args, mvg, dev, synthetic, torch)
    if args.workload == "serving":
        return run_serving(args, mvg, dev, synthetic, torch)
    if args.workload == "mloe":
        return run_mloe(args, mvg, dev, synthetic, torch)
    if args.workload == "mle":
        args.n = 22464 if args.n == 25600 else args.n
        return run_mle(args, mvg, dev, synthetic, torch)
    if args.workload == "trivariate":
        args.n = 17066 if args.n == 25600 else args.n
        return run_trivariate(args, mvg, dev, synthetic, torch)
    th = (1.0, 1.0, args.a, 0.5, 1.0, 0.5)
    n = args.n
    # --- data: Morton-ordered locations, Z = L eps at the true theta (setup)
    xr, yr = synthetic.jittered_grid(n, args.seed)
    _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
    _step("dense: Z = L eps, n=%d" % n)
    A = mvg.cov_generate(xs, ys, th, {"nb": args.nb})
    info = mvg.potrf_tiled(A)
    if info:
        raise SystemExit("Sigma(theta) not positive definite at pivot %d" % info)
    z = mvg.mvg_trmv(A, dev(synthetic.normal_eps(2 * n, args.seed)))
    del A
    tuned = None
    if tune_nb:  # the library's autotuner picks the tile size on this problem (setup)
        _step("dense: autotuning the tile size")
        args.nb, tuned = mvg.mvg_autotune_nb(xs, ys, z, th, {}, [256, 512, 768, 1024])
    x0r, y0r = synthetic.uniform_targets(args.targets, args.seed)
    x0, y0 = dev(x0r), dev(y0r)
    opts = {"nb": args.nb}
    torch.cuda.synchronize()

    last = {}

    def step():
        res, F = mvg.loglik(xs, ys, z, th, opts, keep=True)
        zhat = mvg.cokrige_predict(F, x0, y0)
        last["loglik"] = float(res["loglik"][0])
        last["zhat0"] = zhat[0].tolist()
        del F

    _step("dense: nb %d, %d warm-up + %d timed steps" % (args.nb, args.warmup, args.steps))
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    mvg.mvg_prof_enable(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = {k: mvg.mvg_prof_read(k) for k in ("trailing", "gen", "potrf", "solve", "cokrige")}
    mvg.mvg_prof_enable(False)
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    N = 2 * n
    chol_flops = N ** 3 / 3.0
    potrf_ms = prof["potrf"]["ms"] / max(1, prof["potrf"]["launches"])
    tr = prof["trailing"]
    achieved = tr["flops"] / (tr["ms"] * 1e-3) / 1e12 if tr["ms"] > 0 else None
    out = {
        "metric": "loglik evals/s + Cholesky TFLOP/s (FP64 vs mixed/TLR at |dl|<=1e-6); p99 latency",
        "value": args.steps / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dense FP64 bivariate Matern loglik + cokriging, N=%d locations "
                               "(%dx%d covariance), theta=(1,1,%g,0.5,1,0.5), nb=%d, %d targets"
                               % (n, N, N, args.a, args.nb, args.targets),
                   "n_loc": n, "matrix": N, "nb": args.nb, "precision": "fp64",
                   "parallelism": "single GPU"},
        "cholesky_tflops": chol_flops / (potrf_ms * 1e-3) / 1e12,
        "phases_ms_per_step": {k: prof[k]["ms"] / max(1, args.steps)
                               for k in ("gen", "potrf", "solve", "cokrige")},
        "loglik": last["loglik"],
        "autotune_seconds_per_eval": ({str(k): v for k, v in tuned.items()} if tuned else None),
        "roofline": {"kernel": "k_update_trailing", "bound": "mfma",
                     "achieved": achieved, "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": (achieved / FP64_MFMA_PEAK_TFLOPS) if achieved else None,
                     "traffic": measured_traffic("k_update_trailing<%d, 0>" % args.nb,
                                                 "cfg1_n%d_nb%d" % (n, args.nb)),
                     "launches": tr["launches"],
                     "avg_launch_ms": tr["ms"] / max(1, tr["launches"]),
                     "flops_per_launch": tr["flops"] / max(1, tr["launches"])},
    }
    if not args.no_variants:
        _step("dense: mixed-precision and DST variants")
        out["variants"] = run_variants(mvg, xs, ys, z, th, args, last["loglik"])
    if not args.no_cpu:
        _step("dense: oracle timing on the host (bounded sample)")
        out["cpu_baseline"] = cpu_baseline(n, args.cpu_sample_n, th, args.seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
