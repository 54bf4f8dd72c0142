#!/usr/bin/env python3
"""Benchmark of the bivariate Matern log-likelihood hot path on one MI355X.

Default line (the largest single-GPU workload): one step = one tile-low-rank
likelihood evaluation l(theta) at N = 100,000 Morton-ordered jittered-grid
locations (200,000 x 200,000 covariance, tile 1200, accuracy 1e-7, maximum
rank 300): tile generation, compression, TLR Cholesky, log-determinant and
solve.  Inputs (locations, Z = L eps drawn with the dense FP64 factor in the
set-up) are resident in HBM before the timed region.  The same line carries
the dense FP64 evaluation of the same inputs and the relative delta loglik,
the ranks and the compressed-to-dense memory ratio, the roofline of the
dominant kernel (HIP events on the stream each launch runs on), the dense
FP64 workload (N = 25,600, tile size autotuned, cokriging of 100 targets) and
the mixed-precision workload (N = 50,000, FP32 / FP32X against FP64) as
nested records, and the CPU oracle timed on a bounded sample.  Other
workloads: --workload dense | tlr | mixed | batched | serving | mloe |
trivariate | mle.
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
    """The oracle (as is: plain C, OpenMP, FP64 Crout Cholesky) on the leading
    sample_n locations of the same workload, timed on this host, scaled to
    evals/s at n_full by the (2n)^3 / 3 cost of the factorisation that
    dominates it.  The full-size oracle evaluation at n = 25,600 stored with
    the golden values (timed once on the build host) is reported beside it
    to show how well the cubic scaling holds there."""
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
    out = {"value": scale / dt, "unit": "evals/s", "cores": oracle.num_threads(),
           "kind": "oracle",
           "sample": "one oracle loglik at N=%d (the first %d Morton-ordered locations of the "
                     "N=%d workload) took %.2f s on %d host threads; scaled by (%d/%d)^3"
                     % (sample_n, sample_n, n_full, dt, oracle.num_threads(), sample_n, n_full)}
    gpath = os.path.join(ROOT, "tests", "golden", "dense_n25600.json")
    if os.path.exists(gpath):
        g = json.load(open(gpath))
        for key, case in sorted(g.get("cases", {}).items()):
            out["full_size_reference"] = {
                "n_loc": g["n_loc"], "seconds": case["oracle_seconds"],
                "threads": case["oracle_threads"], "host": g["host"]["cpu"],
                "extrapolated_from_this_sample_s": dt * (g["n_loc"] / sample_n) ** 3,
                "note": "one full oracle evaluation at n = %d (%s) on the build host" %
                        (g["n_loc"], key)}
            break
    return out


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
            ("mixed_fp32x", mvg.MVG_MIXED_FP32X, FP32_MFMA_PEAK_TFLOPS, args.band),
            # three BF16 MFMAs per product: its useful-flop ceiling is a third of BF16's
            ("mixed_bf16x3", mvg.MVG_MIXED_BF16X3, BF16_MFMA_PEAK_TFLOPS / 3.0, args.band)):
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


def _plain(o):
    """numpy scalars and arrays as JSON values."""
    if isinstance(o, np.generic):
        return o.item()
    if isinstance(o, np.ndarray):
        return o.tolist()
    raise TypeError(type(o).__name__)


def _line(metric, value, unit, steps, warmup, ms, dtype, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}
    out.update(extra)
    print(json.dumps(out, default=_plain), flush=True)


def _prof(mvg, kinds):
    return {k: mvg.mvg_prof_read(k) for k in kinds}


def tlr_memory(ranks, nb, N):
    """Compressed storage of the TLR Sigma (dense diagonal tiles, U and V per
    off-diagonal tile, dense fall-back tiles nb^2) against the dense matrix."""
    T = ranks.shape[0]
    low = ranks[np.tril_indices(T, -1)]
    comp = T * nb * nb + sum(nb * nb if k < 0 else 2 * nb * int(k) for k in low)
    return {"compressed_gb": 8.0 * comp / 1e9, "dense_full_gb": 8.0 * N * N / 1e9,
            "dense_lower_tiles_gb": 8.0 * T * (T + 1) / 2 * nb * nb / 1e9,
            "ratio_full_over_tlr": float(N) * N / comp,
            "ratio_lower_tiles_over_tlr": T * (T + 1) / 2 * nb * nb / comp}


def tlr_record(args, mvg, dev, synthetic, torch, n, acc, steps, warmup, simplex=False):
    """TLR likelihood on the N = n workload (2n x 2n, tile 1200, maximum rank
    300): warm-up and timed evaluations, beside the dense FP64 evaluation of
    the same inputs (the set-up factor: generation + Cholesky timed, then the
    solve and log-determinant on that factor)."""
    nb = 1200
    th = (1.0, 1.0, args.a, 0.5, 1.0, 0.5)
    xr, yr = synthetic.jittered_grid(n, args.seed)
    _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
    if args.white_z:  # counter runs: Z = eps, no dense factor (kernel work does not depend on Z)
        z = dev(synthetic.normal_eps(2 * n, args.seed))
        ref = {"loglik": float("nan"), "logdet": float("nan"), "quad": float("nan")}
        dense = None
    else:
        # Z = L eps at the true theta from the FP64 factor (set-up; 160 GB
        # resident), and the dense FP64 likelihood of the same inputs from it
        _step("tlr: dense FP64 factor, Z = L eps, n=%d" % n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A = mvg.cov_generate(xs, ys, th, {"nb": 1024})
        if mvg.potrf_tiled(A):
            raise SystemExit("Sigma(theta) not positive definite")
        torch.cuda.synchronize()
        t_fact = time.perf_counter() - t0
        z = mvg.mvg_trmv(A, dev(synthetic.normal_eps(2 * n, args.seed)))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ref = mvg.mvg_mat_loglik(A, z)
        torch.cuda.synchronize()
        t_solve = time.perf_counter() - t1
        del A
        dense = {"seconds": t_fact + t_solve, "evals_per_s": 1.0 / (t_fact + t_solve), "nb": 1024,
                 "loglik": ref["loglik"], "logdet": ref["logdet"], "quad": ref["quad"],
                 "cholesky_tflops": (2.0 * n) ** 3 / 3.0 / t_fact / 1e12}
    o = {"nb": nb, "precision": mvg.MVG_TLR, "tlr_acc": acc, "tlr_max_rank": 300}
    _step("tlr: acc %g, %d warm-up + %d timed evaluations" % (acc, warmup, steps))
    for _ in range(warmup):
        mvg.loglik(xs, ys, z, th, o)
    torch.cuda.synchronize()
    mvg.mvg_prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r = mvg.loglik(xs, ys, z, th, o)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    pr = _prof(mvg, ("gen", "potrf", "solve", "trailing", "tlr_gemm", "qr"))
    mvg.mvg_prof_enable(False)
    per = lambda k: pr[k]["ms"] / steps   # noqa: E731
    rec = {"evals_per_s": 1.0 / dt, "s_per_eval": dt, "status": int(r["status"][0]),
           "loglik": float(r["loglik"][0]), "logdet": float(r["logdet"][0]),
           "quad": float(r["quad"][0]),
           "rel_dloglik_vs_fp64": abs(r["loglik"][0] - ref["loglik"]) / abs(ref["loglik"]),
           "rel_dlogdet_vs_fp64": abs(r["logdet"][0] - ref["logdet"]) / abs(ref["logdet"]),
           "rel_dquad_vs_fp64": abs(r["quad"][0] - ref["quad"]) / abs(ref["quad"]),
           "speedup_vs_dense_fp64": dense["seconds"] / dt if dense else None,
           "phases_ms_per_eval": {"compress": per("gen"), "factor": per("potrf"),
                                  "solve": per("solve"), "update_gemm": per("trailing"),
                                  "all_batched_gemm": per("tlr_gemm"), "qr": per("qr")},
           "update_gemm_tflops": (pr["trailing"]["flops"] / (pr["trailing"]["ms"] * 1e-3) / 1e12
                                  if pr["trailing"]["ms"] > 0 else None)}
    # dominant kernel: the column-update GEMM of the factorisation (one
    # k_gemm_nt_sub_lds launch per tile column, algorithmic 2 M N K flops with
    # K the summed ranks, not the zero-padded K); the other batched GEMMs and
    # the QR launch groups are reported beside it
    g, q, b = pr["trailing"], pr["qr"], pr["tlr_gemm"]
    ach = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else None
    roof = {"kernel": "k_gemm_nt_sub_lds", "bound": "mfma", "achieved": ach,
            "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP64_MFMA_PEAK_TFLOPS if ach else None,
            "traffic": measured_traffic("k_gemm_nt_sub_lds", "tlr_n%d_nb%d" % (n, nb)),
            "launches": g["launches"], "avg_launch_ms": g["ms"] / max(1, g["launches"]),
            "flops_per_launch": g["flops"] / max(1, g["launches"]),
            "share_of_eval": g["ms"] / steps / (1e3 * dt),
            "batched_gemm_share_of_eval": b["ms"] / steps / (1e3 * dt),
            "batched_gemm_tflops": b["flops"] / (b["ms"] * 1e-3) / 1e12 if b["ms"] > 0 else None,
            "qr_groups_share_of_eval": q["ms"] / steps / (1e3 * dt)}
    _, ranks = mvg.tlr_compress(xs, ys, th, {"nb": nb, "tlr_acc": acc, "tlr_max_rank": 300})
    T = ranks.shape[0]
    low = ranks[np.tril_indices(T, -1)]
    rk = {"acc": acc, "median_offset1": int(np.median(np.diag(ranks, -1))),
          "median_all": int(np.median(low[low >= 0])) if (low >= 0).any() else None,
          "max": int(low.max()), "dense_tiles": int((low < 0).sum()), "tiles": int(low.size)}
    out = {"n_loc": n, "nb": nb, "acc": acc, "tlr": rec, "dense_fp64": dense, "ranks": rk,
           "memory": tlr_memory(ranks, nb, 2 * n), "roofline": roof}
    if simplex:  # the 7 points of a Nelder-Mead step in one call
        pts = synthetic.nelder_mead_simplex(th)
        _step("tlr: %d simplex points in one call" % len(pts))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r7 = mvg.loglik(xs, ys, z, pts, o)
        torch.cuda.synchronize()
        dt7 = time.perf_counter() - t0
        out["simplex7"] = {"points": len(pts), "seconds": dt7, "evals_per_s": len(pts) / dt7,
                           "vs_one_at_a_time": (len(pts) / dt7) * dt,
                           "failed": int((r7["status"] != 0).sum())}
    return out


METRIC = "loglik evals/s + Cholesky TFLOP/s (FP64 vs mixed/TLR at |dl|<=1e-6); p99 latency"


def run_tlr(args, mvg, dev, synthetic, torch):
    """TLR alone (any n / accuracy), with the simplex in one call."""
    acc = float(args.accs.split(",")[0])
    rec = tlr_record(args, mvg, dev, synthetic, torch, args.n, acc, max(1, args.steps),
                     args.warmup, simplex=not args.no_simplex)
    _line(METRIC, rec["tlr"]["evals_per_s"], "evals/s", max(1, args.steps), args.warmup,
          1e3 * rec["tlr"]["s_per_eval"], "f64",
          {"workload": "TLR bivariate Matern loglik, N=%d locations (%dx%d), tile 1200, acc %g, "
                       "max rank 300, theta=(1,1,%g,0.5,1,0.5)" % (args.n, 2 * args.n, 2 * args.n,
                                                                   acc, args.a),
           "n_loc": args.n, "nb": 1200, "precision": "tlr"},
          roofline=rec["roofline"], **{k: v for k, v in rec.items() if k != "roofline"})


def dense_record(args, mvg, dev, synthetic, torch, n, steps, warmup, tune_set):
    """Dense FP64 likelihood + cokriging of args.targets locations on the
    N = n workload; tile size by the library's autotuner over tune_set."""
    th = (1.0, 1.0, args.a, 0.5, 1.0, 0.5)
    xr, yr = synthetic.jittered_grid(n, args.seed)
    _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
    _step("dense: Z = L eps, n=%d" % n)
    A = mvg.cov_generate(xs, ys, th, {"nb": 1024})
    info = mvg.potrf_tiled(A)
    if info:
        raise SystemExit("Sigma(theta) not positive definite at pivot %d" % info)
    z = mvg.mvg_trmv(A, dev(synthetic.normal_eps(2 * n, args.seed)))
    del A
    tuned = None
    nb = args.nb
    if not nb:  # the library's autotuner picks the tile size on this problem (set-up)
        _step("dense: autotuning the tile size over %s" % (tune_set,))
        nb, tuned = mvg.mvg_autotune_nb(xs, ys, z, th, {}, list(tune_set))
    x0r, y0r = synthetic.uniform_targets(args.targets, args.seed)
    x0, y0 = dev(x0r), dev(y0r)
    opts = {"nb": nb}
    last = {}

    def step():
        res, F = mvg.loglik(xs, ys, z, th, opts, keep=True)
        mvg.cokrige_predict(F, x0, y0)
        last["loglik"] = float(res["loglik"][0])
        del F

    _step("dense: nb %d, %d warm-up + %d timed steps" % (nb, warmup, steps))
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    mvg.mvg_prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = _prof(mvg, ("trailing", "gen", "potrf", "solve", "cokrige"))
    mvg.mvg_prof_enable(False)
    N = 2 * n
    potrf_ms = prof["potrf"]["ms"] / max(1, prof["potrf"]["launches"])
    tr = prof["trailing"]
    achieved = tr["flops"] / (tr["ms"] * 1e-3) / 1e12 if tr["ms"] > 0 else None
    return {"workload": "dense FP64 bivariate Matern loglik + cokriging, N=%d locations (%dx%d), "
                        "theta=(1,1,%g,0.5,1,0.5), nb=%d, %d targets"
                        % (n, N, N, args.a, nb, args.targets),
            "n_loc": n, "nb": nb, "steps": steps, "warmup": warmup,
            "evals_per_s": steps / wall, "ms_per_step": 1e3 * wall / steps,
            "cholesky_tflops": N ** 3 / 3.0 / (potrf_ms * 1e-3) / 1e12,
            "phases_ms_per_step": {k: prof[k]["ms"] / max(1, steps)
                                   for k in ("gen", "potrf", "solve", "cokrige")},
            "loglik": last["loglik"],
            "autotune_seconds_per_eval": ({str(k): v for k, v in tuned.items()} if tuned else None),
            "roofline": {"kernel": "k_update_trailing", "bound": "mfma", "achieved": achieved,
                         "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": (achieved / FP64_MFMA_PEAK_TFLOPS) if achieved else None,
                         "traffic": measured_traffic("k_update_trailing<%d, 0>" % nb,
                                                     "dense_n%d_nb%d" % (n, nb)),
                         "launches": tr["launches"],
                         "avg_launch_ms": tr["ms"] / max(1, tr["launches"]),
                         "flops_per_launch": tr["flops"] / max(1, tr["launches"])}}, (xs, ys, z, th)


def mixed_record(args, mvg, dev, synthetic, torch, n, nu, beta, reps=1):
    """Mixed precision on the N = n workload (theta = (1, 1, 0.1, nu11, nu22,
    beta), Z = L eps): FP64 (set-up factor, then timed evaluations), FP32X and
    FP32 storage with a 2-tile FP64 band; evals/s, relative delta loglik and
    delta log|Sigma| against FP64 on the same inputs."""
    th = (1.0, 1.0, 0.1, nu[0], nu[1], beta)
    nb = 1024
    xr, yr = synthetic.jittered_grid(n, args.seed)
    _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
    _step("mixed: Z = L eps, n=%d, nu=%s, beta=%g" % (n, nu, beta))
    A = mvg.cov_generate(xs, ys, th, {"nb": nb})
    if mvg.potrf_tiled(A):
        raise SystemExit("Sigma(theta) not positive definite")
    z = mvg.mvg_trmv(A, dev(synthetic.normal_eps(2 * n, args.seed)))
    del A
    out = {"n_loc": n, "theta": th, "nb": nb, "band_tiles": 2}
    ref = None
    peaks = {"fp32x": FP32_MFMA_PEAK_TFLOPS, "fp32": FP32_MFMA_PEAK_TFLOPS,
             "bf16x3": BF16_MFMA_PEAK_TFLOPS / 3.0}   # three BF16 MFMAs per product
    for name, prec in (("fp64", mvg.MVG_FP64), ("fp32x", mvg.MVG_MIXED_FP32X),
                       ("bf16x3", mvg.MVG_MIXED_BF16X3), ("fp32", mvg.MVG_MIXED_FP32)):
        o = {"nb": nb, "precision": prec, "band_tiles": 2}
        mvg.loglik(xs, ys, z, th, o)   # warm-up (arena sizes)
        torch.cuda.synchronize()
        mvg.mvg_prof_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            r = mvg.loglik(xs, ys, z, th, o)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        pr = _prof(mvg, ("potrf", "lowp", "trailing"))
        mvg.mvg_prof_enable(False)
        rec = {"evals_per_s": 1.0 / dt, "status": int(r["status"][0]),
               "loglik": float(r["loglik"][0])}
        if prec == mvg.MVG_FP64:
            ref = r
        elif int(r["status"][0]) == 0:
            # a lost pivot or an unconverged refinement makes the library
            # evaluate theta in FP64
            rec["fp64_fallback"] = bool(mvg.mvg_ir_stats(0)["fp64_fallback"])
            rec["rel_dloglik_vs_fp64"] = abs(r["loglik"][0] - ref["loglik"][0]) / abs(ref["loglik"][0])
            rec["dlogdet_vs_fp64"] = float(r["logdet"][0] - ref["logdet"][0])
            rec["rel_dquad_vs_fp64"] = abs(r["quad"][0] - ref["quad"][0]) / abs(ref["quad"][0])
            rec["meets_1e-6"] = bool(rec["rel_dloglik_vs_fp64"] <= 1e-6 and not rec["fp64_fallback"])
            rec["speedup_vs_fp64"] = out["fp64"]["evals_per_s"] and rec["evals_per_s"] / out["fp64"]["evals_per_s"]
            lp = pr["lowp"]
            if lp["ms"] > 0:
                ach = lp["flops"] / (lp["ms"] * 1e-3) / 1e12
                rec["offband_gemm"] = {"achieved": ach, "peak": peaks[name],
                                       "unit": "TFLOP/s", "frac": ach / peaks[name]}
        out[name] = rec
    return out


def run_headline(args, mvg, dev, synthetic, torch):
    """The default line: TLR at N = 100,000 (the largest single-GPU workload)
    with the dense FP64 workload (N = 25,600) and the mixed-precision workload
    (N = 50,000) as nested records, and the CPU oracle."""
    n = args.n or 100000
    acc = float(args.accs.split(",")[0])
    rec = tlr_record(args, mvg, dev, synthetic, torch, n, acc, args.steps, args.warmup,
                     simplex=args.simplex)
    dense_rec = mixed_rec = None
    if not args.no_nested:
        dense_rec, _ = dense_record(args, mvg, dev, synthetic, torch, 25600, args.nested_steps, 1,
                                    (256, 512, 768))
        mixed_rec = mixed_record(args, mvg, dev, synthetic, torch, 50000, (0.5, 1.0), 0.5)
    cpu = None
    if not args.no_cpu:
        _step("oracle timing on the host (bounded sample)")
        cpu = cpu_baseline(n, args.cpu_sample_n, (1.0, 1.0, args.a, 0.5, 1.0, 0.5), args.seed)
    t = rec["tlr"]
    _line(METRIC, t["evals_per_s"], "evals/s", args.steps, args.warmup, 1e3 * t["s_per_eval"],
          "f64",
          {"workload": "TLR bivariate parsimonious Matern loglik (generation, compression, TLR "
                       "Cholesky, log-determinant, solve), N=%d locations (%dx%d), tile 1200, "
                       "acc %g, max rank 300, theta=(1,1,%g,0.5,1,0.5), Z = L eps"
                       % (n, 2 * n, 2 * n, acc, args.a),
           "n_loc": n, "nb": 1200, "precision": "tlr", "parallelism": "single GPU"},
          roofline=rec["roofline"], cpu_baseline=cpu,
          tlr=t, dense_fp64=rec["dense_fp64"], ranks=rec["ranks"], memory=rec["memory"],
          simplex7=rec.get("simplex7"), dense_n25600=dense_rec, mixed_n50000=mixed_rec)


def run_batched(args, mvg, dev, synthetic, torch):
    """Many theta on the N = 400 workload (800 x 800) in one persistent launch."""
    n = 400
    th0 = synthetic.THETA_REF
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
    _line(METRIC,
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
    _line(METRIC,
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
    _line(METRIC,
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
    (Section 6.4.1, Experiment 2): 22,464 + 2,500 jittered-grid locations,
    Z = L eps simulated jointly at theta = (1, 1, a, 0.5, 1, 0.5) for each a in
    --mle-as (0.03, 0.09, 0.2); theta estimated from the 22,464 by the
    library's Nelder-Mead driver (exact FP64 likelihoods) from a perturbed
    start, run in chunks of --mle-chunk evaluations restarted from the best
    point (a restarted Nelder-Mead; each chunk reports its progress) until a
    chunk converges or --max-evals is spent; the 2,500 held-out locations are
    then predicted by cokriging with theta-hat and with the true theta."""
    n_fit, n_hold = 22464, 2500
    n = n_fit + n_hold
    nb = args.nb
    recs = []
    for a in [float(v) for v in args.mle_as.split(",")]:
        th = (1.0, 1.0, a, 0.5, 1.0, 0.5)
        start = (1.2, 0.8, 1.3 * a, 0.6, 0.9, 0.3)
        xr, yr = synthetic.jittered_grid(n, args.seed)
        _, xs, ys = mvg.morton_order(dev(xr), dev(yr), sorted_xy=True)
        _step("mle a=%g: Z = L eps on %d locations" % (a, n))
        A = mvg.cov_generate(xs, ys, th, {"nb": nb})
        if mvg.potrf_tiled(A):
            raise SystemExit("Sigma(theta) not positive definite")
        z = mvg.mvg_trmv(A, dev(synthetic.normal_eps(2 * n, args.seed)))
        del A
        hold = np.sort(synthetic.rng(args.seed, 6).permutation(n)[:n_hold])
        fit_idx = np.setdiff1d(np.arange(n), hold)
        hi = torch.as_tensor(hold).cuda()
        fi = torch.as_tensor(fit_idx).cuda()
        zz = z.view(n, 2)
        xf, yf = xs[fi].contiguous(), ys[fi].contiguous()
        zf = zz[fi].reshape(-1).contiguous()
        x0, y0 = xs[hi].contiguous(), ys[hi].contiguous()
        z0 = zz[hi].cpu().numpy()
        o = {"nb": nb}
        l_true = float(mvg.loglik(xf, yf, zf, th, o)["loglik"][0])
        cur = start
        evals = 0
        best = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while evals < args.max_evals:
            fit = mvg.mle_fit(xf, yf, zf, cur, o, max_evals=min(args.mle_chunk,
                                                                args.max_evals - evals))
            evals += fit["evals"]
            best = fit
            cur = fit["theta"]
            _step("mle a=%g: %d evaluations, loglik %.3f (true theta %.3f), theta %s%s"
                  % (a, evals, fit["loglik"], l_true, np.round(cur, 4).tolist(),
                     ", converged" if fit["converged"] else ""))
            if fit["converged"]:
                break
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mspe = {}
        for tag, t in (("theta_hat", best["theta"]), ("theta_true", th)):
            _, F = mvg.loglik(xf, yf, zf, t, o, keep=True)
            zh = mvg.cokrige_predict(F, x0, y0).cpu().numpy().reshape(n_hold, 2)
            del F
            mspe[tag] = [float(np.mean((zh[:, j] - z0[:, j]) ** 2)) for j in range(2)]
        recs.append({"a": a, "theta_true": th, "theta_start": start, "theta_hat": best["theta"],
                     "loglik_hat": best["loglik"], "loglik_true": l_true,
                     "converged": best["converged"], "evals": evals, "seconds": dt,
                     "evals_per_s": evals / dt, "mspe": mspe})
    tot_e = sum(r["evals"] for r in recs)
    tot_t = sum(r["seconds"] for r in recs)
    _line(METRIC, tot_e / tot_t, "evals/s", tot_e, 0, 1e3 * tot_t / tot_e, "f64",
          {"workload": "Nelder-Mead MLE at the shape of Experiment 2: fit on %d of %d locations "
                       "(%dx%d), cokriging of the %d held out, nb %d, FP64, a in %s"
                       % (n_fit, n, 2 * n_fit, 2 * n_fit, n_hold, nb, args.mle_as),
           "n_loc": n_fit, "held_out": n_hold, "precision": "fp64"},
          fits=recs)


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
    _line(METRIC,
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


def run_dense(args, mvg, dev, synthetic, torch):
    """The dense FP64 workload alone (N = 25,600), with the mixed-precision
    and DST variants of the same inputs."""
    n = args.n or 25600
    tune = (256, 512, 768, 1024) if args.tune_1024 else (256, 512, 768)
    rec, (xs, ys, z, th) = dense_record(args, mvg, dev, synthetic, torch, n, args.steps,
                                        args.warmup, tune)
    args.nb = rec["nb"]
    args.n = n
    extra = {}
    if not args.no_variants:
        _step("dense: mixed-precision and DST variants")
        extra["variants"] = run_variants(mvg, xs, ys, z, th, args, rec["loglik"])
    if not args.no_cpu:
        _step("dense: oracle timing on the host (bounded sample)")
        extra["cpu_baseline"] = cpu_baseline(n, args.cpu_sample_n, th, args.seed)
    roof = rec.pop("roofline")
    steps, warmup = rec.pop("steps"), rec.pop("warmup")  # the line's own fields
    _line(METRIC, rec["evals_per_s"], "evals/s", steps, warmup, rec["ms_per_step"],
          "f64", {"workload": rec.pop("workload"), "n_loc": n, "matrix": 2 * n, "nb": rec["nb"],
                  "precision": "fp64", "parallelism": "single GPU"},
          roofline=roof, **rec, **extra)


def run_mixed(args, mvg, dev, synthetic, torch):
    """Mixed precision on the N = 50,000 workload for one (nu11, nu22, beta)."""
    n = args.n or 50000
    nu = tuple(float(v) for v in args.nu.split(","))
    rec = mixed_record(args, mvg, dev, synthetic, torch, n, nu, args.beta, reps=max(1, args.steps))
    best = max((rec[k] for k in ("fp32x", "bf16x3", "fp32") if rec[k].get("meets_1e-6")),
               key=lambda r: r["evals_per_s"], default=rec["fp64"])
    _line(METRIC, best["evals_per_s"], "evals/s", max(1, args.steps), 1,
          1e3 / best["evals_per_s"], "f64/f32/bf16",
          {"workload": "mixed-precision bivariate Matern loglik, N=%d locations (%dx%d), nb 1024, "
                       "FP64 band of 2 tiles, nu=%s, beta=%g" % (n, 2 * n, 2 * n, nu, args.beta),
           "n_loc": n, "precision": "mixed"}, **rec)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=None,
                    help="locations (default: 100,000 for the headline and tlr, 25,600 for dense, "
                         "50,000 for mixed)")
    ap.add_argument("--a", type=float, default=0.1)
    ap.add_argument("--nb", type=int, default=0,
                    help="dense tile size (0: autotuned among 256/512/768; mloe / trivariate / "
                         "mle use 1024)")
    ap.add_argument("--tune-1024", action="store_true", help="dense: also try tile size 1024")
    ap.add_argument("--targets", type=int, default=100)
    ap.add_argument("--cpu-sample-n", type=int, default=6000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-nested", action="store_true",
                    help="headline: skip the nested dense (N=25,600) and mixed (N=50,000) records")
    ap.add_argument("--nested-steps", type=int, default=3)
    ap.add_argument("--simplex", action="store_true",
                    help="headline: also the 7-point simplex in one call")
    ap.add_argument("--no-variants", action="store_true",
                    help="dense: skip the mixed-precision evaluations of the same inputs")
    ap.add_argument("--band", type=int, default=2, help="FP64 band width in tiles (mixed)")
    ap.add_argument("--wide-band", type=int, default=16,
                    help="second, wider FP64 band for the FP32 variant")
    ap.add_argument("--nu", default="0.5,1.0", help="mixed: nu11,nu22")
    ap.add_argument("--beta", type=float, default=0.5, help="mixed: beta")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "dense", "tlr", "mixed", "batched", "serving", "mloe",
                             "trivariate", "mle"],
                    help="headline: TLR at N=100,000 with nested dense / mixed records; dense: "
                         "N=25,600 FP64 (+ mixed variants); tlr: TLR alone (+ simplex); mixed: "
                         "N=50,000 FP32X / FP32 vs FP64; batched: many theta at N=400 in one "
                         "launch; serving: request stream; mloe: MLOE/MMOM at N=25,600; "
                         "trivariate: p = 3 at N=17,066; mle: Nelder-Mead at N=22,464")
    ap.add_argument("--accs", default="1e-7", help="TLR accuracy")
    ap.add_argument("--white-z", action="store_true",
                    help="tlr: Z = eps without the dense FP64 set-up (counter runs only)")
    ap.add_argument("--no-simplex", action="store_true",
                    help="tlr: skip the 7-point simplex evaluated in one call")
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--max-evals", type=int, default=1500, help="MLE: evaluation budget per fit")
    ap.add_argument("--mle-chunk", type=int, default=100,
                    help="MLE: evaluations per restarted Nelder-Mead chunk")
    ap.add_argument("--mle-as", default="0.03,0.09,0.2", help="MLE: ranges a to fit")
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
    if args.workload == "headline":
        return run_headline(args, mvg, dev, synthetic, torch)
    if args.workload == "tlr":
        args.n = args.n or 100000
        return run_tlr(args, mvg, dev, synthetic, torch)
    if args.workload == "dense":
        return run_dense(args, mvg, dev, synthetic, torch)
    if args.workload == "mixed":
        return run_mixed(args, mvg, dev, synthetic, torch)
    args.n = args.n or 25600
    args.nb = args.nb or 1024
    if args.workload == "batched":
        return run_batched(args, mvg, dev, synthetic, torch)
    if args.workload == "serving":
        return run_serving(args, mvg, dev, synthetic, torch)
    if args.workload == "mloe":
        return run_mloe(args, mvg, dev, synthetic, torch)
    if args.workload == "mle":
        return run_mle(args, mvg, dev, synthetic, torch)
    if args.workload == "trivariate":
        args.n = 17066 if args.n == 25600 else args.n
        return run_trivariate(args, mvg, dev, synthetic, torch)


if __name__ == "__main__":
    main()
