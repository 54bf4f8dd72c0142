#!/usr/bin/env python3
"""Writes tests/golden/dense_n25600.json: Eq. (1) evaluated by the oracle on
the dense workload's inputs (n = 25,600 jittered-grid locations, Morton
ordered, 51,200 x 51,200 covariance) for a in {0.1, 0.3, 0.03}, and the FP64
noise floor of that evaluation.

Only the oracle computes the stored values.  The inputs come from the seeded
generators: locations from ``synthetic.jittered_grid(n, seed)`` ordered by
``oracle.morton_order``, Z = ``synthetic.normal_eps(2n, seed)`` (white noise:
the quadratic form then weighs the smallest eigenvalues of Sigma, a harder
case for its relative accuracy than model data).

Noise floor: the Cholesky factorisation is unique for an SPD matrix, so two
correct FP64 evaluations differ only by rounding.  The same Sigma (built by the
oracle) is factored a second time, by a blocked right-looking Cholesky made of
LAPACK / BLAS calls on 4096-wide blocks (scipy's cholesky and
solve_triangular, numpy's matmul; a single LAPACK call on the whole
51,200 x 51,200 matrix overflows 32-bit indexing inside OpenBLAS), and the
log-determinant and quadratic form are recomputed from that factor; the
relative difference to the oracle's values is the floor a third FP64
implementation (the GPU) is judged against.

Each a takes about two hours on eight host cores (the oracle's Crout loop
streams the 21 GB factor once per column); results are appended per a, so an
interrupted run keeps what it finished.  Run from the repository root:

    OMP_NUM_THREADS=6 python tests/golden/make_dense_n25600.py
"""
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle      # noqa: E402
import synthetic   # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "dense_n25600.json")
N_LOC = 25600
SEED = 0
A_VALUES = (0.1, 0.3, 0.03)


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


def host_cpu() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


BLOCK = 4096


def lapack_floor(x, y, z, theta):
    """log|Sigma| and Z^T Sigma^-1 Z from a blocked LAPACK / BLAS Cholesky
    factor of the oracle's Sigma (lower triangle, factored in place)."""
    import scipy.linalg as sla
    S = oracle.cov_dense(x, y, theta)            # row-major, symmetric
    F = S.T                                      # the same matrix, Fortran order: no copy
    N = F.shape[0]
    for k0 in range(0, N, BLOCK):
        k1 = min(N, k0 + BLOCK)
        L11 = sla.cholesky(np.array(F[k0:k1, k0:k1]), lower=True, check_finite=False)
        F[k0:k1, k0:k1] = L11
        if k1 == N:
            break
        L21 = sla.solve_triangular(L11, np.array(F[k1:, k0:k1]).T, lower=True,
                                   check_finite=False).T      # A21 L11^-T
        F[k1:, k0:k1] = L21
        for i0 in range(k1, N, BLOCK):                         # lower part of the trailing update
            i1 = min(N, i0 + BLOCK)
            F[i0:i1, k1:i1] -= L21[i0 - k1:i1 - k1] @ L21[:i1 - k1].T
        del L21
    logdet = 2.0 * float(np.sum(np.log(np.diagonal(F))))
    yv = np.array(z, dtype=np.float64)
    for k0 in range(0, N, BLOCK):                              # forward substitution by blocks
        k1 = min(N, k0 + BLOCK)
        r = yv[k0:k1] - (F[k0:k1, :k0] @ yv[:k0] if k0 else 0.0)
        yv[k0:k1] = sla.solve_triangular(np.array(F[k0:k1, k0:k1]), r, lower=True,
                                         check_finite=False)
    quad = float(np.dot(yv, yv))
    del S, F
    return logdet, quad


def save(rec):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    os.replace(tmp, OUT)


def main():
    oracle.build(force=False)
    x, y = synthetic.jittered_grid(N_LOC, SEED)
    p = oracle.morton_order(x, y)
    x, y = np.ascontiguousarray(x[p]), np.ascontiguousarray(y[p])
    z = synthetic.normal_eps(2 * N_LOC, SEED)
    rec = {}
    if os.path.exists(OUT):
        rec = json.load(open(OUT))
    rec.update({
        "_comment": "Eq. (1) by the oracle at n = 25,600 (51,200 x 51,200), written by "
                    "tests/golden/make_dense_n25600.py; floor = relative difference to a "
                    "LAPACK factorisation of the same oracle-built Sigma",
        "n_loc": N_LOC, "seed": SEED,
        "inputs": "x, y = synthetic.jittered_grid(n, seed) ordered by oracle.morton_order; "
                  "z = synthetic.normal_eps(2n, seed)",
        "sha256_x": sha(x), "sha256_y": sha(y), "sha256_z": sha(z),
        "host": {"cpu": host_cpu(), "threads": oracle.num_threads()},
    })
    rec.setdefault("cases", {})
    for a in A_VALUES:
        key = "a%g" % a
        if "floor_quad" in rec["cases"].get(key, {}):
            continue
        theta = (1.0, 1.0, a, 0.5, 1.0, 0.5)
        print("oracle loglik, a = %g ..." % a, flush=True)
        t0 = time.perf_counter()
        r = oracle.loglik(x, y, z, theta)
        t_oracle = time.perf_counter() - t0
        print("  %.1f s: %r" % (t_oracle, r), flush=True)
        rec["cases"][key] = {
            "theta": list(theta),
            "loglik": r["loglik"], "logdet": r["logdet"], "quad": r["quad"], "info": r["info"],
            "oracle_seconds": t_oracle, "oracle_threads": oracle.num_threads(),
        }
        save(rec)
        t1 = time.perf_counter()
        ld_l, q_l = lapack_floor(x, y, z, theta)
        t_lapack = time.perf_counter() - t1
        case = {
            "theta": list(theta),
            "loglik": r["loglik"], "logdet": r["logdet"], "quad": r["quad"], "info": r["info"],
            "oracle_seconds": t_oracle, "oracle_threads": oracle.num_threads(),
            "lapack_logdet": ld_l, "lapack_quad": q_l, "lapack_seconds": t_lapack,
            "floor_logdet": abs(ld_l - r["logdet"]) / abs(r["logdet"]),
            "floor_quad": abs(q_l - r["quad"]) / abs(r["quad"]),
        }
        print("  LAPACK %.1f s: logdet %.17g quad %.17g; floor %.2e / %.2e"
              % (t_lapack, ld_l, q_l, case["floor_logdet"], case["floor_quad"]), flush=True)
        rec["cases"][key] = case
        save(rec)


if __name__ == "__main__":
    main()
