"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: it only draws locations, the
standard-normal vector eps that becomes Z = L eps, prediction targets, parameter
sets and request streams.  Every draw comes from numpy's Philox counter-based
generator keyed by an explicit seed, so both the GPU path and the oracle see
identical inputs.

Workload shapes follow the paper's synthetic experiments (Section 6.4): points
on the unit square, grid-like, theta = (sigma11^2, sigma22^2, a, nu11, nu22, beta)
near (1, 1, a, 0.5, 1, 0.5).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# the workloads' reference theta (sigma11^2, sigma22^2, a, nu11, nu22, beta)
THETA_REF = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """Philox generator for (seed, stream); streams separate independent draws."""
    return np.random.Generator(np.random.Philox(key=[int(seed), int(stream)]))


def jittered_grid(n: int, seed: int):
    """n locations on [0,1]^2: a k x k grid (k = ceil(sqrt n)) with cell-centred
    points jittered by U(-0.4, 0.4) cell widths, k^2 - n points dropped at random.
    Returns (x, y) float64 in generation order (not Morton-ordered)."""
    if n < 1:
        raise ValueError("n must be >= 1")
    k = int(math.ceil(math.sqrt(n)))
    g = rng(seed, 1)
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    ii = ii.reshape(-1).astype(np.float64)
    jj = jj.reshape(-1).astype(np.float64)
    jx = g.uniform(-0.4, 0.4, size=k * k)
    jy = g.uniform(-0.4, 0.4, size=k * k)
    x = (ii + 0.5 + jx) / k
    y = (jj + 0.5 + jy) / k
    if k * k > n:
        keep = np.sort(g.permutation(k * k)[:n])
        x, y = x[keep], y[keep]
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def normal_eps(m: int, seed: int) -> np.ndarray:
    """m iid N(0, 1) draws (the eps of Z = L eps)."""
    return rng(seed, 2).standard_normal(m)


def uniform_targets(m: int, seed: int):
    """m prediction locations uniform on [0,1]^2."""
    g = rng(seed, 3)
    return g.uniform(0.0, 1.0, size=m), g.uniform(0.0, 1.0, size=m)


def nelder_mead_simplex(theta0, step: float = 0.10, beta_step: float = 0.05):
    """The 7 points of an initial Nelder-Mead simplex over the 6 parameters:
    theta0 and theta0 with one coordinate moved (+10 %, beta by +0.05)."""
    t0 = np.asarray(theta0, dtype=np.float64)
    pts = [t0.copy()]
    for i in range(6):
        t = t0.copy()
        if i == 5:
            t[i] = t[i] + beta_step
        else:
            t[i] = t[i] * (1.0 + step)
        pts.append(t)
    return np.stack(pts)


def jittered_thetas(count: int, seed: int, theta0=THETA_REF, rel: float = 0.2):
    """count parameter vectors theta0 * U(1-rel, 1+rel) per coordinate, beta
    clipped to |beta| < 0.99."""
    g = rng(seed, 4)
    t = np.asarray(theta0, dtype=np.float64)[None, :] * g.uniform(1 - rel, 1 + rel, size=(count, 6))
    t[:, 5] = np.clip(t[:, 5], -0.99, 0.99)
    return t


@dataclass
class Request:
    arrival_s: float
    kind: str          # "loglik" or "cokrige"
    dataset: int
    n: int
    theta: np.ndarray
    n_targets: int


def serving_stream(num: int, seed: int, rate_hz: float = 50.0, n_datasets: int = 32,
                   n_lo: int = 1000, n_hi: int = 20000, cokrige_frac: float = 0.10,
                   n_targets: int = 100):
    """Poisson arrivals of likelihood / cokriging requests over a pool of
    datasets with n ~ U[n_lo, n_hi].  Returns (requests, dataset_sizes)."""
    g = rng(seed, 5)
    sizes = g.integers(n_lo, n_hi + 1, size=n_datasets)
    gaps = g.exponential(1.0 / rate_hz, size=num)
    t = np.cumsum(gaps)
    thetas = jittered_thetas(num, seed + 7919)
    reqs = []
    for i in range(num):
        kind = "cokrige" if g.uniform() < cokrige_frac else "loglik"
        d = int(g.integers(0, n_datasets))
        reqs.append(Request(float(t[i]), kind, d, int(sizes[d]), thetas[i],
                            n_targets if kind == "cokrige" else 0))
    return reqs, sizes
