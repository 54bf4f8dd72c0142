"""Integrity of the stored full-size FP64 values (tests/golden/dense_n25600.json,
written by tests/golden/make_dense_n25600.py from the oracle alone): the
inputs they were computed on are still what the seeded generators and the
oracle's Morton order produce, each stored l(theta) is Eq. (1) assembled from
its own log-determinant and quadratic form, and each noise floor is the stated
relative difference to its LAPACK values.  A drift in any of these would make
the GPU comparison at that size check against values of other inputs."""
import hashlib
import json
import math
import os

import numpy as np
import pytest

import synthetic

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dense_n25600.json")


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float64).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def golden():
    return json.load(open(PATH))


def test_stored_inputs_are_the_seeded_ones(golden, orc):
    n, seed = golden["n_loc"], golden["seed"]
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    assert _sha(x[p]) == golden["sha256_x"] and _sha(y[p]) == golden["sha256_y"]
    assert _sha(synthetic.normal_eps(2 * n, seed)) == golden["sha256_z"]


@pytest.mark.parametrize("a", [0.1, 0.3, 0.03])
def test_stored_case_is_consistent(golden, a):
    case = golden["cases"]["a%g" % a]
    n = golden["n_loc"]
    assert case["info"] == 0
    assert case["theta"] == [1.0, 1.0, a, 0.5, 1.0, 0.5]
    # Eq. (1): l = -n log(2 pi) - log|Sigma| / 2 - Z^T Sigma^-1 Z / 2 (2n observations)
    ll = -n * math.log(2.0 * math.pi) - 0.5 * case["logdet"] - 0.5 * case["quad"]
    assert abs(ll - case["loglik"]) <= 1e-13 * abs(case["loglik"])
    assert case["quad"] > 0.0
    for key in ("logdet", "quad"):
        fl = abs(case["lapack_" + key] - case[key]) / abs(case[key])
        assert fl == pytest.approx(case["floor_" + key], rel=1e-9, abs=1e-300)
        assert fl <= 1e-10   # two FP64 factorisations of one matrix agree closely
