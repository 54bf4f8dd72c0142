"""GPU checks of the prediction-efficiency criteria of Section 5.4 (Eq. (5)-(8),
Algorithm 1): per-target LOE and MOM and their means MLOE / MMOM from the
library against the oracle on the same seeded locations, targets and
parameter pairs.

Tolerance: the three mean squared errors are FP64 differences between
tr C(0) and quadratic forms of size ~tr C(0); on these workloads
(condition numbers up to ~1e6) each carries an absolute error of a few
1e-12 in either implementation, so LOE and MOM, ratios of those errors
minus one, agree to 1e-8 absolute; the means likewise."""
import sys

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    import paper_2008_07437_amd as m
    m._lib._load()
    return m


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _sites(orc, n, m, seed):
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    x0, y0 = synthetic.uniform_targets(m, seed + 100)
    return x[p], y[p], x0, y0


TH = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)


@pytest.mark.parametrize("n,m,nb,tha", [
    (500, 30, 128, (1.1, 0.9, 0.13, 0.6, 0.9, 0.45)),
    (333, 17, 128, (0.8, 1.3, 0.07, 0.4, 1.2, 0.6)),     # ragged last tile
    (900, 64, 256, (1.0, 1.0, 0.1, 0.5, 1.0, 0.2)),      # only the colocated correlation differs
    (250, 1, 128, (1.1, 0.9, 0.13, 0.6, 0.9, 0.45)),     # two right-hand sides: per-column kernels
])
def test_mloe_mmom_matches_oracle(lib, orc, n, m, nb, tha):
    x, y, x0, y0 = _sites(orc, n, m, 5)
    _say("mloe n=%d m=%d nb=%d theta_a=%s" % (n, m, nb, tha))
    ref = orc.mloe_mmom(x, y, TH, tha, x0, y0)
    got = lib.mloe_mmom(_dev(x), _dev(y), TH, tha, _dev(x0), _dev(y0), {"nb": nb})
    assert got["status"] == 0
    loe, mom = got["loe"].cpu().numpy(), got["mom"].cpu().numpy()
    _say("  MLOE %.6e (oracle %.6e)  MMOM %.6e (oracle %.6e)  max|dLOE| %.2e max|dMOM| %.2e"
         % (got["mloe"], ref["mloe"], got["mmom"], ref["mmom"],
            np.max(np.abs(loe - ref["loe"])), np.max(np.abs(mom - ref["mom"]))))
    assert np.max(np.abs(loe - ref["loe"])) <= 1e-8
    assert np.max(np.abs(mom - ref["mom"])) <= 1e-8
    assert abs(got["mloe"] - ref["mloe"]) <= 1e-8
    assert abs(got["mmom"] - ref["mmom"]) <= 1e-8
    assert np.all(loe >= -1e-10)   # the true model's predictor is optimal


def test_mloe_mmom_zero_at_true_theta(lib, orc):
    x, y, x0, y0 = _sites(orc, 400, 25, 9)
    got = lib.mloe_mmom(_dev(x), _dev(y), TH, TH, _dev(x0), _dev(y0), {"nb": 128})
    assert got["status"] == 0
    assert np.max(np.abs(got["loe"].cpu().numpy())) <= 1e-9
    assert np.max(np.abs(got["mom"].cpu().numpy())) <= 1e-9


def test_mloe_mmom_rejects_bad_arguments(lib, orc):
    x, y, x0, y0 = _sites(orc, 100, 5, 2)
    with pytest.raises(lib.MvgError):
        lib.mloe_mmom(_dev(x), _dev(y), TH, TH, _dev(x0), _dev(y0),
                      {"nb": 128, "precision": lib.MVG_MIXED_FP32})
    with pytest.raises(lib.MvgError):
        lib.mloe_mmom(_dev(x), _dev(y), TH, (1.0, 1.0, -0.1, 0.5, 1.0, 0.5), _dev(x0), _dev(y0),
                      {"nb": 128})
