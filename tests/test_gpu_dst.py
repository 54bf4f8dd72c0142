"""GPU checks of the Diagonal Super Tile approximation (Section 4.4; DST 40/60
and 70/30 of Experiment 2, Section 6.4.1): Sigma with the tiles far from the
diagonal annihilated, factored exactly in FP64.  The oracle masks its own
dense Sigma with the same band (``dst_mask``) and factors it; both sides
factor the same matrix, so the likelihood agrees to FP64 rounding (1e-9
relative, as for the exact path), and a truncated matrix that is not
positive definite fails at the same pivot."""
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


def _data(orc, n, seed, th):
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    z = orc.simulate_z(x, y, th, synthetic.normal_eps(2 * n, seed))
    return x, y, z


def _opts(lib, nb, w):
    return {"nb": nb, "precision": lib.MVG_DST, "band_tiles": w}


@pytest.mark.parametrize("n,nb,keep,a", [
    (1000, 128, 0.4, 0.03), (1000, 128, 0.7, 0.03), (1000, 128, 0.7, 0.1),
    (1337, 256, 0.5, 0.05),                            # ragged last tile
])
def test_dst_loglik_matches_oracle(lib, orc, n, nb, keep, a):
    th = (1.0, 1.0, a, 0.5, 1.0, 0.5)
    x, y, z = _data(orc, n, 7, th)
    T = (2 * n + nb - 1) // nb
    w = lib.mvg_dst_band(n, nb, keep)
    assert w == orc.dst_band(T, keep)
    _say("dst n=%d nb=%d keep=%g a=%g -> band %d of %d tiles" % (n, nb, keep, a, w, T))
    ref = orc.loglik_from_matrix(orc.dst_mask(orc.cov_dense(x, y, th), nb, w), z)
    got = lib.loglik(_dev(x), _dev(y), _dev(z), th, _opts(lib, nb, w))
    _say("  oracle %s  gpu %s (status %d)" % (ref["loglik"], got["loglik"][0], got["status"][0]))
    if ref["info"]:
        assert got["status"][0] == ref["info"]
        return
    assert got["status"][0] == 0
    for k in ("loglik", "logdet", "quad"):
        assert abs(got[k][0] - ref[k]) <= 1e-9 * abs(ref[k]), k


def test_dst_not_positive_definite_reported(lib, orc):
    """Strong dependence with a narrow band: the truncated matrix is
    indefinite; the GPU reports the oracle's first failing pivot."""
    th = (1.0, 1.0, 0.2, 0.5, 1.0, 0.5)
    x, y, z = _data(orc, 800, 2, th)
    nb, w = 128, 2
    ref = orc.loglik_from_matrix(orc.dst_mask(orc.cov_dense(x, y, th), nb, w), z)
    got = lib.loglik(_dev(x), _dev(y), _dev(z), th, _opts(lib, nb, w))
    _say("  dst a=0.2 band 2: oracle info %d, gpu status %d" % (ref["info"], got["status"][0]))
    assert got["status"][0] == ref["info"]
    if ref["info"]:
        assert got["loglik"][0] == -np.inf


def test_dst_full_band_equals_fp64_and_band_one_is_block_diagonal(lib, orc):
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y, z = _data(orc, 700, 5, th)
    nb, T = 128, (1400 + 127) // 128
    d64 = lib.loglik(_dev(x), _dev(y), _dev(z), th, {"nb": nb})
    full = lib.loglik(_dev(x), _dev(y), _dev(z), th, _opts(lib, nb, T))
    assert full["loglik"][0] == d64["loglik"][0]   # same kernels, nothing annihilated
    one = lib.loglik(_dev(x), _dev(y), _dev(z), th, _opts(lib, nb, 1))
    ref = orc.loglik_from_matrix(orc.dst_mask(orc.cov_dense(x, y, th), nb, 1), z)
    assert one["status"][0] == 0
    assert abs(one["loglik"][0] - ref["loglik"]) <= 1e-9 * abs(ref["loglik"])


def test_dst_generated_tiles(lib, orc):
    """Kept tiles equal the FP64 generation bitwise; annihilated tiles read
    as exact zeros."""
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y = synthetic.jittered_grid(500, 4)
    nb, w = 128, 3
    A = lib.cov_generate(_dev(x), _dev(y), th, _opts(lib, nb, w)).to_dense().cpu().numpy()
    B = lib.cov_generate(_dev(x), _dev(y), th, {"nb": nb}).to_dense().cpu().numpy()
    np.testing.assert_array_equal(A, orc.dst_mask(B, nb, w))


def test_dst_factor_cokriging_and_mse(lib, orc):
    """Predictions and their MSE from a resident DST factor (the many-column
    solve skips the annihilated tiles) against the oracle's masked matrix."""
    th = (1.0, 1.0, 0.03, 0.5, 1.0, 0.5)   # positive definite at keep 0.5 (oracle)
    x, y, z = _data(orc, 900, 11, th)
    x0, y0 = synthetic.uniform_targets(30, 11)
    nb = 128
    w = lib.mvg_dst_band(900, nb, 0.5)
    res, F = lib.loglik(_dev(x), _dev(y), _dev(z), th, _opts(lib, nb, w), keep=True)
    assert res["status"][0] == 0 and F is not None
    zh, mse = lib.cokrige_predict(F, _dev(x0), _dev(y0), with_mse=True)
    S = orc.dst_mask(orc.cov_dense(x, y, th), nb, w)
    L, info = orc.potrf(S)
    assert info == 0
    wv = orc.trsv_lower(L, orc.trsv_lower(L, z), trans=True)
    c0 = orc.cross_cov_targets(x, y, x0, y0, th)
    ref = (c0.T @ wv).reshape(-1, 2)
    U = np.column_stack([orc.trsv_lower(L, c0[:, j]) for j in range(c0.shape[1])])
    ref_mse = 2.0 - (U ** 2).sum(axis=0).reshape(-1, 2).sum(axis=1)
    err = float(np.max(np.abs(zh.cpu().numpy() - ref)))
    merr = float(np.max(np.abs(mse.cpu().numpy() - ref_mse)))
    _say("  dst cokriging max err %.2e, mse max err %.2e" % (err, merr))
    assert err <= 1e-9 and merr <= 1e-9
