"""GPU checks of the tile-low-rank path (Section 5.3) against the FP64 oracle.

Compression is checked tile by tile against the oracle's truncated SVD of the
same tiles under the same Frobenius tail rule (the GPU's column-pivoted QR is
not the optimal truncation, so its rank may exceed the SVD's by a few; the
sketch sees the same singular values) and by the 2-norm of each tile's error
(<= a small multiple of acc).  The
log-likelihood is checked against the exact oracle value (relative 1e-6 at
acc <= 1e-7, the target for the TLR form) and against the oracle's likelihood
of its own truncated matrix (the compression-only error)."""
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


def _data(orc, n, seed, theta, simulate=True):
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    z = orc.simulate_z(x, y, theta, synthetic.normal_eps(2 * n, seed)) if simulate else None
    return x, y, z


TH = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)


@pytest.mark.parametrize("acc", [1e-5, 1e-9])
def test_tlr_compress_tiles(lib, orc, acc):
    n, nb = 600, 200
    x, y, _ = _data(orc, n, 3, TH, simulate=False)
    _say("tlr_compress n=%d nb=%d acc=%g" % (n, nb, acc))
    A, ranks = lib.tlr_compress(_dev(x), _dev(y), TH, {"nb": nb, "tlr_acc": acc})
    S = orc.cov_dense(x, y, TH)
    _, oranks = orc.tlr_truncate_tiles(S, nb, acc, 300, rule="frobenius")
    St = A.to_dense().cpu().numpy()
    T = ranks.shape[0]
    worst = 0.0
    for I in range(T):
        for J in range(I):
            o = int(oranks[I, J])
            assert o - 1 <= int(ranks[I, J]) <= o + max(4, o // 8), (I, J, ranks[I, J], o)
            assert ranks[I, J] == ranks[J, I]
            d = St[I * nb:(I + 1) * nb, J * nb:(J + 1) * nb] - S[I * nb:(I + 1) * nb, J * nb:(J + 1) * nb]
            worst = max(worst, np.linalg.norm(d, 2))
    _say("  ranks %s\n  worst tile error %.2e" % (ranks[np.tril_indices(T, -1)], worst))
    assert worst <= 4 * acc
    # diagonal tiles are the generated tiles (GPU K_nu vs the oracle's: 1e-13)
    for I in range(T):
        blk = slice(I * nb, (I + 1) * nb)
        assert np.max(np.abs(np.tril(St[blk, blk]) - np.tril(S[blk, blk]))) <= 1e-13


def test_tlr_dense_fallback(lib, orc):
    """max_rank below the needed rank keeps tiles dense (rank -1), exactly."""
    n, nb = 400, 160
    x, y, _ = _data(orc, n, 4, TH, simulate=False)
    A, ranks = lib.tlr_compress(_dev(x), _dev(y), TH, {"nb": nb, "tlr_acc": 1e-9,
                                                        "tlr_max_rank": 6})
    S = orc.cov_dense(x, y, TH)
    St = A.to_dense().cpu().numpy()
    T = ranks.shape[0]
    assert (ranks[np.tril_indices(T, -1)] == -1).any()
    for I in range(T):
        for J in range(I):
            r = int(ranks[I, J])
            assert r == -1 or r <= 6
            blk = (slice(I * nb, min(800, (I + 1) * nb)), slice(J * nb, (J + 1) * nb))
            err = np.abs(St[blk] - S[blk]).max()
            if r == -1:
                assert err <= 1e-13
            else:
                assert err <= 1e-8


@pytest.mark.parametrize("acc", [1e-5, 1e-7, 1e-9])
def test_tlr_loglik(lib, orc, acc):
    n, nb = 900, 256   # N = 1800: 8 tiles, the last one 8 rows
    x, y, z = _data(orc, n, 5, TH)
    ref = orc.loglik(x, y, z, TH)
    S = orc.cov_dense(x, y, TH)
    St, _ = orc.tlr_truncate_tiles(S, nb, acc, 300)
    ref_t = orc.loglik_from_matrix(St, z)
    got = lib.loglik(_dev(x), _dev(y), _dev(z), TH,
                     {"nb": nb, "precision": lib.MVG_TLR, "tlr_acc": acc})
    assert got["status"][0] == 0
    d_exact = abs(got["loglik"][0] - ref["loglik"]) / abs(ref["loglik"])
    d_trunc = abs(got["loglik"][0] - ref_t["loglik"]) / abs(ref["loglik"])
    d_ocomp = abs(ref_t["loglik"] - ref["loglik"]) / abs(ref["loglik"])
    _say("  acc %g: rel dl vs exact %.2e, vs oracle-truncated %.2e (oracle compression alone %.2e)"
         % (acc, d_exact, d_trunc, d_ocomp))
    assert d_exact <= max(1e-6, 20 * d_ocomp)
    if acc <= 1e-7:
        assert d_exact <= 1e-6


def test_tlr_tile_1200_padding(lib, orc):
    """Tile size 1200 (not a multiple of 64: padded diagonal tiles)."""
    n = 1500
    x, y, z = _data(orc, n, 6, TH)
    ref = orc.loglik(x, y, z, TH)
    got = lib.loglik(_dev(x), _dev(y), _dev(z), TH,
                     {"nb": 1200, "precision": lib.MVG_TLR, "tlr_acc": 1e-9})
    d = abs(got["loglik"][0] - ref["loglik"]) / abs(ref["loglik"])
    _say("  nb 1200 rel dl %.2e" % d)
    assert got["status"][0] == 0 and d <= 1e-8


def test_tlr_factor_reproduces_compressed_sigma(lib, orc):
    n, nb = 500, 128
    x, y, _ = _data(orc, n, 7, TH, simulate=False)
    o = {"nb": nb, "precision": lib.MVG_TLR, "tlr_acc": 1e-9}
    A, _ = lib.tlr_compress(_dev(x), _dev(y), TH, o)
    St = A.to_dense().cpu().numpy()
    St = np.tril(St) + np.tril(St, -1).T
    assert lib.potrf_tiled(A, o) == 0
    L = A.to_dense().cpu().numpy()
    err = np.abs(L @ L.T - St).max()
    _say("  |L L^T - Sigma~| %.2e" % err)
    assert err <= 1e-7


def test_tlr_cokriging_and_batch(lib, orc):
    n, nb = 700, 200
    x, y, z = _data(orc, n, 8, TH)
    x0, y0 = synthetic.uniform_targets(30, 8)
    o = {"nb": nb, "precision": lib.MVG_TLR, "tlr_acc": 1e-9}
    res, F = lib.loglik(_dev(x), _dev(y), _dev(z), TH, o, keep=True)
    zh = lib.cokrige_predict(F, _dev(x0), _dev(y0)).cpu().numpy()
    ref = orc.cokrige(x, y, z, TH, x0, y0)
    rmse = float(np.sqrt(np.mean((zh - ref) ** 2)))
    _say("  TLR cokriging rmse diff %.2e" % rmse)
    assert rmse <= 1e-6
    ths = synthetic.nelder_mead_simplex(TH)[:3]
    batch = lib.loglik(_dev(x), _dev(y), _dev(z), ths, o)
    for i, t in enumerate(ths):
        one = lib.loglik(_dev(x), _dev(y), _dev(z), t, o)
        assert one["loglik"][0] == batch["loglik"][i]
