"""GPU parity of the dense FP64 path against the CPU oracle (same seeded inputs).

Tolerances: covariance entries 1e-13 relative (both sides evaluate K_nu to
~1e-15 with different methods); Cholesky factor within 10x the oracle-vs-LAPACK
noise floor of the same matrix; log-likelihood 1e-9 relative (the target the
method is held to for FP64)."""
import math
import sys

import numpy as np
import pytest
import scipy.linalg

import synthetic

pytestmark = pytest.mark.gpu

THETA0 = synthetic.THETA_REF


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
    if simulate:
        z = orc.simulate_z(x, y, theta, synthetic.normal_eps(2 * n, seed))
    else:
        z = synthetic.normal_eps(2 * n, seed)
    return x, y, z


@pytest.mark.parametrize("n,nb", [(400, 128), (400, 256), (333, 256), (700, 512)])
def test_cov_generate_entries(lib, orc, n, nb):
    _say("cov_generate n=%d nb=%d" % (n, nb))
    th = (1.3, 0.7, 0.1, 0.5, 1.0, 0.5)
    x, y, _ = _data(orc, n, 11, th, simulate=False)
    A = lib.cov_generate(_dev(x), _dev(y), th, {"nb": nb})
    S = A.to_dense().cpu().numpy()
    R = np.tril(orc.cov_dense(x, y, th))
    assert np.all(np.isfinite(S))
    err = np.abs(S - R) / np.maximum(np.abs(R), 1e-300)
    assert err.max() <= 1e-13, err.max()


@pytest.mark.parametrize("nu", [(0.5, 1.0), (0.25, 0.8), (1.5, 2.5), (0.7, 3.3), (4.5, 5.0)])
@pytest.mark.parametrize("a", [0.03, 0.3, 2.0])
def test_cov_generate_smoothness_range(lib, orc, nu, a):
    """Quadrature levels and closed forms across smoothness and range."""
    th = (1.0, 2.0, a, nu[0], nu[1], -0.4)
    _say("cov_generate nu=%s a=%g" % (nu, a))
    x, y, _ = _data(orc, 160, 5, th, simulate=False)
    x = np.concatenate([x, [0.5, 0.5 + 1e-9, 3.0, 40.0]])   # near-coincident and far points
    y = np.concatenate([y, [0.5, 0.5, 3.0, -40.0]])
    A = lib.cov_generate(_dev(x), _dev(y), th, {"nb": 128})
    S = A.to_dense().cpu().numpy()
    R = np.tril(orc.cov_dense(x, y, th))
    big = np.abs(R) > 1e-280
    err = np.abs(S[big] - R[big]) / np.abs(R[big])
    assert err.max() <= 2e-13, err.max()
    assert np.all(np.abs(S[~big]) <= 1e-280)


def test_cov_generate_gather_matches_dense(lib, orc):
    th = THETA0
    x, y, _ = _data(orc, 300, 3, th, simulate=False)
    A = lib.cov_generate(_dev(x), _dev(y), th, {"nb": 256})
    g = np.random.default_rng(0)
    r = g.integers(0, 600, 500)
    c = g.integers(0, 600, 500)
    r, c = np.maximum(r, c), np.minimum(r, c)
    got = A.gather(r, c).cpu().numpy()
    ref = orc.cov_entries(x, y, th, r, c)
    assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-300)) <= 1e-13


@pytest.mark.parametrize("n,nb,a", [(400, 128, 0.1), (400, 256, 0.03), (400, 256, 0.3),
                                    (555, 256, 0.1), (1000, 512, 0.1),
                                    (1600, 768, 0.1), (1600, 1024, 0.3), (1600, 1024, 0.03)])
def test_potrf_factor_matches_oracle(lib, orc, n, nb, a):
    _say("potrf n=%d nb=%d a=%g" % (n, nb, a))
    th = (1.0, 1.0, a, 0.5, 1.0, 0.5)
    x, y, _ = _data(orc, n, 7, th, simulate=False)
    A = lib.cov_generate(_dev(x), _dev(y), th, {"nb": nb})
    info = lib.potrf_tiled(A)
    assert info == 0
    Lg = A.to_dense().cpu().numpy()
    S = orc.cov_dense(x, y, th)
    Lo, oinfo = orc.potrf(S)
    assert oinfo == 0
    Ll = scipy.linalg.cholesky(S, lower=True)
    floor = np.max(np.abs(Lo - Ll))
    err = np.max(np.abs(Lg - Lo))
    _say("  factor err %.3e, oracle-vs-LAPACK floor %.3e" % (err, floor))
    assert err <= max(10 * floor, 1e-13)


@pytest.mark.parametrize("a", [0.03, 0.1, 0.3])
@pytest.mark.parametrize("nb", [128, 256])
def test_loglik_n400(lib, orc, a, nb):
    """N = 400 jittered 20 x 20 grid, theta of the small workload with a varied."""
    th = (1.0, 1.0, a, 0.5, 1.0, 0.5)
    _say("loglik N=400 a=%g nb=%d" % (a, nb))
    x, y, z = _data(orc, 400, 0, th)
    ref = orc.loglik(x, y, z, th)
    got = lib.loglik(_dev(x), _dev(y), _dev(z), th, {"nb": nb})
    assert got["status"][0] == 0
    for key in ("loglik", "logdet", "quad"):
        rel = abs(got[key][0] - ref[key]) / abs(ref[key])
        _say("  %s gpu %.15e oracle %.15e rel %.2e" % (key, got[key][0], ref[key], rel))
        assert rel <= 1e-9, key


def test_loglik_ragged_multi_tile(lib, orc):
    th = (1.5, 0.8, 0.15, 0.8, 1.7, -0.6)
    x, y, z = _data(orc, 1337, 21, th)
    ref = orc.loglik(x, y, z, th)
    got = lib.loglik(_dev(x), _dev(y), _dev(z), th, {"nb": 256})
    assert abs(got["loglik"][0] - ref["loglik"]) <= 1e-9 * abs(ref["loglik"])


def test_loglik_single_location(lib, orc):
    th = (1.7, 0.4, 0.2, 0.8, 1.3, -0.45)
    z = np.array([0.3, -1.1])
    got = lib.loglik(_dev([0.5]), _dev([0.5]), _dev(z), th, {"nb": 128})
    ref = orc.loglik([0.5], [0.5], z, th)
    assert abs(got["loglik"][0] - ref["loglik"]) <= 1e-13 * abs(ref["loglik"])


def test_loglik_not_positive_definite(lib, orc):
    """Duplicate location: Sigma is singular; the first failing pivot is reported
    and loglik is -inf, as the oracle does."""
    x = np.array([0.1, 0.5, 0.5, 0.9, 0.3])
    y = np.array([0.2, 0.3, 0.3, 0.7, 0.8])
    z = np.ones(10)
    th = THETA0
    ref = orc.loglik(x, y, z, th)
    got = lib.loglik(_dev(x), _dev(y), _dev(z), th, {"nb": 128})
    assert ref["info"] > 0
    assert got["loglik"][0] == -math.inf
    assert got["status"][0] == ref["info"]


def test_invalid_theta_is_rejected(lib):
    x = _dev([0.1, 0.2])
    with pytest.raises(lib.MvgError) as e:
        lib.loglik(x, x, _dev([1.0, 2.0, 3.0, 4.0]), (1, 1, -0.1, 0.5, 1, 0.5))
    assert e.value.code == -5
    with pytest.raises(lib.MvgError):
        lib.loglik(x, x, _dev([1.0, 2.0, 3.0, 4.0]), (1, 1, 0.1, 0.5, 1, 1.5))
    with pytest.raises(lib.MvgError):
        lib.cov_generate(x, x, (1, 1, 0.1, 0.5, 1, 0.5), {"nb": 100})


def test_batched_equals_single_bitwise(lib, orc):
    """Above the small-problem size a batch of theta runs the tiled path theta
    after theta on one arena: bitwise equal to single calls."""
    th0 = THETA0
    x, y, z = _data(orc, 600, 2, th0)
    simplex = synthetic.nelder_mead_simplex(th0)
    b = lib.loglik(_dev(x), _dev(y), _dev(z), simplex, {"nb": 256})
    for i, t in enumerate(simplex):
        s = lib.loglik(_dev(x), _dev(y), _dev(z), t, {"nb": 256})
        assert s["loglik"][0] == b["loglik"][i]
        ref = orc.loglik(x, y, z, t)
        assert abs(b["loglik"][i] - ref["loglik"]) <= 1e-9 * abs(ref["loglik"])


def test_small_batch_agrees_with_single_calls(lib, orc):
    """2n <= 1024: the batch takes the one-launch path (its own summation
    order), single calls the tiled path; they agree to rounding."""
    x, y, z = _data(orc, 400, 2, THETA0)
    simplex = synthetic.nelder_mead_simplex(THETA0)
    b = lib.loglik(_dev(x), _dev(y), _dev(z), simplex, {"nb": 256})
    for i, t in enumerate(simplex):
        s = lib.loglik(_dev(x), _dev(y), _dev(z), t, {"nb": 256})
        assert abs(s["loglik"][0] - b["loglik"][i]) <= 1e-12 * abs(s["loglik"][0])


def test_morton_order_bit_exact(lib, orc):
    x, y = synthetic.jittered_grid(5000, 4)
    x = np.concatenate([x, [0.25, 0.25, 1.0, 0.0, 1.5, -0.2]])
    y = np.concatenate([y, [0.75, 0.75, 1.0, 0.0, 0.5, 2.0]])
    p = lib.morton_order(_dev(x), _dev(y)).cpu().numpy()
    np.testing.assert_array_equal(p, orc.morton_order(x, y))


@pytest.mark.parametrize("nb", [128, 256])
def test_cokrige_matches_oracle(lib, orc, nb):
    th = THETA0
    n = 600
    x, y, z = _data(orc, n, 9, th)
    x0, y0 = synthetic.uniform_targets(100, 9)
    ref, ref_mse = orc.cokrige(x, y, z, th, x0, y0, with_mse=True)
    res, F = lib.loglik(_dev(x), _dev(y), _dev(z), th, {"nb": nb}, keep=True)
    zhat, mse = lib.cokrige_predict(F, _dev(x0), _dev(y0), with_mse=True)
    zhat = zhat.cpu().numpy()
    mse = mse.cpu().numpy()
    rmse = float(np.sqrt(np.mean((zhat - ref) ** 2)))
    _say("  cokrige RMSE(gpu - oracle) = %.3e" % rmse)
    assert rmse <= 1e-10
    np.testing.assert_allclose(mse, ref_mse, rtol=1e-8, atol=1e-12)
    # interpolation at observed sites
    idx = np.array([0, 123, n - 1])
    zo = lib.cokrige_predict(F, _dev(x[idx]), _dev(y[idx])).cpu().numpy()
    np.testing.assert_allclose(zo, z.reshape(n, 2)[idx], rtol=1e-7, atol=1e-7)


def test_mat_loglik_from_factor(lib, orc):
    """Eq. (1) from an existing FP64 factor (mvg_mat_loglik): the same value
    as loglik on the same inputs (same kernels, bitwise) and the oracle's
    within 1e-9; Z drawn as L eps from that factor, as the benchmark does."""
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y, _ = _data(orc, 700, 5, th, simulate=False)
    X, Y = _dev(x), _dev(y)
    A = lib.cov_generate(X, Y, th, {"nb": 256})
    assert lib.potrf_tiled(A) == 0
    z = lib.mvg_trmv(A, _dev(synthetic.normal_eps(1400, 5)))
    got = lib.mvg_mat_loglik(A, z)
    ref = lib.loglik(X, Y, z, th, {"nb": 256})
    for key in ("loglik", "logdet", "quad"):
        assert got[key] == ref[key][0], key
    o = orc.loglik(x, y, z.cpu().numpy(), th)
    assert abs(got["loglik"] - o["loglik"]) <= 1e-9 * abs(o["loglik"])
