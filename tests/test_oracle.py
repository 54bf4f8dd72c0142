"""Pins of the FP64 CPU oracle against facts that do not come from the oracle:
closed forms, mpmath / scipy / LAPACK routines, the paper's printed numbers,
invariants and brute force on tiny inputs.  CPU only."""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg
import scipy.special
import scipy.stats

import synthetic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------- Gamma, K_nu

def test_rgamma_series_matches_mpmath(orc):
    mp.mp.dps = 40
    for z in np.linspace(-0.5, 0.5, 41):
        ref = float(mp.rgamma(1 + mp.mpf(float(z))))
        assert abs(orc.rgamma1p(z) - ref) <= 5e-16 * abs(ref)   # a few ulp of Horner rounding


@pytest.mark.parametrize("x", [1e-3, 0.1, 0.3, 0.5, 0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.5, 6.0, 9.75])
def test_gamma_matches_library(orc, x):
    mp.mp.dps = 40
    ref = float(mp.gamma(x))
    assert abs(orc.gamma(x) - ref) <= 4e-16 * ref
    assert abs(orc.gamma(x) - scipy.special.gamma(x)) <= 1e-15 * ref


def test_bessel_k_matches_mpmath_grid(orc):
    mp.mp.dps = 40
    xs = np.concatenate([np.logspace(-10, math.log10(700.0), 70), [1.999999, 2.0, 2.000001]])
    for nu in [0.0, 0.1, 0.25, 0.5, 0.75, 1.0, 1.25, 1.5, 2.0, 2.5, 3.0, 3.7]:
        got = orc.bessel_k(nu, xs)
        for x, g in zip(xs, got):
            ref = float(mp.besselk(nu, x))
            assert abs(g - ref) <= 1e-14 * abs(ref), (nu, x, g, ref)


def test_bessel_k_half_integer_closed_forms(orc):
    x = np.logspace(-6, 2.5, 200)
    k12 = np.sqrt(np.pi / (2 * x)) * np.exp(-x)
    np.testing.assert_allclose(orc.bessel_k(0.5, x), k12, rtol=1e-14)
    np.testing.assert_allclose(orc.bessel_k(1.5, x), k12 * (1 + 1 / x), rtol=1e-14)
    np.testing.assert_allclose(orc.bessel_k(2.5, x), k12 * (1 + 3 / x + 3 / x ** 2), rtol=1e-14)


def test_bessel_k_recurrence_and_scipy(orc):
    x = np.logspace(-3, 2, 50)
    for nu in [0.3, 0.75, 1.0, 1.6]:
        lhs = orc.bessel_k(nu + 1, x)
        rhs = orc.bessel_k(nu - 1, x) + (2 * nu / x) * orc.bessel_k(nu, x)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-13)
        np.testing.assert_allclose(orc.bessel_k(nu, x), scipy.special.kv(nu, x), rtol=1e-13)


# --------------------------------------------------------------------- Matern

def test_matern_reductions(orc):
    x = np.concatenate([[0.0, 1e-10], np.logspace(-4, 2.5, 100)])
    np.testing.assert_allclose(orc.matern(x, 0.5), np.exp(-x), rtol=1e-14)
    np.testing.assert_allclose(orc.matern(x, 1.5), (1 + x) * np.exp(-x), rtol=1e-14)
    np.testing.assert_allclose(orc.matern(x, 2.5), (1 + x + x * x / 3) * np.exp(-x), rtol=1e-14)
    for nu in [0.25, 0.75, 1.0, 2.2]:
        assert orc.matern(0.0, nu)[0] == 1.0
        # near 0, M(x) = 1 - O(x^(2 nu)) for nu < 1: compare with mpmath
        mp.mp.dps = 40
        ref = float(mp.mpf(1e-10) ** nu * mp.besselk(nu, 1e-10) / (2 ** (nu - 1) * mp.gamma(nu)))
        assert abs(orc.matern(1e-10, nu)[0] - ref) <= 1e-14
        # monotone decreasing in x
        m = orc.matern(np.linspace(0, 10, 400), nu)
        assert np.all(np.diff(m) < 0)


def test_paper_printed_drop_to_0p05(orc):
    pins = json.load(open(os.path.join(GOLDEN, "paper_pins.json")))["marginal_drop_to_0p05"]
    th = pins["theta"]
    for case in pins["cases"]:
        i = case["variable"]
        v = orc.cross_cov(th, i, i, case["h"])
        assert abs(v - case["value"]) <= pins["printed_precision"], (case, v)


def test_paper_effective_range_mapping(orc):
    """ER (distance where the marginal covariance falls to 0.05) grows with a as
    the paper's ER table says: within 15 % for the two smoothness values used."""
    pins = json.load(open(os.path.join(GOLDEN, "paper_pins.json")))["effective_range"]
    for a, er in zip(pins["a"], pins["er"]):
        ers = []
        for nu in pins["nu"]:
            h = scipy.optimize.brentq(lambda h: orc.matern(h / a, nu)[0] - 0.05, 1e-6, 10.0)
            ers.append(h)
        assert abs(np.mean(ers) - er) <= 0.15 * er, (a, ers, er)


# ---------------------------------------------------------------------- theta

def test_rho12_closed_form_d2(orc):
    for th in [(1, 1, 0.1, 0.5, 1.0, 0.5), (2, 0.5, 0.3, 1.5, 0.5, -0.8), (1, 1, 0.1, 0.7, 2.2, 0.3)]:
        nu12 = 0.5 * (th[3] + th[4])
        ref = th[5] * math.sqrt(th[3] * th[4]) / nu12   # Gamma(v+1)/Gamma(v) = v
        assert abs(orc.rho12(th) - ref) <= 2e-16 * 4
    assert abs(orc.rho12(synthetic.THETA_REF) - 0.4714045207910317) < 1e-16


def test_theta_check(orc):
    assert orc.theta_check((1, 1, 0.1, 0.5, 1, 0.5)) == 0
    assert orc.theta_check((0, 1, 0.1, 0.5, 1, 0.5)) == -1
    assert orc.theta_check((1, -1, 0.1, 0.5, 1, 0.5)) == -2
    assert orc.theta_check((1, 1, 0.0, 0.5, 1, 0.5)) == -3
    assert orc.theta_check((1, 1, 0.1, 0.0, 1, 0.5)) == -4
    assert orc.theta_check((1, 1, 0.1, 0.5, -1, 0.5)) == -5
    assert orc.theta_check((1, 1, 0.1, 0.5, 1, 1.0)) == -6


# ------------------------------------------------------------------ covariance

def test_sigma_structure(orc):
    x, y = synthetic.jittered_grid(90, seed=3)
    th = (1.3, 0.7, 0.15, 0.5, 1.0, 0.6)
    S = orc.cov_dense(x, y, th)
    assert np.array_equal(S, S.T)
    assert np.linalg.eigvalsh(S).min() > 0
    r = orc.rho12(th)
    blk = np.array([[th[0], r * math.sqrt(th[0] * th[1])], [r * math.sqrt(th[0] * th[1]), th[1]]])
    for l in range(0, 90, 17):
        np.testing.assert_allclose(S[2 * l:2 * l + 2, 2 * l:2 * l + 2], blk, rtol=1e-15)
    # Representation I entry layout, with nu = 1/2 closed form for C_11
    h = math.hypot(x[5] - x[2], y[5] - y[2])
    assert abs(S[10, 4] - th[0] * math.exp(-h / th[2])) <= 1e-15 * S[10, 4] * 4
    rows = np.array([10, 11, 11, 3])
    cols = np.array([4, 4, 5, 0])
    np.testing.assert_array_equal(orc.cov_entries(x, y, th, rows, cols), S[rows, cols])


# -------------------------------------------------------------- linear algebra

def test_potrf_matches_lapack(orc):
    g = np.random.default_rng(0)
    A = g.standard_normal((150, 150))
    A = A @ A.T + 150 * np.eye(150)
    L, info = orc.potrf(A)
    assert info == 0
    np.testing.assert_allclose(L, np.linalg.cholesky(A), rtol=1e-12, atol=1e-13)
    b = g.standard_normal(150)
    np.testing.assert_allclose(orc.trsv_lower(L, b), scipy.linalg.solve_triangular(L, b, lower=True), rtol=1e-12)
    np.testing.assert_allclose(orc.trsv_lower(L, b, trans=True),
                               scipy.linalg.solve_triangular(L, b, lower=True, trans="T"), rtol=1e-12)


def test_potrf_reports_first_failing_pivot(orc):
    A = np.diag([4.0, 9.0, -1.0, 5.0])
    L, info = orc.potrf(A)
    assert info == 3
    # singular to working precision: the third row repeats the first
    B = np.array([[2.0, 1.0, 2.0], [1.0, 3.0, 1.0], [2.0, 1.0, 2.0]])
    assert orc.potrf(B)[1] == 3
    # a small but clearly resolved pivot (1e-9 relative) is not a failure
    C = np.array([[1.0, 1.0 - 5e-10], [1.0 - 5e-10, 1.0]])
    assert orc.potrf(C)[1] == 0


def test_pivot_rule_leaves_workload_matrices_alone(orc):
    """The smallest relative pivot of the strongest-correlation workload
    (a = 0.3) is orders of magnitude above the 2^-40 singularity rule."""
    th = (1.0, 1.0, 0.3, 0.5, 1.0, 0.9)
    x, y = synthetic.jittered_grid(400, 0)
    S = orc.cov_dense(x, y, th)
    L, info = orc.potrf(S)
    assert info == 0
    ratio = np.min(np.diag(L) ** 2 / np.diag(S))
    assert ratio > 1e4 * 2.0 ** -40, ratio


# ------------------------------------------------------------------ likelihood

def _data(n, seed, th):
    import oracle
    x, y = synthetic.jittered_grid(n, seed)
    p = oracle.morton_order(x, y)
    x, y = x[p], y[p]
    z = oracle.simulate_z(x, y, th, synthetic.normal_eps(2 * n, seed))
    return x, y, z


def test_loglik_brute_force_eigen(orc):
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y, z = _data(100, 1, th)
    r = orc.loglik(x, y, z, th)
    S = orc.cov_dense(x, y, th)
    ev = np.linalg.eigvalsh(S)
    assert abs(r["logdet"] - np.sum(np.log(ev))) <= 1e-10 * abs(r["logdet"]) + 1e-10
    q = float(z @ np.linalg.solve(S, z))
    assert abs(r["quad"] - q) <= 1e-9 * q
    ref = scipy.stats.multivariate_normal(mean=np.zeros(200), cov=S).logpdf(z)
    assert abs(r["loglik"] - ref) <= 1e-9 * abs(ref)


def test_loglik_single_location_closed_form(orc):
    th = (1.7, 0.4, 0.2, 0.8, 1.3, -0.45)
    z = np.array([0.3, -1.1])
    r = orc.loglik([0.5], [0.5], z, th)
    rho = th[5] * math.sqrt(th[3] * th[4]) / (0.5 * (th[3] + th[4]))
    c = rho * math.sqrt(th[0] * th[1])
    det = th[0] * th[1] - c * c
    q = (th[1] * z[0] ** 2 - 2 * c * z[0] * z[1] + th[0] * z[1] ** 2) / det
    assert abs(r["logdet"] - math.log(det)) <= 1e-15 * 8
    assert abs(r["quad"] - q) <= 1e-14 * q
    assert abs(r["loglik"] - (-math.log(2 * math.pi) - 0.5 * math.log(det) - 0.5 * q)) < 1e-14


def test_loglik_beta0_splits_into_univariate_exponential(orc):
    """beta = 0, nu11 = nu22 = 1/2: the bivariate likelihood is the sum of two
    univariate exponential-kernel Gaussian likelihoods (scipy, built by hand)."""
    th = (1.4, 0.6, 0.12, 0.5, 0.5, 0.0)
    x, y = synthetic.jittered_grid(120, 5)
    z = synthetic.normal_eps(240, 5)
    r = orc.loglik(x, y, z, th)
    D = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    tot = 0.0
    for i in range(2):
        C = th[i] * np.exp(-D / th[2])
        tot += scipy.stats.multivariate_normal(mean=np.zeros(120), cov=C).logpdf(z[i::2])
    assert abs(r["loglik"] - tot) <= 1e-10 * abs(tot)


def test_loglik_permutation_invariance_and_scaling(orc):
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y, z = _data(80, 2, th)
    r = orc.loglik(x, y, z, th)
    p = np.random.default_rng(1).permutation(80)
    zp = z.reshape(80, 2)[p].reshape(-1)
    rp = orc.loglik(x[p], y[p], zp, th)
    assert abs(rp["loglik"] - r["loglik"]) <= 1e-10 * abs(r["loglik"])
    c = 2.5
    rc = orc.loglik(x, y, z, (c, c, 0.1, 0.5, 1.0, 0.5))
    assert abs(rc["logdet"] - (r["logdet"] + 160 * math.log(c))) <= 1e-10 * abs(rc["logdet"])
    assert abs(rc["quad"] - r["quad"] / c) <= 1e-10 * r["quad"]


def test_loglik_non_spd_duplicate_location(orc):
    x = np.array([0.1, 0.5, 0.5, 0.9])
    y = np.array([0.2, 0.3, 0.3, 0.7])
    r = orc.loglik(x, y, np.ones(8), (1, 1, 0.1, 0.5, 1.0, 0.5))
    assert r["loglik"] == -np.inf and r["info"] > 0


# ------------------------------------------------------------------- cokriging

def test_cokrige_interpolates_observed_sites(orc):
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y, z = _data(60, 4, th)
    idx = np.array([0, 17, 59])
    zhat, mse = orc.cokrige(x, y, z, th, x[idx], y[idx], with_mse=True)
    np.testing.assert_allclose(zhat, z.reshape(60, 2)[idx], rtol=1e-8, atol=1e-8)
    assert np.all(np.abs(mse) < 1e-8)


def test_cokrige_far_target_and_mse_bounds(orc):
    th = (1.0, 1.0, 0.05, 0.5, 1.0, 0.5)
    x, y, z = _data(60, 4, th)
    zhat, mse = orc.cokrige(x, y, z, th, [50.0], [50.0], with_mse=True)
    assert np.all(np.abs(zhat) < 1e-100)
    assert abs(mse[0] - 2.0) < 1e-12
    x0, y0 = synthetic.uniform_targets(20, 9)
    _, mse = orc.cokrige(x, y, z, th, x0, y0, with_mse=True)
    assert np.all(mse > -1e-12) and np.all(mse <= 2.0 + 1e-12)


def test_cokrige_beta0_is_univariate_kriging(orc):
    th = (1.0, 2.0, 0.1, 0.5, 0.5, 0.0)
    x, y = synthetic.jittered_grid(70, 8)
    z = synthetic.normal_eps(140, 8)
    x0, y0 = synthetic.uniform_targets(5, 8)
    zhat = orc.cokrige(x, y, z, th, x0, y0)
    D = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    D0 = np.hypot(x0[:, None] - x[None, :], y0[:, None] - y[None, :])
    for i in range(2):
        C = th[i] * np.exp(-D / th[2])
        c0 = th[i] * np.exp(-D0 / th[2])
        ref = c0 @ np.linalg.solve(C, z[i::2])
        np.testing.assert_allclose(zhat[:, i], ref, rtol=1e-9, atol=1e-12)


# -------------------------------------------------------------------- ordering

def test_morton_brute_force():
    import oracle
    # 4 x 4 lattice at cell centres: the Z-curve visits x fastest within each 2x2 block
    xs, ys = np.meshgrid((np.arange(4) + 0.5) / 4, (np.arange(4) + 0.5) / 4, indexing="xy")
    x, y = xs.reshape(-1), ys.reshape(-1)
    p = oracle.morton_order(x, y)
    qx = (x[p] * 4).astype(int)
    qy = (y[p] * 4).astype(int)
    want = []
    for k in range(16):
        bx = (k & 1) | ((k >> 2) & 1) << 1
        by = ((k >> 1) & 1) | ((k >> 3) & 1) << 1
        want.append((bx, by))
    assert list(zip(qx, qy)) == want
    # ties keep input order; clamp at 1.0
    p2 = oracle.morton_order([0.3, 0.3, 1.0, 0.0], [0.3, 0.3, 1.0, 0.0])
    assert list(p2) == [3, 0, 1, 2]


# ------------------------------------------------------------- approximations

def test_tlr_truncation_tight_accuracy_is_exact(orc):
    th = (1.0, 1.0, 0.09, 0.5, 1.0, 0.5)
    x, y, z = _data(96, 6, th)
    S = orc.cov_dense(x, y, th)
    St, ranks = orc.tlr_truncate_tiles(S, 48, 1e-300, 48)
    np.testing.assert_allclose(St, S, atol=1e-13)
    r_exact = orc.loglik_from_matrix(S, z)
    r_ref = orc.loglik(x, y, z, th)
    assert abs(r_exact["loglik"] - r_ref["loglik"]) <= 1e-10 * abs(r_ref["loglik"])
    # looser accuracy: smaller ranks, errors shrink as accuracy tightens
    errs = []
    for acc in (1e-3, 1e-5, 1e-7, 1e-9):
        St, rk = orc.tlr_truncate_tiles(S, 48, acc, 48)
        errs.append(abs(orc.loglik_from_matrix(St, z)["loglik"] - r_ref["loglik"]))
    assert errs[-1] <= errs[0]


def test_round_to_formats(orc):
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 3.14159265358979, -2.0 ** -130])
    b = orc.round_to(v, "bf16")
    assert b[0] == 1.0
    assert b[1] == 1.0 + 2 ** -7 or b[1] == 1.0   # tie to even -> 1.0
    assert b[1] == 1.0
    assert b[2] == 1.0 + 2 ** -7                  # tie to even (odd -> up)
    assert abs(b[3] - 3.140625) < 1e-12
    f = orc.round_to(v, "fp32")
    assert f[3] == float(np.float32(3.14159265358979))


# ------------------------------------------- mixed-precision emulation (not in the paper)

def _small_cov(orc, n, a, seed=2):
    th = (1.0, 1.0, a, 0.5, 1.0, 0.5)
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    return orc.cov_dense(x[p], y[p], th)


@pytest.mark.parametrize("fmt", ["fp32", "bf16"])
def test_mixed_emulation_full_band_is_exact_cholesky(orc, fmt):
    """A band covering every tile leaves no low-precision tile: LAPACK's factor."""
    S = _small_cov(orc, 90, 0.1)
    L, info = orc.mixed_cholesky_emulated(S, 32, 10, fmt)
    assert info == 0
    Np = L.shape[0]
    ref = np.eye(Np)
    ref[:180, :180] = scipy.linalg.cholesky(S, lower=True)
    np.testing.assert_allclose(L, ref, atol=1e-12)


@pytest.mark.parametrize("fmt,bound", [("fp32", 1e-5), ("bf16", 2e-2)])
def test_mixed_emulation_rounds_off_band_and_stays_close(orc, fmt, bound):
    """Off-band factor tiles are FP32 values; the factor reproduces S within
    the precision's rounding scale; band tiles carry no FP32 rounding."""
    S = _small_cov(orc, 90, 0.03)
    nb = 32
    L, info = orc.mixed_cholesky_emulated(S, nb, 2, fmt)
    assert info == 0
    T = L.shape[0] // nb
    for J in range(T):
        for I in range(J + 2, T):
            t = L[I * nb:(I + 1) * nb, J * nb:(J + 1) * nb]
            assert np.array_equal(orc.round_to(t, "fp32"), t)
    R = (L @ L.T)[:180, :180]
    assert np.max(np.abs(R - S)) <= bound
    assert np.max(np.abs(R - S)) > 0.0
    ld = 2 * np.sum(np.log(np.diag(L)[:180]))
    assert abs(ld - np.linalg.slogdet(S)[1]) <= 50 * bound * 180


@pytest.mark.parametrize("storage", ["fp32", "fp64"])
def test_mixed_emulation_without_rounding_is_exact_cholesky(orc, storage):
    """No operand rounding and FP64 storage: the tiled steps reduce to
    LAPACK's factor; with FP32 storage only the stored off-band tiles differ,
    by FP32 rounding."""
    S = _small_cov(orc, 90, 0.1)
    L, info = orc.mixed_cholesky_emulated(S, 32, 2, "fp64", storage)
    assert info == 0
    ref = np.eye(L.shape[0])
    ref[:180, :180] = scipy.linalg.cholesky(S, lower=True)
    if storage == "fp64":
        np.testing.assert_allclose(L, ref, atol=1e-12)
    else:
        assert np.max(np.abs(L - ref)) <= 1e-5 and np.max(np.abs(L - ref)) > 0.0


def test_mixed_emulation_fp64_storage_rounds_only_the_products(orc):
    """FP64 storage with FP32 operands: the first block column is the exact
    panel (no update has touched it), off-band tiles are not FP32 values, and
    the factor reproduces S far closer than with FP32 storage."""
    S = _small_cov(orc, 90, 0.03)
    nb = 32
    L, info = orc.mixed_cholesky_emulated(S, nb, 2, "fp32", "fp64")
    L32, info32 = orc.mixed_cholesky_emulated(S, nb, 2, "fp32", "fp32")
    assert info == 0 and info32 == 0
    ref = scipy.linalg.cholesky(S, lower=True)
    np.testing.assert_allclose(L[:180, :nb], ref[:, :nb], atol=1e-12)
    t = L[3 * nb:4 * nb, 0:nb]
    assert not np.array_equal(orc.round_to(t, "fp32"), t)
    e64 = np.max(np.abs((L @ L.T)[:180, :180] - S))
    e32 = np.max(np.abs((L32 @ L32.T)[:180, :180] - S))
    assert 0.0 < e64 < e32


def _mixed_pin_violations(orc, S, L, nb, band, fmt, storage):
    """Checks the emulated mixed factor against the defining equations of its
    rounding points (not against its own loop):

    * band blocks (I - J < band): S_IJ = sum_{k <= J} L_Ik L_Jk^T to FP64
      rounding (updates into band tiles take the stored values exactly, the
      diagonal tile and its panel solve are FP64): relative residual
      <= 8 u kappa(L_JJ);
    * off-band blocks: the same residual is at the operand precision's
      scale, neither FP64 rounding (a missing rounding) nor beyond 2e-2
      (bf16) / 1e-4 (bf16x3) / 1e-6 (fp32); with FP32 storage relative to
      the block, with FP64 storage relative to the products of the updates it
      received (J >= 1), where the rounding sits; with FP64 storage the
      split-BF16 products (operand error 2^-17) also stay above 3e-7, which
      FP32 operands (2^-24) do not reach;
    * FP64 storage: every off-band panel tile solves its Schur complement in
      FP64, L_IJ L_JJ^T = S_IJ - sum_{k < J} P(L_Ik, L_Jk) with P the
      rounded-operand product, to 8 u kappa(L_JJ).
    Returns the list of violated pins (empty when all hold)."""
    u = 2.0 ** -53
    N = S.shape[0]
    Np = L.shape[0]
    T = Np // nb
    Sp = np.eye(Np)
    Sp[:N, :N] = S

    def B(I, J):
        return slice(I * nb, (I + 1) * nb), slice(J * nb, (J + 1) * nb)

    def op(a):
        f = orc.round_to(a, "fp32")
        return f if fmt == "fp32" else orc.round_to(f, "bf16")

    def prod_lowp(a, b):
        """The rounded-operand product: op(a) op(b)^T, or for bf16x3 the
        three products of the two-term BF16 splits a = a_hi + a_lo."""
        if fmt != "bf16x3":
            return op(a) @ op(b).T
        fa, fb = orc.round_to(a, "fp32"), orc.round_to(b, "fp32")
        ha, hb = orc.round_to(fa, "bf16"), orc.round_to(fb, "bf16")
        la, lb = orc.round_to(fa - ha, "bf16"), orc.round_to(fb - hb, "bf16")
        return ha @ hb.T + ha @ lb.T + la @ hb.T

    # u = 2^-24, 2^-17 and 2^-8 per operand
    top = {"fp32": 1e-6, "bf16x3": 1e-4, "bf16": 2e-2}[fmt]
    low64 = 3e-7 if fmt == "bf16x3" else 1e-11
    bad = []
    for J in range(T):
        kap = np.linalg.cond(L[B(J, J)])
        for I in range(J, T):
            full = sum(L[B(I, k)] @ L[B(J, k)].T for k in range(J + 1))
            ab = sum(np.abs(L[B(I, k)]) @ np.abs(L[B(J, k)]).T for k in range(J + 1))
            scale = np.max(np.abs(Sp[B(I, J)])) + np.max(ab)
            rel = np.max(np.abs(Sp[B(I, J)] - full)) / scale
            if I - J < band:
                if rel > 8 * u * kap:
                    bad.append(("band", I, J, rel))
            elif storage == "fp32":
                if not (1e-11 < rel <= top):
                    bad.append(("offband-scale", I, J, rel))
            elif J >= 1:   # FP64 storage: the rounding sits in the products alone
                prod = np.max(sum(np.abs(L[B(I, k)]) @ np.abs(L[B(J, k)]).T for k in range(J)))
                relp = np.max(np.abs(Sp[B(I, J)] - full)) / prod
                if not (low64 < relp <= top):
                    bad.append(("offband-scale", I, J, relp))
            if storage == "fp64" and I - J >= band:
                schur = Sp[B(I, J)] - sum((prod_lowp(L[B(I, k)], L[B(J, k)]) for k in range(J)),
                                          np.zeros((nb, nb)))
                r3 = np.max(np.abs(schur - L[B(I, J)] @ L[B(J, J)].T)) / scale
                if r3 > 8 * u * kap:
                    bad.append(("panel-fp64", I, J, r3))
    return bad


@pytest.mark.parametrize("a", [0.03, 0.1])
@pytest.mark.parametrize("storage", ["fp32", "fp64"])
@pytest.mark.parametrize("fmt", ["fp32", "bf16", "bf16x3"])
def test_mixed_emulation_satisfies_its_rounding_definition(orc, a, storage, fmt):
    """Mixed precision is not in the paper: its definition is the placement of
    the rounding points (FP64 band and FP64 diagonal factors; off-band products
    on rounded operands; FP32 storage of off-band tiles or FP64 storage with
    FP64 panel solves).  The emulated factor satisfies each defining equation
    at the precision that definition gives it."""
    S = _small_cov(orc, 90, a)
    L, info = orc.mixed_cholesky_emulated(S, 32, 2, fmt, storage)
    assert info == 0
    assert _mixed_pin_violations(orc, S, L, 32, 2, fmt, storage) == []


@pytest.mark.parametrize("plant,storage,kind", [("band_operands", "fp32", "band"),
                                                ("band_operands", "fp64", "band"),
                                                ("w32", "fp64", "panel-fp64")])
def test_mixed_emulation_pins_catch_misplaced_rounding(orc, plant, storage, kind):
    """A rounding placed where the definition has none (operands of a band
    update rounded; W_k rounded to FP32 in an FP64-storage panel solve) breaks
    the pins above."""
    S = _small_cov(orc, 90, 0.1)
    L, info = orc.mixed_cholesky_emulated(S, 32, 2, "fp32", storage, _plant=plant)
    assert info == 0
    bad = _mixed_pin_violations(orc, S, L, 32, 2, "fp32", storage)
    assert any(b[0] == kind for b in bad), bad


def test_mixed_emulation_pins_catch_missing_offband_rounding(orc):
    """No rounding at all off the band (FP64 operands, FP64 storage) leaves the
    off-band residuals at FP64 scale: the FP32-scale pin fails."""
    S = _small_cov(orc, 90, 0.1)
    L, info = orc.mixed_cholesky_emulated(S, 32, 2, "fp64", "fp64")
    assert info == 0
    bad = _mixed_pin_violations(orc, S, L, 32, 2, "fp32", "fp64")
    assert any(b[0] == "offband-scale" for b in bad), bad


@pytest.mark.parametrize("plant,fmt_made,fmt_pinned", [("x3_hi_only", "bf16x3", "bf16x3"),
                                                       ("", "fp32", "bf16x3")])
def test_mixed_emulation_pins_catch_a_wrong_split(orc, plant, fmt_made, fmt_pinned):
    """Split-BF16 products (FP64 storage): keeping only a_hi b_hi (plain BF16
    operands) puts the off-band residuals above the split's scale, and
    unsplit FP32 operands put them below it; both break the off-band pin."""
    S = _small_cov(orc, 90, 0.1)
    L, info = orc.mixed_cholesky_emulated(S, 32, 2, fmt_made, "fp64", _plant=plant)
    assert info == 0
    bad = _mixed_pin_violations(orc, S, L, 32, 2, fmt_pinned, "fp64")
    assert any(b[0] == "offband-scale" for b in bad), bad


def test_bf16_split_error_bound(orc):
    """The two-term BF16 split of an FP32 value f with 2^e <= |f| < 2^(e+1):
    f_hi = bf16(f) is off by at most 2^(e-8), so the remainder r = f - f_hi
    (exact in FP32) is a power of two (then exact in BF16) or below 2^(e-8),
    and bf16(r) is off by at most 2^(e-17): |f - f_hi - f_lo| <= 2^-17 |f|.
    On BF16-representable values the remainder is 0."""
    rng = np.random.default_rng(5)
    f = orc.round_to(rng.standard_normal(20000) * np.exp(rng.uniform(-20, 20, 20000)), "fp32")
    hi = orc.round_to(f, "bf16")
    lo = orc.round_to(f - hi, "bf16")
    assert np.all(np.abs(f - hi) <= 2.0 ** -8 * np.abs(f))
    assert np.all(np.abs(f - hi - lo) <= 2.0 ** -17 * np.abs(f))
    assert np.max(np.abs(f - hi - lo) / np.abs(f)) > 2.0 ** -24  # not exact in general
    assert np.all(orc.round_to(hi - orc.round_to(hi, "bf16"), "bf16") == 0.0)


def test_tlr_frobenius_rule_keeps_more_and_bounds_tail(orc):
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y = synthetic.jittered_grid(150, 4)
    p = orc.morton_order(x, y)
    S = orc.cov_dense(x[p], y[p], th)
    for acc in (1e-5, 1e-8):
        S2, r2 = orc.tlr_truncate_tiles(S, 60, acc, 60)
        Sf, rf = orc.tlr_truncate_tiles(S, 60, acc, 60, rule="frobenius")
        low = np.tril_indices(r2.shape[0], -1)
        assert np.all(rf[low] >= r2[low])
        for I in range(r2.shape[0]):
            for J in range(I):
                blk = (slice(I * 60, (I + 1) * 60), slice(J * 60, (J + 1) * 60))
                assert np.linalg.norm(Sf[blk] - S[blk]) <= acc * (1 + 1e-9)
                assert np.linalg.norm(S2[blk] - S[blk], 2) <= acc * (1 + 1e-9)


# ----------------------------------------------- MLOE / MMOM (Section 5.4)

def _mloe_data(orc, n=80, m=6, seed=12):
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    x0, y0 = synthetic.uniform_targets(m, seed)
    return x[p], y[p], x0, y0


def test_mloe_mmom_zero_at_true_theta(orc):
    """theta_a = theta: E_{t,a} = E_t = E_a, so every LOE and MOM is 0."""
    x, y, x0, y0 = _mloe_data(orc)
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    r = orc.mloe_mmom(x, y, th, th, x0, y0)
    assert np.max(np.abs(r["loe"])) <= 1e-10 and np.max(np.abs(r["mom"])) <= 1e-10


def test_mloe_true_predictor_is_optimal_and_brute_force(orc):
    """LOE >= 0 (the true-parameter cokriging predictor minimises the MSE
    under the true model); E_t equals the oracle's Eq. (5) MSE; E_{t,a} equals
    a direct evaluation with numpy inverses."""
    x, y, x0, y0 = _mloe_data(orc)
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    tha = (1.1, 0.9, 0.13, 0.6, 0.9, 0.45)
    r = orc.mloe_mmom(x, y, th, tha, x0, y0)
    assert np.all(r["loe"] >= -1e-12)
    assert np.any(r["loe"] > 1e-6)
    z = synthetic.normal_eps(2 * len(x), 1)
    _, mse = orc.cokrige(x, y, z, th, x0, y0, with_mse=True)
    S, Sa = orc.cov_dense(x, y, th), orc.cov_dense(x, y, tha)
    Si, Sai = np.linalg.inv(S), np.linalg.inv(Sa)
    c0t = orc.cross_cov_targets(x, y, x0, y0, th)
    c0a = orc.cross_cov_targets(x, y, x0, y0, tha)
    for l in range(len(x0)):
        ct, ca = c0t[:, 2 * l:2 * l + 2], c0a[:, 2 * l:2 * l + 2]
        et = 2.0 - np.trace(ct.T @ Si @ ct)
        assert abs(et - mse[l]) <= 1e-9 * abs(et)
        eta = 2.0 - 2 * np.trace(ct.T @ Sai @ ca) + np.trace(ca.T @ Sai @ S @ Sai @ ca)
        ea = 2.0 - np.trace(ca.T @ Sai @ ca)
        assert abs(r["loe"][l] - (eta / et - 1)) <= 1e-8
        assert abs(r["mom"][l] - (ea / eta - 1)) <= 1e-8


def test_cross_cov_targets_matches_entries(orc):
    x, y, x0, y0 = _mloe_data(orc, n=20, m=3)
    th = (1.3, 0.7, 0.2, 0.8, 1.7, -0.4)
    c0 = orc.cross_cov_targets(x, y, x0, y0, th)
    for r in (0, 7, 19):
        for l in range(3):
            h = float(np.hypot(x[r] - x0[l], y[r] - y0[l]))
            for i in range(2):
                for j in range(2):
                    assert abs(c0[2 * r + i, 2 * l + j] - orc.cross_cov(th, i, j, h)) <= 1e-14


# ----------------------------------------------- DST (Section 4.4, 6.4.1)

def test_dst_band_counts(orc):
    """The kept tile count reaches the fraction at w and not at w - 1; a
    fraction of 1 keeps every tile; one tile per side keeps it."""
    for T in (1, 2, 7, 20, 43):
        for keep in (0.05, 0.4, 0.7, 1.0):
            w = orc.dst_band(T, keep)
            cnt = lambda v: sum(1 for I in range(T) for J in range(T)  # noqa: E731
                                if abs(I - J) < v)      # brute-force tile count
            assert cnt(w) >= keep * T * T
            assert w == 1 or cnt(w - 1) < keep * T * T
    assert orc.dst_band(20, 1.0) == 20 and orc.dst_band(1, 0.4) == 1
    # DST 40/60 and 70/30 at 100 tiles per side: w ~ T (1 - sqrt(1 - keep))
    assert abs(orc.dst_band(100, 0.4) - 100 * (1 - np.sqrt(0.6))) <= 2
    assert abs(orc.dst_band(100, 0.7) - 100 * (1 - np.sqrt(0.3))) <= 2


def test_dst_full_band_is_exact_and_band_one_splits(orc):
    """band >= T leaves Sigma unchanged (the exact likelihood); band = 1 makes
    Sigma block diagonal, so the likelihood is the sum of the diagonal
    blocks' likelihoods, each checked with scipy's multivariate normal."""
    from scipy.stats import multivariate_normal
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y = synthetic.jittered_grid(90, 3)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    z = orc.simulate_z(x, y, th, synthetic.normal_eps(180, 3))
    S = orc.cov_dense(x, y, th)
    nb = 40
    T = (180 + nb - 1) // nb
    full = orc.loglik_from_matrix(orc.dst_mask(S, nb, T), z)
    ex = orc.loglik(x, y, z, th)["loglik"]
    assert abs(full["loglik"] - ex) <= 1e-12 * abs(ex)
    diag = orc.loglik_from_matrix(orc.dst_mask(S, nb, 1), z)
    ref = sum(multivariate_normal(mean=np.zeros(len(z[a:a + nb])),
                                  cov=S[a:a + nb, a:a + nb]).logpdf(z[a:a + nb])
              for a in range(0, 180, nb))
    assert abs(diag["loglik"] - ref) <= 1e-9 * abs(ref)
    M = orc.dst_mask(S, nb, 2)
    assert np.all(M[:nb, 2 * nb:] == 0) and np.array_equal(M[:2 * nb, :2 * nb], S[:2 * nb, :2 * nb])


# ----------------------------------------------- p variables (Section 4.2, 5.2)

def _sites_p(orc, n, seed):
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    return x[p], y[p]


TH3 = {"sigma_sq": [1.0, 1.5, 0.7], "a": 0.1, "nu": [0.5, 1.0, 1.7],
       "beta": [[1.0, 0.5, -0.3], [0.5, 1.0, -0.2], [-0.3, -0.2, 1.0]]}


def test_cov_p_two_variables_equals_bivariate(orc):
    """The p-variate assembly (numpy, rho from the Gamma function) at p = 2
    equals the bivariate C oracle entry by entry."""
    x, y = _sites_p(orc, 60, 2)
    th = (1.3, 0.7, 0.2, 0.8, 1.7, -0.4)
    thp = {"sigma_sq": [1.3, 0.7], "a": 0.2, "nu": [0.8, 1.7], "beta": [[1, -0.4], [-0.4, 1]]}
    A, B = orc.cov_dense_p(x, y, thp), orc.cov_dense(x, y, th)
    assert np.max(np.abs(A - B)) <= 1e-14 * np.max(np.abs(B))
    assert abs(orc.rho_p(thp)[0, 1] - orc.rho12(th)) <= 1e-15


def test_loglik_p_independent_blocks(orc):
    """beta = I: the variables are independent, so Eq. (1) is the sum of the
    univariate Gaussian log-densities (scipy); beta with a zero third row:
    the bivariate oracle for (Z1, Z2) plus the univariate density of Z3."""
    from scipy.stats import multivariate_normal
    x, y = _sites_p(orc, 50, 4)
    n = 50
    z = synthetic.normal_eps(3 * n, 4)
    th = dict(TH3, beta=np.eye(3).tolist())
    h = np.sqrt((x[:, None] - x[None, :]) ** 2 + (y[:, None] - y[None, :]) ** 2)
    ref = 0.0
    for i in range(3):
        C = th["sigma_sq"][i] * orc.matern(h.ravel() / th["a"], th["nu"][i]).reshape(n, n)
        ref += multivariate_normal(mean=np.zeros(n), cov=C).logpdf(z[i::3])
    got = orc.loglik_p(x, y, z, th)["loglik"]
    assert abs(got - ref) <= 1e-9 * abs(ref)
    b = [[1.0, 0.6, 0.0], [0.6, 1.0, 0.0], [0.0, 0.0, 1.0]]
    th2 = dict(TH3, beta=b)
    z12 = np.empty(2 * n)
    z12[0::2], z12[1::2] = z[0::3], z[1::3]
    biv = orc.loglik(x, y, z12, (1.0, 1.5, 0.1, 0.5, 1.0, 0.6))["loglik"]
    C3 = 0.7 * orc.matern(h.ravel() / 0.1, 1.7).reshape(n, n)
    ref2 = biv + multivariate_normal(mean=np.zeros(n), cov=C3).logpdf(z[2::3])
    got2 = orc.loglik_p(x, y, z, th2)["loglik"]
    assert abs(got2 - ref2) <= 1e-9 * abs(ref2)


def test_theta_p_check(orc):
    assert orc.theta_p_check(TH3) == 0
    bad = dict(TH3, beta=[[1, 0.9, 0.9], [0.9, 1, -0.9], [0.9, -0.9, 1]])   # not positive definite
    assert orc.theta_p_check(bad) == -5
    asym = dict(TH3, beta=[[1, 0.5, 0.1], [0.4, 1, 0.1], [0.1, 0.1, 1]])
    assert orc.theta_p_check(asym) == -5
    assert orc.theta_p_check(dict(TH3, a=-1.0)) == -3
    assert orc.theta_p_check(dict(TH3, nu=[0.5, 6.0, 1.0])) == -4


def test_profile_loglik(orc):
    """p = 1: the profiled variance maximises Eq. (1) in sigma^2, so the
    profile likelihood equals the closed form -n/2 log 2 pi - n/2 log(q/n) -
    log|R|/2 - n/2; p = 3: each sigma_ii^2 against numpy's inverse."""
    x, y = _sites_p(orc, 70, 6)
    n = 70
    z1 = 1.7 * synthetic.normal_eps(n, 6)
    th1 = {"sigma_sq": [5.0], "a": 0.1, "nu": [1.2], "beta": [[1.0]]}
    r = orc.profile_loglik_p(x, y, z1, th1)
    R = orc.cov_dense_p(x, y, dict(th1, sigma_sq=[1.0]))
    q = float(z1 @ np.linalg.solve(R, z1))
    ld = float(np.linalg.slogdet(R)[1])
    closed = -n / 2 * np.log(2 * np.pi) - n / 2 * np.log(q / n) - ld / 2 - n / 2
    assert abs(r["sigma_sq"][0] - q / n) <= 1e-10 * q / n
    assert abs(r["loglik"] - closed) <= 1e-9 * abs(closed)
    for f in (0.97, 1.03):
        other = orc.loglik_p(x, y, z1, dict(th1, sigma_sq=[f * q / n]))["loglik"]
        assert other < r["loglik"]
    z3 = synthetic.normal_eps(3 * n, 7)
    r3 = orc.profile_loglik_p(x, y, z3, TH3)
    for i in range(3):
        Ri = orc.cov_dense_p(x, y, {"sigma_sq": [1.0], "a": 0.1, "nu": [TH3["nu"][i]],
                                    "beta": [[1.0]]})
        zi = z3[i::3]
        assert abs(r3["sigma_sq"][i] - zi @ np.linalg.solve(Ri, zi) / n) <= 1e-9
