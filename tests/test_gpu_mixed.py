"""GPU checks of the mixed-precision likelihood (FP64 band tiles, FP32 / BF16
off the band, FP64 iterative refinement of the solve) against the FP64 oracle
and the FP64 GPU path on the same seeded inputs.

Tolerances: relative |delta loglik| <= 1e-6 for FP32 off-band tiles (the
target for the mixed form) on the small workload's smoothness; the refined
quadratic form Z^T Sigma^-1 Z to 1e-9 relative (the refinement stops at
||r|| <= 1e-14 ||Z|| or when the residual stagnates at the FP64 floor); the
log-determinant of the mixed factor within 3x (FP32) or 10x (BF16) the error
that the oracle's FP64 emulation of the same rounding points predicts: that
emulation rounds each tile update once, the GPU sums 16 products per MFMA
stage in FP32 first.  BF16 operands are 2^8 times coarser than FP32: its
log-determinant error is held to the emulation's prediction, not to 1e-6."""
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


def _data(orc, n, seed, theta):
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    z = orc.simulate_z(x, y, theta, synthetic.normal_eps(2 * n, seed))
    return x, y, z


_CASES = {}


def _case(orc, n, seed, th, nb, band, fmt, storage="fp32"):
    """Oracle loglik and the emulated mixed log-determinant (cached per module)."""
    key = (n, seed, tuple(th), nb, band, fmt, storage)
    if key not in _CASES:
        x, y, z = _data(orc, n, seed, th)
        ref = orc.loglik(x, y, z, th)
        S = orc.cov_dense(x, y, th)
        L, info = orc.mixed_cholesky_emulated(S, nb, band, fmt, storage)
        eld = 2.0 * float(np.sum(np.log(np.diag(L)[:2 * n]))) if info == 0 else float("nan")
        _CASES[key] = (x, y, z, ref, eld, info)
    return _CASES[key]


def test_mixed_full_band_matches_fp64(lib, orc):
    """A band covering every tile: the mixed path factors exactly like FP64."""
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y, z = _data(orc, 700, 4, th)
    _say("mixed full band n=700 nb=128")
    d64 = lib.loglik(_dev(x), _dev(y), _dev(z), th, {"nb": 128})
    for prec in (lib.MVG_MIXED_FP32, lib.MVG_MIXED_BF16, lib.MVG_MIXED_FP32X,
                 lib.MVG_MIXED_BF16X3):
        got = lib.loglik(_dev(x), _dev(y), _dev(z), th,
                         {"nb": 128, "precision": prec, "band_tiles": 64})
        assert got["status"][0] == 0
        assert got["logdet"][0] == d64["logdet"][0]
        assert abs(got["quad"][0] - d64["quad"][0]) <= 1e-12 * abs(d64["quad"][0])
        st = lib.mvg_ir_stats(0)
        assert st["converged"], st


@pytest.mark.parametrize("nb", [128, 256])
@pytest.mark.parametrize("a", [0.03, 0.1, 0.3])
def test_mixed_fp32_loglik(lib, orc, a, nb):
    th = (1.0, 1.0, a, 0.5, 1.0, 0.5)
    n = 1000
    x, y, z, ref, eld, einfo = _case(orc, n, 1, th, nb, 2, "fp32")
    _say("mixed fp32 n=%d nb=%d a=%g" % (n, nb, a))
    got = lib.loglik(_dev(x), _dev(y), _dev(z), th,
                     {"nb": nb, "precision": lib.MVG_MIXED_FP32})
    assert einfo == 0 and got["status"][0] == 0
    st = lib.mvg_ir_stats(0)
    dl = abs(got["loglik"][0] - ref["loglik"]) / abs(ref["loglik"])
    dld = got["logdet"][0] - ref["logdet"]
    _say("  rel dloglik %.2e  dlogdet %.3e (emulated %.3e)  quad rel %.2e  IR %s"
         % (dl, dld, eld - ref["logdet"], abs(got["quad"][0] - ref["quad"]) / ref["quad"], st))
    assert st["converged"], st
    assert abs(got["quad"][0] - ref["quad"]) <= 1e-9 * abs(ref["quad"])
    if a <= 0.1:  # at a = 0.3 kappa * 2^-24 nears 1e-1: both errors are noise-dominated
        assert abs(dld) <= max(3.0 * abs(eld - ref["logdet"]), 1e-10 * abs(ref["logdet"]))
    assert dl <= 1e-6


@pytest.mark.parametrize("nb", [128, 256])
@pytest.mark.parametrize("a", [0.03, 0.1, 0.3])
def test_mixed_fp32x_loglik(lib, orc, a, nb):
    """FP64 tiles and panel solves, FP32 operands in the off-band trailing
    GEMMs: the log-determinant error against the oracle's emulation with FP64
    storage.  The emulation forms the products of FP32-rounded operands
    exactly; the GPU also rounds each 16-product stage sum to FP32, an error
    of the same order per product as the operand rounding but not in the
    emulation, so the bound is 50x the emulated size or 2e-9 relative
    (measured up to ~25x at a = 0.1).  At a = 0.3 both are noise-dominated
    (kappa 2^-24 nears 1e-1) and only the likelihood is held."""
    th = (1.0, 1.0, a, 0.5, 1.0, 0.5)
    n = 1000
    x, y, z, ref, eld, einfo = _case(orc, n, 1, th, nb, 2, "fp32", "fp64")
    _say("mixed fp32x n=%d nb=%d a=%g" % (n, nb, a))
    got = lib.loglik(_dev(x), _dev(y), _dev(z), th,
                     {"nb": nb, "precision": lib.MVG_MIXED_FP32X})
    assert einfo == 0 and got["status"][0] == 0
    st = lib.mvg_ir_stats(0)
    dl = abs(got["loglik"][0] - ref["loglik"]) / abs(ref["loglik"])
    dld = got["logdet"][0] - ref["logdet"]
    _say("  rel dloglik %.2e  dlogdet %.3e (emulated %.3e)  IR %s"
         % (dl, dld, eld - ref["logdet"], st))
    assert st["converged"], st
    assert abs(got["quad"][0] - ref["quad"]) <= 1e-9 * abs(ref["quad"])
    if a <= 0.1:
        assert abs(dld) <= max(50.0 * abs(eld - ref["logdet"]), 2e-9 * abs(ref["logdet"]))
        assert dl <= 1e-7
    assert dl <= 1e-6


@pytest.mark.parametrize("nb", [128, 256])
@pytest.mark.parametrize("a", [0.03, 0.1, 0.3])
def test_mixed_bf16x3_loglik(lib, orc, a, nb):
    """FP64 tiles and panel solves, off-band operands split into two BF16
    terms (three BF16 MFMAs per product, FP32 accumulation over the tile's
    K): the likelihood within 1e-6 of the oracle, the refined quadratic form
    to 1e-9, and the log-determinant error within 10x the oracle's emulation
    of the same split (which forms the three products exactly; the FP32
    accumulation adds about 2^-24 sqrt(K) per entry, below the split's
    2^-17) or 2e-9 relative.  At a = 0.3 (condition number ~1e7 at n = 1000)
    the split's rounding alone moves log|Sigma| by ~3e-3 in the emulation and
    the likelihood misses 1e-6 (2.5e-6 measured at nb 128): held to the
    regression bound 1e-5, then reported as an expected failure."""
    th = (1.0, 1.0, a, 0.5, 1.0, 0.5)
    n = 1000
    x, y, z, ref, eld, einfo = _case(orc, n, 1, th, nb, 2, "bf16x3", "fp64")
    _say("mixed bf16x3 n=%d nb=%d a=%g" % (n, nb, a))
    got = lib.loglik(_dev(x), _dev(y), _dev(z), th,
                     {"nb": nb, "precision": lib.MVG_MIXED_BF16X3})
    assert einfo == 0 and got["status"][0] == 0
    st = lib.mvg_ir_stats(0)
    dl = abs(got["loglik"][0] - ref["loglik"]) / abs(ref["loglik"])
    dld = got["logdet"][0] - ref["logdet"]
    _say("  rel dloglik %.2e  dlogdet %.3e (emulated %.3e)  IR %s"
         % (dl, dld, eld - ref["logdet"], st))
    assert st["converged"], st
    assert abs(got["quad"][0] - ref["quad"]) <= 1e-9 * abs(ref["quad"])
    if a <= 0.1:
        assert abs(dld) <= max(10.0 * abs(eld - ref["logdet"]), 2e-9 * abs(ref["logdet"]))
        assert dl <= 1e-6
        return
    assert dl <= 1e-5
    if dl > 1e-6:
        pytest.xfail("split-BF16 operands miss |delta loglik| <= 1e-6 at a = %g: %.2e" % (a, dl))


@pytest.mark.parametrize("a", [0.03, 0.1])
def test_mixed_bf16_loglik(lib, orc, a):
    """BF16 operands (FP32 storage) at n = 1000: the refined quadratic form
    matches the oracle and the log-determinant is within 10x the oracle's
    emulation of the same rounding points, but BF16 rounding (u = 2^-8) of
    the off-band operands misses the 1e-6 target on the likelihood: the
    regression bound 1e-4 is asserted, then the miss is reported as an
    expected failure."""
    th = (1.0, 1.0, a, 0.5, 1.0, 0.5)
    n, nb = 1000, 128
    x, y, z, ref, eld, einfo = _case(orc, n, 1, th, nb, 2, "bf16")
    _say("mixed bf16 n=%d nb=%d a=%g" % (n, nb, a))
    got = lib.loglik(_dev(x), _dev(y), _dev(z), th,
                     {"nb": nb, "precision": lib.MVG_MIXED_BF16})
    assert einfo == 0 and got["status"][0] == 0
    st = lib.mvg_ir_stats(0)
    dl = abs(got["loglik"][0] - ref["loglik"]) / abs(ref["loglik"])
    dld = got["logdet"][0] - ref["logdet"]
    _say("  rel dloglik %.2e  dlogdet %.3e (emulated %.3e)  IR %s"
         % (dl, dld, eld - ref["logdet"], st))
    assert st["converged"], st
    assert abs(got["quad"][0] - ref["quad"]) <= 1e-9 * abs(ref["quad"])
    assert abs(dld) <= 10.0 * abs(eld - ref["logdet"])
    assert dl <= 1e-4
    if dl > 1e-6:
        pytest.xfail("BF16 operands miss |delta loglik| <= 1e-6: %.2e" % dl)


@pytest.mark.parametrize("mode", ["fp32", "fp32x"])
def test_mixed_ragged_and_wide_band(lib, orc, mode):
    """Ragged last tile; bands of 2 and 3 tiles; smoother second variable and
    negative beta.  The condition number is ~4e7, so kappa 2^-24 > 1: FP32
    storage alone moves the log-determinant by ~1e-2 (emulated) and the
    error is dominated by the few smallest eigenvalues; held to 1e-5 (FP32X,
    FP64 storage, is held to the same bound)."""
    th = (1.5, 0.8, 0.15, 0.8, 1.7, -0.6)
    x, y, z = _data(orc, 1337, 21, th)
    ref = orc.loglik(x, y, z, th)
    S = orc.cov_dense(x, y, th)
    prec = lib.MVG_MIXED_FP32 if mode == "fp32" else lib.MVG_MIXED_FP32X
    storage = "fp32" if mode == "fp32" else "fp64"
    for band in (2, 3):
        L, info = orc.mixed_cholesky_emulated(S, 256, band, "fp32", storage)
        eld = 2.0 * float(np.sum(np.log(np.diag(L)[:2 * 1337])))
        got = lib.loglik(_dev(x), _dev(y), _dev(z), th,
                         {"nb": 256, "precision": prec, "band_tiles": band})
        dl = abs(got["loglik"][0] - ref["loglik"]) / abs(ref["loglik"])
        dld = got["logdet"][0] - ref["logdet"]
        _say("  band %d rel dloglik %.2e dlogdet %.3e (emulated %.3e)"
             % (band, dl, dld, eld - ref["logdet"]))
        assert got["status"][0] == 0 and info == 0
        assert abs(got["quad"][0] - ref["quad"]) <= 1e-9 * abs(ref["quad"])
        assert dl <= 1e-5


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_mixed_batch_equals_single_calls(lib, orc, mode):
    th0 = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y, z = _data(orc, 600, 8, th0)
    ths = synthetic.nelder_mead_simplex(th0)[:3]
    prec = lib.MVG_MIXED_FP32 if mode == "fp32" else lib.MVG_MIXED_BF16X3
    o = {"nb": 128, "precision": prec}
    batch = lib.loglik(_dev(x), _dev(y), _dev(z), ths, o)
    for i, t in enumerate(ths):
        one = lib.loglik(_dev(x), _dev(y), _dev(z), t, o)
        assert one["loglik"][0] == batch["loglik"][i]


@pytest.mark.parametrize("mode", ["fp32", "bf16x3"])
def test_mixed_factor_cokriging(lib, orc, mode):
    """Predictions from a resident mixed factor use the refined Sigma^-1 Z."""
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y, z = _data(orc, 800, 3, th)
    x0, y0 = synthetic.uniform_targets(40, 3)
    prec = lib.MVG_MIXED_FP32 if mode == "fp32" else lib.MVG_MIXED_BF16X3
    res, F = lib.loglik(_dev(x), _dev(y), _dev(z), th,
                        {"nb": 128, "precision": prec}, keep=True)
    assert F is not None
    zh = lib.cokrige_predict(F, _dev(x0), _dev(y0)).cpu().numpy()
    ref = orc.cokrige(x, y, z, th, x0, y0)
    rmse = float(np.sqrt(np.mean((zh - ref) ** 2)))
    _say("  cokriging rmse diff %.2e" % rmse)
    assert rmse <= 1e-9


def test_mixed_rejects_band_below_two(lib, orc):
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y = synthetic.jittered_grid(100, 0)
    z = synthetic.normal_eps(200, 0)
    with pytest.raises(lib.MvgError):
        lib.loglik(_dev(x), _dev(y), _dev(z), th,
                   {"nb": 128, "precision": lib.MVG_MIXED_FP32, "band_tiles": 1})


@pytest.mark.parametrize("prec,fmt,storage,atol", [(1, "fp32", "fp32", 1e-5), (2, "bf16", "fp32", 5e-3),
                                                   (6, "bf16x3", "fp64", 2e-5)])
def test_mixed_factor_matches_emulation(lib, orc, prec, fmt, storage, atol):
    """potrf_tiled on a mixed-layout matrix: the factor entry by entry against
    the oracle's emulation of the same rounding points (FP32 accumulation
    order differs, hence the tolerance); band tiles to FP64 accuracy where no
    low-precision tile feeds them (the first block column)."""
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    x, y = synthetic.jittered_grid(300, 6)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    A = lib.cov_generate(_dev(x), _dev(y), th, {"nb": 128, "precision": prec})
    assert lib.potrf_tiled(A, {"nb": 128, "precision": prec}) == 0
    Lg = A.to_dense().cpu().numpy()
    S = orc.cov_dense(x, y, th)
    Le, info = orc.mixed_cholesky_emulated(S, 128, 2, fmt, storage)
    assert info == 0
    Le = Le[:600, :600]
    err = np.max(np.abs(Lg - Le))
    _say("  %s factor max |gpu - emulated| %.2e" % (fmt, err))
    assert err <= atol
    assert np.max(np.abs(Lg[:, :128] - Le[:, :128])[:256]) <= 1e-12


def test_mixed_unconverged_refinement_falls_back_to_fp64(lib, orc):
    """A refinement that stops without meeting a criterion (here a budget of
    one sweep and an unreachable tolerance) must not return its unconverged
    quadratic form, nor a factor whose w is unconverged: loglik evaluates
    that theta in FP64 instead (the FP64 values bitwise, and the FP64 factor
    with keep), and mvg_ir_stats reports it."""
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    n, nb = 600, 128
    x, y, z = _data(orc, n, 1, th)
    X, Y, Z = _dev(x), _dev(y), _dev(z)
    f64 = lib.loglik(X, Y, Z, th, {"nb": nb})
    # BF16 operands: one sweep cannot reach the quadratic-form criterion either
    o = {"nb": nb, "precision": lib.MVG_MIXED_BF16, "ir_max_iter": 1, "ir_tol": 1e-300}
    got = lib.loglik(X, Y, Z, [th, th], o)
    st = [lib.mvg_ir_stats(i) for i in range(2)]
    assert all(s["fp64_fallback"] for s in st), st
    for key in ("loglik", "logdet", "quad"):
        assert got[key][0] == f64[key][0] and got[key][1] == f64[key][0], key
    # with keep only the residual criterion applies
    o = {"nb": nb, "precision": lib.MVG_MIXED_FP32, "ir_max_iter": 1, "ir_tol": 1e-300}
    res, F = lib.loglik(X, Y, Z, th, o, keep=True)
    assert lib.mvg_ir_stats(0)["fp64_fallback"]
    assert res["loglik"][0] == f64["loglik"][0]
    x0, y0 = synthetic.uniform_targets(7, 4)
    _, F64 = lib.loglik(X, Y, Z, th, {"nb": nb}, keep=True)
    a = lib.cokrige_predict(F, _dev(x0), _dev(y0)).cpu().numpy()
    b = lib.cokrige_predict(F64, _dev(x0), _dev(y0)).cpu().numpy()
    assert np.array_equal(a, b)


def test_mixed_lost_definiteness_falls_back_to_fp64(lib, orc):
    """A smooth, strongly correlated field (nu = 1.5 in both variables,
    a = 0.3; condition number about 5e7 at n = 600) is positive definite in
    FP64, but BF16 operands in the off-band updates drive the first tile they
    reach to a non-positive pivot (the emulation fails at pivot 385, the first
    row of tile 3): loglik evaluates that theta in FP64 instead (the FP64
    values bitwise, status 0, the FP64 factor with keep), and mvg_ir_stats
    reports the fall-back with no refinement sweep."""
    th = (1.0, 1.0, 0.3, 1.5, 1.5, 0.5)
    n, nb = 600, 128
    x, y, z = _data(orc, n, 1, th)
    S = orc.cov_dense(x, y, th)
    _, info = orc.mixed_cholesky_emulated(S, nb, 2, "bf16", "fp32")
    assert info > 0
    X, Y, Z = _dev(x), _dev(y), _dev(z)
    f64 = lib.loglik(X, Y, Z, th, {"nb": nb})
    assert f64["status"][0] == 0
    o = {"nb": nb, "precision": lib.MVG_MIXED_BF16, "band_tiles": 2}
    got = lib.loglik(X, Y, Z, [th, th], o)
    for i in range(2):
        s = lib.mvg_ir_stats(i)
        assert s["fp64_fallback"] and s["iters"] == 0 and np.isnan(s["relres"]), s
        assert got["status"][i] == 0
        for key in ("loglik", "logdet", "quad"):
            assert got[key][i] == f64[key][0], key
    res, F = lib.loglik(X, Y, Z, th, o, keep=True)
    assert lib.mvg_ir_stats(0)["fp64_fallback"] and F is not None
    assert res["loglik"][0] == f64["loglik"][0]
    _, F64 = lib.loglik(X, Y, Z, th, {"nb": nb}, keep=True)
    x0, y0 = synthetic.uniform_targets(7, 4)
    a = lib.cokrige_predict(F, _dev(x0), _dev(y0)).cpu().numpy()
    b = lib.cokrige_predict(F64, _dev(x0), _dev(y0)).cpu().numpy()
    assert np.array_equal(a, b)


def test_mixed_singular_sigma_reports_the_fp64_pivot(lib, orc):
    """A repeated location makes Sigma singular: the mixed factor fails, the
    FP64 evaluation fails too, and loglik reports FP64's pivot with
    loglik = -inf (no kept factor)."""
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    n, nb = 600, 128
    x, y, z = _data(orc, n, 1, th)
    x, y = x.copy(), y.copy()
    x[300], y[300] = x[299], y[299]
    X, Y, Z = _dev(x), _dev(y), _dev(z)
    f64 = lib.loglik(X, Y, Z, th, {"nb": nb})
    assert f64["status"][0] > 0
    for prec in (lib.MVG_MIXED_FP32, lib.MVG_MIXED_BF16X3):
        res, F = lib.loglik(X, Y, Z, th, {"nb": nb, "precision": prec, "band_tiles": 2},
                            keep=True)
        assert lib.mvg_ir_stats(0)["fp64_fallback"]
        assert res["status"][0] == f64["status"][0] and res["loglik"][0] == -np.inf
        assert F is None
