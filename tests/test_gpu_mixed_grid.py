"""Mixed precision on the n = 50,000 workload (100,000 x 100,000), every cell
of its smoothness x colocated-correlation grid: nu11, nu22 in {0.5, 1.5},
beta in {0, 0.5, 0.9}, a = 0.1, Z = L eps drawn with the FP64 factor of
each cell's Sigma, FP64 band of 2 tiles, tile 1024.  Mixed precision is not
in the paper; its target is relative |delta loglik| <= 1e-6 against the FP64
result on the same inputs, at a higher likelihood-evaluation rate.

Each (cell, mode) asserts the outcome measured and recorded for it:

* "meets": status 0, |delta loglik| <= 1e-6, and faster than FP64 (the FP64
  time is the cell's own generation + Cholesky + solve);
* "not SPD": the mixed factor meets a non-positive pivot (FP64 succeeds), so
  the library evaluates the theta in FP64 instead (mvg_ir_stats says so, with
  no refinement sweep; the result is FP64's, the time that of both), reported
  as an expected failure;
* "FP64 fallback": the mixed factor exists but the FP64 refinement of the
  solve stops unconverged, so the library evaluates the theta in FP64
  instead (mvg_ir_stats says so; the result is FP64's, the time that of
  both), reported as an expected failure.

Modes: MVG_MIXED_FP32X (FP64 tiles and panel solves, FP32 operands in the
off-band GEMMs), MVG_MIXED_BF16X3 (the same with each off-band operand split
into two BF16 terms, three BF16 MFMAs per product), MVG_MIXED_FP32 (FP32
storage off the band), MVG_MIXED_BF16 (FP32 storage, BF16 operands)."""
import sys
import time

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

N_LOC = 50000
NUS = [(0.5, 0.5), (0.5, 1.5), (1.5, 0.5), (1.5, 1.5)]
BETAS = [0.0, 0.5, 0.9]
MEETS, NOT_SPD, FALLBACK = "meets", "not SPD", "FP64 fallback"

# recorded outcomes (n = 50,000, seed-1 sites, Z = L eps seed 1).  Plain BF16
# operands on the rough field keep the factor positive definite, but it is
# too far off for the refinement to converge (without the fall-back its
# log-determinant alone put the relative delta loglik at 2.5e-4 - 3.9e-4)
ROUGH = {0.0: {"fp32x": MEETS, "bf16x3": MEETS, "fp32": MEETS, "bf16": FALLBACK},
         0.5: {"fp32x": MEETS, "bf16x3": MEETS, "fp32": MEETS, "bf16": FALLBACK},
         0.9: {"fp32x": MEETS, "bf16x3": MEETS, "fp32": MEETS, "bf16": NOT_SPD}}
SMOOTH = {0.0: {"fp32x": FALLBACK, "bf16x3": NOT_SPD, "fp32": NOT_SPD, "bf16": NOT_SPD},
          0.5: {"fp32x": FALLBACK, "bf16x3": NOT_SPD, "fp32": NOT_SPD, "bf16": NOT_SPD},
          0.9: {"fp32x": NOT_SPD, "bf16x3": NOT_SPD, "fp32": NOT_SPD, "bf16": NOT_SPD}}


def expected(nu, beta, mode):
    return (ROUGH if nu == (0.5, 0.5) else SMOOTH)[beta][mode]


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


@pytest.fixture(scope="module")
def sites(lib, orc):
    x, y = synthetic.jittered_grid(N_LOC, 1)
    p = orc.morton_order(x, y)
    return _dev(x[p]), _dev(y[p])


_cells = {}


def _cell(lib, sites, nu, beta):
    """Z = L eps and the FP64 evaluation (timed) of one cell, cached."""
    import torch
    key = (nu, beta)
    if key not in _cells:
        X, Y = sites
        th = (1.0, 1.0, 0.1, nu[0], nu[1], beta)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        A = lib.cov_generate(X, Y, th, {"nb": 1024})
        assert lib.potrf_tiled(A) == 0
        z = lib.mvg_trmv(A, _dev(synthetic.normal_eps(2 * N_LOC, 1)))
        ref = lib.mvg_mat_loglik(A, z)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        del A
        _cells.clear()   # one cell resident at a time
        _cells[key] = (th, z, ref, t64)
    return _cells[key]


_warm = set()


@pytest.mark.parametrize("mode", ["fp32x", "bf16x3", "fp32", "bf16"])
@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("nu", NUS, ids=lambda nu: "nu%g,%g" % nu)
def test_mixed_grid_cell(lib, sites, nu, beta, mode):
    import torch
    X, Y = sites
    th, z, ref, t64 = _cell(lib, sites, nu, beta)
    prec = {"fp32x": lib.MVG_MIXED_FP32X, "bf16x3": lib.MVG_MIXED_BF16X3,
            "fp32": lib.MVG_MIXED_FP32, "bf16": lib.MVG_MIXED_BF16}[mode]
    o = {"nb": 1024, "precision": prec, "band_tiles": 2}
    if mode not in _warm:  # the first call of a precision sizes its arena
        lib.loglik(X, Y, z, th, o)
        _warm.add(mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = lib.loglik(X, Y, z, th, o)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = int(r["status"][0])
    irs = lib.mvg_ir_stats(0)
    fell_back = bool(irs["fp64_fallback"])
    exp = expected(nu, beta, mode)
    dl = abs(r["loglik"][0] - ref["loglik"]) / abs(ref["loglik"]) if st == 0 else None
    _say("  nu=%s beta=%g %-5s: status %d, rel dl %s, %.2f s (FP64 %.2f s), expected %s"
         % (nu, beta, mode, st, "%.2e" % dl if dl is not None else "-", dt, t64, exp))
    if exp == MEETS:
        assert st == 0 and dl <= 1e-6 and not fell_back
        assert dt < t64
        return
    if exp == FALLBACK:
        if st == 0 and not fell_back and dl <= 1e-6 and dt < t64:
            return   # better than recorded
        assert st == 0 and fell_back and dl <= 1e-9
        pytest.xfail("refinement unconverged: evaluated in FP64 (%.2f s)" % dt)
    if exp == NOT_SPD:
        if st == 0 and not fell_back and dl <= 1e-6 and dt < t64:
            return   # better than recorded
        assert st == 0 and fell_back and irs["iters"] == 0 and dl <= 1e-9
        pytest.xfail("not positive definite in this precision: evaluated in FP64 (%.2f s)" % dt)
    raise AssertionError("no recorded outcome for this cell: %r" % (exp,))
