"""GPU checks of the maximum-likelihood driver (Nelder-Mead around Eq. (1)):
the estimate's likelihood against the oracle at the same theta, the maximum
property (the estimate beats the true theta and every coordinate step around
it), and agreement with scipy's Nelder-Mead run on the oracle's likelihood
from the same start in the same coordinates.  The two searches take
different paths (different rounding of the objective), so they are compared
on the maximum they reach: |delta loglik| <= 1e-3, theta within 5 %."""
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


def _u(th):
    s1, s2, a, n1, n2, b = th
    return np.array([np.log(s1), np.log(s2), np.log(a), -np.log(5 / n1 - 1), -np.log(5 / n2 - 1),
                     np.arctanh(b)])


def _th(u):
    return (np.exp(u[0]), np.exp(u[1]), np.exp(u[2]), 5 / (1 + np.exp(-u[3])),
            5 / (1 + np.exp(-u[4])), np.tanh(u[5]))


TRUE = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
START = (1.2, 0.8, 0.13, 0.6, 0.9, 0.3)


def test_mle_fit_matches_scipy_nelder_mead_on_oracle(lib, orc):
    from scipy.optimize import minimize
    n = 150
    x, y = synthetic.jittered_grid(n, 21)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    z = orc.simulate_z(x, y, TRUE, synthetic.normal_eps(2 * n, 21))
    _say("mle n=%d from %s" % (n, START))
    fit = lib.mle_fit(_dev(x), _dev(y), _dev(z), START, {"nb": 128}, max_evals=3000,
                      ftol=1e-8, xtol=1e-6)
    _say("  gpu: %s loglik %.8f evals %d converged %s" % (np.round(fit["theta"], 5),
                                                          fit["loglik"], fit["evals"],
                                                          fit["converged"]))
    assert fit["converged"]
    ref_at = orc.loglik(x, y, z, fit["theta"])["loglik"]
    assert abs(fit["loglik"] - ref_at) <= 1e-9 * abs(ref_at)
    assert ref_at >= orc.loglik(x, y, z, TRUE)["loglik"]
    u_hat = _u(fit["theta"])
    for j in range(6):
        for d in (-1e-2, 1e-2):
            u = u_hat.copy()
            u[j] += d
            assert orc.loglik(x, y, z, _th(u))["loglik"] <= ref_at + 1e-9

    def f(u):
        r = orc.loglik(x, y, z, _th(u))["loglik"]
        return -r if np.isfinite(r) else np.inf
    init = np.array([_u(START)] + [_u(START) + 0.1 * np.eye(6)[i] for i in range(6)])
    sp = minimize(f, _u(START), method="Nelder-Mead",
                  options={"initial_simplex": init, "xatol": 1e-6, "fatol": 1e-8,
                           "maxfev": 4000})
    th_sp = np.array(_th(sp.x))
    _say("  scipy on oracle: %s loglik %.8f evals %d" % (np.round(th_sp, 5), -sp.fun, sp.nfev))
    assert abs(-sp.fun - ref_at) <= 1e-3
    assert np.max(np.abs(np.array(fit["theta"]) - th_sp) / np.abs(th_sp)) <= 0.05


def test_mle_fit_large_problem_runs_on_the_tiled_path(lib, orc):
    """n = 700 (above the one-launch size): the tiled path; a short fit
    improves the likelihood from the start, and the reported value is the
    oracle's at the returned theta."""
    n = 700
    x, y = synthetic.jittered_grid(n, 5)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    z = orc.simulate_z(x, y, TRUE, synthetic.normal_eps(2 * n, 5))
    fit = lib.mle_fit(_dev(x), _dev(y), _dev(z), START, {"nb": 256}, max_evals=40)
    ref_at = orc.loglik(x, y, z, fit["theta"])["loglik"]
    _say("  n=700 after %d evals: loglik %.6f (start %.6f)" % (
        fit["evals"], fit["loglik"], orc.loglik(x, y, z, START)["loglik"]))
    assert abs(fit["loglik"] - ref_at) <= 1e-9 * abs(ref_at)
    assert ref_at > orc.loglik(x, y, z, START)["loglik"]
    assert 40 <= fit["evals"] <= 40 + 6


def test_mle_fit_rejects_bad_start(lib, orc):
    x, y = synthetic.jittered_grid(50, 1)
    z = synthetic.normal_eps(100, 1)
    with pytest.raises(lib.MvgError):
        lib.mle_fit(_dev(x), _dev(y), _dev(z), (1, 1, 0.1, 5.0, 1, 0.5), {"nb": 128})
