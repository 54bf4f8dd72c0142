"""GPU checks of the batched small-problem likelihood (one persistent launch,
one workgroup per task) against the FP64 oracle, and of its independence of
the batch it runs in."""
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


def _dataset(orc, n, seed, theta):
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    z = orc.simulate_z(x, y, theta, synthetic.normal_eps(2 * n, seed))
    return x, y, z


TH0 = synthetic.THETA_REF


def test_simplex_batch_matches_oracle_and_single_calls(lib, orc):
    """The 7 Nelder-Mead simplex points on the N = 400 workload in one launch."""
    x, y, z = _dataset(orc, 400, 0, TH0)
    ths = synthetic.nelder_mead_simplex(TH0)
    got = lib.loglik(_dev(x), _dev(y), _dev(z), ths, {"nb": 128})
    for i, t in enumerate(ths):
        ref = orc.loglik(x, y, z, t)
        one = lib.loglik(_dev(x), _dev(y), _dev(z), t, {"nb": 128})  # tiled path
        rel = abs(got["loglik"][i] - ref["loglik"]) / abs(ref["loglik"])
        _say("  theta %d rel dl %.2e (vs tiled %.2e)" % (i, rel, abs(got["loglik"][i] - one["loglik"][0]) / abs(ref["loglik"])))
        assert got["status"][i] == 0
        assert rel <= 1e-9
        for key in ("logdet", "quad"):
            assert abs(got[key][i] - ref[key]) <= 1e-9 * abs(ref[key])


def test_many_datasets_alone_equals_in_mix(lib, orc):
    rng = synthetic.rng(5, 1)
    tasks, refs = [], []
    for k in range(12):
        n = int(rng.integers(1, 513))
        th = synthetic.jittered_thetas(1, 100 + k)[0]
        x, y, z = _dataset(orc, n, 20 + k, th)
        tasks.append((_dev(x), _dev(y), _dev(z), th))
        refs.append(orc.loglik(x, y, z, th))
    mix = lib.loglik_many(tasks)
    for k, t in enumerate(tasks):
        alone = lib.loglik_many([t])
        assert alone["loglik"][0] == mix["loglik"][k]
        assert alone["logdet"][0] == mix["logdet"][k]
        rel = abs(mix["loglik"][k] - refs[k]["loglik"]) / abs(refs[k]["loglik"])
        assert rel <= 1e-9, (k, rel)


def test_batch_with_a_failing_task(lib, orc):
    """A non-positive-definite task reports its pivot; the others are unaffected."""
    x, y, z = _dataset(orc, 200, 3, TH0)
    xb = np.concatenate([x[:50], x[:50]])    # duplicated locations: singular
    yb = np.concatenate([y[:50], y[:50]])
    zb = synthetic.normal_eps(200, 3)
    good = (_dev(x), _dev(y), _dev(z), TH0)
    bad = (_dev(xb), _dev(yb), _dev(zb), TH0)
    res = lib.loglik_many([good, bad, good])
    ref = orc.loglik(xb, yb, zb, TH0)
    assert res["status"][0] == 0 and res["status"][2] == 0
    assert res["loglik"][0] == res["loglik"][2]
    assert res["status"][1] == ref["info"] and res["loglik"][1] == -np.inf


def test_single_location_and_size_limit(lib, orc):
    z = np.array([0.3, -1.1])
    res = lib.loglik_many([(_dev([0.5]), _dev([0.5]), _dev(z), TH0)])
    ref = orc.loglik([0.5], [0.5], z, TH0)
    assert abs(res["loglik"][0] - ref["loglik"]) <= 1e-13 * abs(ref["loglik"])
    x, y = synthetic.jittered_grid(513, 0)
    with pytest.raises(lib.MvgError):
        lib.loglik_many([(_dev(x), _dev(y), _dev(np.zeros(1026)), TH0)])
