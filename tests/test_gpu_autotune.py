"""GPU checks of the tile-size autotuner: it times every candidate on the
problem itself, returns the fastest, caches the choice per (n, precision,
band), and loglik with MVG_NB_AUTO evaluates with exactly that tile size."""
import sys

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


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


def test_autotune_picks_fastest_and_caches(lib, orc):
    th = (1.0, 1.0, 0.1, 0.5, 1.0, 0.5)
    n = 1500
    x, y = synthetic.jittered_grid(n, 2)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    z = synthetic.normal_eps(2 * n, 2)
    best, secs = lib.mvg_autotune_nb(_dev(x), _dev(y), _dev(z), th, {}, [128, 256, 512])
    print("autotune n=%d: %s -> %d" % (n, secs, best), file=sys.stderr, flush=True)
    assert best in (128, 256, 512) and secs is not None
    assert all(np.isfinite(v) for v in secs.values())
    assert secs[best] == min(secs.values())
    again, cached = lib.mvg_autotune_nb(_dev(x), _dev(y), _dev(z), th, {}, [128, 256, 512])
    assert again == best and cached is None
    auto = lib.loglik(_dev(x), _dev(y), _dev(z), th, {"nb": lib.MVG_NB_AUTO})
    fixed = lib.loglik(_dev(x), _dev(y), _dev(z), th, {"nb": best})
    assert auto["loglik"][0] == fixed["loglik"][0]
    ref = orc.loglik(x, y, z, th)["loglik"]
    assert abs(auto["loglik"][0] - ref) <= 1e-9 * abs(ref)


def test_autotune_rejects_bad_candidates(lib, orc):
    x, y = synthetic.jittered_grid(100, 1)
    z = synthetic.normal_eps(200, 1)
    with pytest.raises(lib.MvgError):
        lib.mvg_autotune_nb(_dev(x), _dev(y), _dev(z), (1, 1, 0.1, 0.5, 1, 0.5), {}, [100])
    with pytest.raises(lib.MvgError):
        lib.mvg_autotune_nb(_dev(x), _dev(y), _dev(z), (1, 1, 0.1, 0.5, 1, 0.5),
                            {"precision": lib.MVG_TLR}, [512])
