"""GPU checks of loglik_many_noalloc, the batched small-problem likelihood with
its scratch in the library's fixed device array: the same results as
loglik_many (which allocates its scratch) on two calls in a row, the second
smaller, with the scratch holding fewer workspaces than tasks; and the size
limits rejected before any device work."""
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


def _dataset(orc, n, seed):
    x, y = synthetic.jittered_grid(n, seed)
    p = orc.morton_order(x, y)
    x, y = x[p], y[p]
    return x, y, synthetic.normal_eps(2 * n, seed)


def _same(a, b):
    for key in ("loglik", "logdet", "quad", "status"):
        assert np.array_equal(a[key], b[key]), key


def test_noalloc_equals_loglik_many_twice(lib, orc):
    """600 theta on one n = 400 dataset (800 x 800 each: the 256 MiB scratch
    holds about 50 workspaces, so about 50 workgroups take the 600 tasks),
    then a smaller call of 40 tasks over three datasets of other sizes: both
    equal loglik_many bitwise, and sampled tasks match the oracle."""
    import torch
    x, y, z = _dataset(orc, 400, 0)
    X, Y, Z = _dev(x), _dev(y), _dev(z)
    ths = synthetic.jittered_thetas(600, 11)
    tasks = [(X, Y, Z, t) for t in ths]
    _say("noalloc: call 1, 600 tasks at n = 400")
    got = lib.loglik_many_noalloc(tasks)
    ref = lib.loglik_many(tasks)
    torch.cuda.synchronize()
    _same(got, ref)
    assert np.all(got["status"] == 0)
    for i in (0, 317, 599):
        o = orc.loglik(x, y, z, ths[i])
        assert abs(got["loglik"][i] - o["loglik"]) <= 1e-9 * abs(o["loglik"])
    small = []
    host = []
    for n, seed in ((50, 3), (120, 4), (333, 5)):
        xs, ys, zs = _dataset(orc, n, seed)
        host.append((xs, ys, zs))
        small.append((_dev(xs), _dev(ys), _dev(zs)))
    ths2 = synthetic.jittered_thetas(40, 12)
    tasks2 = [small[i % 3] + (ths2[i],) for i in range(40)]
    _say("noalloc: call 2, 40 tasks at n = 50 / 120 / 333")
    got2 = lib.loglik_many_noalloc(tasks2)
    ref2 = lib.loglik_many(tasks2)
    torch.cuda.synchronize()
    _same(got2, ref2)
    assert np.all(got2["status"] == 0)
    for i in (0, 1, 2, 39):
        xs, ys, zs = host[i % 3]
        o = orc.loglik(xs, ys, zs, ths2[i])
        assert abs(got2["loglik"][i] - o["loglik"]) <= 1e-9 * abs(o["loglik"])


def test_noalloc_rejects_too_many_tasks(lib, orc):
    """More tasks than the static staging holds: MVG_ERR_LIMIT before any
    device work."""
    x, y, z = _dataset(orc, 20, 1)
    X, Y, Z = _dev(x), _dev(y), _dev(z)
    tasks = [(X, Y, Z, synthetic.THETA_REF)] * 4097
    with pytest.raises(lib.MvgError) as e:
        lib.loglik_many_noalloc(tasks)
    assert e.value.code == -104
