"""GPU checks of the request server: likelihood and cokriging requests of
uneven size admitted by footprint and run concurrently must give the same
results as the same requests run alone (bitwise: every kernel sums in a
fixed order), match the oracle, reuse resident factors, and reject what can
never fit."""
import sys
import time

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


def _collect(S, n, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < n and time.time() - t0 < timeout:
        for r in S.poll(64, 200):
            out[r.id] = r
    assert len(out) == n, "server did not finish"
    return out


def test_mix_equals_alone_and_oracle(lib, orc):
    import torch
    sizes = [150, 300, 450, 700, 1100]   # the first two take the batched launch
    data = []
    for k, n in enumerate(sizes):
        x, y = synthetic.jittered_grid(n, 40 + k)
        p = orc.morton_order(x, y)
        x, y = x[p], y[p]
        z = synthetic.normal_eps(2 * n, 40 + k)
        data.append((x, y, z))
    ths = synthetic.jittered_thetas(6, 7)
    x0, y0 = synthetic.uniform_targets(25, 3)
    S = lib.Server(16 << 30, 4, {"nb": 256})
    dsid = [S.add_dataset(_dev(x), _dev(y), _dev(z)) for x, y, z in data]
    reqs = []  # (id, kind, dataset, theta, zhat)
    for rep in range(2):
        for d in range(len(sizes)):
            for t in ths[:3]:
                reqs.append((S.submit(lib.REQ_LOGLIK, dsid[d], t), 0, d, t, None))
        for d in (2, 4):
            zh = torch.empty(50, dtype=torch.float64, device="cuda")
            reqs.append((S.submit(lib.REQ_COKRIGE, dsid[d], ths[0], _dev(x0), _dev(y0), zh), 1, d,
                         ths[0], zh))
    res = _collect(S, len(reqs))
    stats = S.stats()
    S.close()
    _say("  server stats", stats, "batch sizes", sorted({r.batch for r in res.values()}))
    assert max(r.batch for r in res.values()) > 1      # small requests were batched
    assert stats["hits"] >= 2                          # cokriging reused resident factors
    # continuous batching, not a queue: admitted requests run at the same time
    # (their [t_start, t_end] intervals on the server clock overlap)
    iv = sorted((r.t_start, r.t_end) for r in res.values())
    overlaps = sum(1 for i in range(len(iv)) for j in range(i + 1, len(iv))
                   if iv[j][0] < iv[i][1] and iv[i][0] < iv[j][1])
    _say("  overlapping request pairs: %d of %d requests" % (overlaps, len(iv)))
    assert overlaps >= 1
    cache = {}
    for rid, kind, d, t, zh in reqs:
        r = res[rid]
        assert r.status == 0, (rid, r.status)
        x, y, z = data[d]
        if kind == 0:
            if 2 * sizes[d] <= lib._lib.SMALL_MAX_ROWS:
                alone = lib.loglik_many([(_dev(x), _dev(y), _dev(z), t)])["loglik"][0]
            else:
                alone = lib.loglik(_dev(x), _dev(y), _dev(z), t, {"nb": 256})["loglik"][0]
            assert r.loglik == alone, (rid, r.loglik, alone)
            key = (d, tuple(t))
            if key not in cache:
                cache[key] = orc.loglik(x, y, z, t)["loglik"]
            assert abs(r.loglik - cache[key]) <= 1e-9 * abs(cache[key])
        else:
            _, F = lib.loglik(_dev(x), _dev(y), _dev(z), t, {"nb": 256}, keep=True)
            alone = lib.cokrige_predict(F, _dev(x0), _dev(y0)).cpu().numpy().ravel()
            assert np.array_equal(zh.cpu().numpy(), alone)
        assert r.t_arrive <= r.t_start <= r.t_end


def test_request_that_never_fits_is_rejected(lib, orc):
    x, y = synthetic.jittered_grid(2000, 1)
    z = synthetic.normal_eps(4000, 1)
    S = lib.Server(1 << 20, 2, {"nb": 256})   # 1 MiB budget
    d = S.add_dataset(_dev(x), _dev(y), _dev(z))
    rid = S.submit(lib.REQ_LOGLIK, d, synthetic.THETA_REF)
    r = _collect(S, 1)[rid]
    S.close()
    assert r.status == -104   # MVG_ERR_LIMIT
