"""CPU checks of the C ABI: the built library loads and exports every function
that include/mvgeo.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mvgeo.h")
SO = os.path.join(ROOT, "paper_2008_07437_amd", "libmvgeo.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set()
    for m in re.finditer(r"^\s*(?!typedef)(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(",
                         src, re.M):
        name = m.group(1)
        if name not in ("if", "while", "for", "sizeof", "defined"):
            names.add(name)
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("cov_generate", "potrf_tiled", "loglik", "tlr_compress", "cokrige_predict",
              "morton_order", "mvg_footprint", "mvg_last_error"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(SO), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(SO)
    for name in sorted(_declared()):
        assert hasattr(lib, name), name
    lib.mvg_last_error.restype = ctypes.c_char_p
    assert lib.mvg_last_error() == b""


def test_product_path_fails_without_gpu_or_library(monkeypatch):
    import torch
    import paper_2008_07437_amd._lib as L
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises((ImportError, RuntimeError)):
        L._load()


def _lib_cpu():
    lib = ctypes.CDLL(SO)
    lib.mvg_footprint.restype = ctypes.c_size_t
    lib.mvg_footprint.argtypes = [ctypes.c_int64, ctypes.c_void_p]
    return lib


def _opts(**kw):
    import paper_2008_07437_amd._lib as L
    return L.Opts.make(**kw)


@pytest.mark.skipif(not os.path.exists(SO), reason="library not built")
def test_footprint_host_logic():
    """mvg_footprint is host arithmetic (no device call): it grows with n,
    mixed precision adds the FP64 copy kept for the refinement, the TLR
    estimate stays far below dense at large n, and invalid options give 0."""
    lib = _lib_cpu()
    fp = lambda n, **kw: lib.mvg_footprint(n, ctypes.byref(_opts(**kw)))  # noqa: E731
    dense = [fp(n, nb=512) for n in (1000, 5000, 25600)]
    assert dense[0] < dense[1] < dense[2]
    # 51,200^2 lower tiles: 100*101/2 tiles of 2 MiB, about 10.6 GB
    assert 10.5e9 < dense[2] < 11.5e9
    assert fp(25600, nb=512, precision=1) > dense[2]
    assert fp(100000, nb=1200, precision=3) < 0.5 * fp(100000, nb=512)
    assert fp(1000, nb=100) == 0                      # not a supported dense tile size
    assert fp(1000, nb=128, precision=1, band_tiles=1) == 0
    assert fp(1000, nb=1200, precision=3, tlr_max_rank=600) == 0
    assert fp(0, nb=512) == 0
    # FP32X: every tile FP64 plus the FP64 Sigma: about twice the dense size,
    # more than FP32 storage; a band below 2 is refused as for the other modes
    fx = fp(25600, nb=512, precision=5)
    assert fx > fp(25600, nb=512, precision=1) and 1.9 * dense[2] < fx < 2.3 * dense[2]
    assert fp(1000, nb=128, precision=5, band_tiles=1) == 0
    # BF16X3: FP32X's layout plus the two BF16 planes of the staged panel
    # ((T - 1) nb^2 values of 2 + 2 bytes, T = 100)
    f3 = fp(25600, nb=512, precision=6)
    assert f3 - fx == 99 * 512 * 512 * 4
    assert fp(1000, nb=128, precision=6, band_tiles=1) == 0
    assert fp(1000, nb=128, precision=7) == 0         # no such precision


def test_theta_batch_marshalling_rejects_bad_shapes():
    """loglik hands a batch of theta to the library as one k x 6 FP64 array
    (the layout of mvg_theta); other shapes are refused before any device
    or library call."""
    import ctypes as C
    import paper_2008_07437_amd as mvg
    assert C.sizeof(mvg.Theta) == 6 * 8
    assert [f[0] for f in mvg.Theta._fields_] == ["sigma11_sq", "sigma22_sq", "a", "nu11",
                                                  "nu22", "beta"]
    for bad in ([(1.0, 1.0, 0.1)], [[1.0] * 7], np.ones((2, 3, 6))):
        with pytest.raises(ValueError):
            mvg.loglik(None, None, None, bad)


@pytest.mark.skipif(not os.path.exists(SO), reason="library not built")
def test_dst_band_matches_oracle_and_footprint_shrinks(orc):
    """mvg_dst_band (host arithmetic) equals the oracle's tile-by-tile count
    for every size, tile and fraction tried (bit-exact integer); a DST
    matrix stores only its kept tiles plus one zero tile."""
    lib = _lib_cpu()
    lib.mvg_dst_band.restype = ctypes.c_int
    lib.mvg_dst_band.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_double]
    for n in (1, 64, 100, 1000, 1337, 25600):
        for nb in (128, 256, 512):
            T = (2 * n + nb - 1) // nb
            for keep in (0.05, 0.3, 0.4, 0.5, 0.7, 0.999, 1.0):
                assert lib.mvg_dst_band(n, nb, keep) == orc.dst_band(T, keep), (n, nb, keep)
    assert lib.mvg_dst_band(1000, 128, 0.0) == -1 and lib.mvg_dst_band(1000, 128, 1.5) == -1
    assert lib.mvg_dst_band(0, 128, 0.4) == -1
    fp = lambda n, **kw: lib.mvg_footprint(n, ctypes.byref(_opts(**kw)))  # noqa: E731
    w = lib.mvg_dst_band(25600, 512, 0.4)
    dst, dense = fp(25600, nb=512, precision=4, band_tiles=w), fp(25600, nb=512)
    assert dst < 0.75 * dense
    assert fp(25600, nb=512, precision=4, band_tiles=100) == dense


@pytest.mark.skipif(not os.path.exists(SO), reason="library not built")
def test_server_rejects_bad_arguments_without_a_device():
    lib = ctypes.CDLL(SO)
    lib.mvg_server_create.restype = ctypes.c_void_p
    lib.mvg_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    assert lib.mvg_server_create(0, 2, None) is None
    assert lib.mvg_server_create(1 << 30, 0, None) is None
    assert lib.mvg_server_create(1 << 30, 64, None) is None


@pytest.mark.skipif(not os.path.exists(SO), reason="library not built")
def test_nelder_mead_host_optimiser():
    """mvg_nelder_mead (host only) on objectives with known minima: a
    weighted quadratic (minimum at c), Rosenbrock's valley (minimum at
    (1, 1)); the first call evaluates the whole starting simplex in one batch,
    later calls one point (or dim points for a shrink); an objective error stops the
    search and is returned."""
    lib = ctypes.CDLL(SO)
    CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_double), ctypes.c_void_p)
    lib.mvg_nelder_mead.restype = ctypes.c_int
    lib.mvg_nelder_mead.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_double, CB,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    sizes = []

    def run(fun, x0, step, max_evals, ftol, xtol):
        dim = len(x0)

        def cb(m, V, f, ctx):
            sizes.append(m)
            for i in range(m):
                f[i] = fun(np.array([V[i * dim + j] for j in range(dim)]))
            return 0
        cbf = CB(cb)
        xb = np.zeros(dim)
        fb = ctypes.c_double()
        ev, it, cv = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        x0a = np.asarray(x0, dtype=np.float64)
        rc = lib.mvg_nelder_mead(dim, x0a.ctypes.data, step, cbf, None, max_evals, ftol, xtol,
                                 xb.ctypes.data, ctypes.byref(fb), ctypes.byref(ev),
                                 ctypes.byref(it), ctypes.byref(cv))
        return rc, xb, fb.value, ev.value, bool(cv.value)

    c = np.array([0.3, -1.2, 2.0, 0.7])
    w = np.array([1.0, 3.0, 0.5, 2.0])
    rc, xb, fb, ev, cv = run(lambda v: float(np.sum(w * (v - c) ** 2)), [0, 0, 0, 0], 0.5, 4000,
                             1e-14, 1e-8)
    assert rc == 0 and cv and np.max(np.abs(xb - c)) <= 1e-6 and fb <= 1e-12
    assert sizes[0] == 5 and set(sizes[1:]) <= {1, 4}   # starting simplex in one batch
    sizes.clear()
    rosen = lambda v: float(100.0 * (v[1] - v[0] ** 2) ** 2 + (1.0 - v[0]) ** 2)  # noqa: E731
    rc, xb, fb, ev, cv = run(rosen, [-1.2, 1.0], 0.1, 5000, 1e-14, 1e-9)
    assert rc == 0 and cv and np.max(np.abs(xb - 1.0)) <= 1e-5
    assert lib.mvg_nelder_mead(0, None, 0.1, CB(lambda *a: 0), None, 10, 0, 0, None, None, None,
                               None, None) == -1

    def failing(m, V, f, ctx):
        return 7
    fb_ = CB(failing)
    xb = np.zeros(2)
    out = [ctypes.c_double(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()]
    x0 = np.zeros(2)
    assert lib.mvg_nelder_mead(2, x0.ctypes.data, 0.1, fb_, None, 100, 0.0, 0.0, xb.ctypes.data,
                               *[ctypes.byref(o) for o in out]) == 7
