"""ctypes binding of libmvgeo.so: same names as the C ABI, argument marshalling only."""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libmvgeo.so")

MVG_FP64, MVG_MIXED_FP32, MVG_MIXED_BF16, MVG_TLR, MVG_DST, MVG_MIXED_FP32X = 0, 1, 2, 3, 4, 5
MVG_MIXED_BF16X3 = 6

c_double, c_int, c_int64, c_void_p = ctypes.c_double, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p


class MvgError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__("%s failed with code %d: %s" % (fn, code, msg))
        self.code = code


class Theta(ctypes.Structure):
    """theta = (sigma11^2, sigma22^2, a, nu11, nu22, beta) in the paper's order."""
    _fields_ = [("sigma11_sq", c_double), ("sigma22_sq", c_double), ("a", c_double),
                ("nu11", c_double), ("nu22", c_double), ("beta", c_double)]

    @classmethod
    def of(cls, t) -> "Theta":
        t = [float(v) for v in t]
        if len(t) != 6:
            raise ValueError("theta needs 6 entries")
        return cls(*t)


PMAX = 4


class ThetaP(ctypes.Structure):
    """theta of the p-variate model: {'sigma_sq': [p], 'a': a, 'nu': [p],
    'beta': p x p} (beta symmetric, unit diagonal, positive definite)."""
    _fields_ = [("p", c_int), ("sigma_sq", c_double * PMAX), ("a", c_double),
                ("nu", c_double * PMAX), ("beta", c_double * (PMAX * PMAX))]

    @classmethod
    def of(cls, t) -> "ThetaP":
        if isinstance(t, cls):
            return t
        s = [float(v) for v in t["sigma_sq"]]
        p = len(s)
        if not 1 <= p <= PMAX or len(t["nu"]) != p:
            raise ValueError("theta_p: 1 <= p <= %d variables, one nu per variable" % PMAX)
        b = np.asarray(t["beta"], dtype=np.float64).reshape(p, p)
        out = cls()
        out.p = p
        out.a = float(t["a"])
        for i in range(p):
            out.sigma_sq[i] = s[i]
            out.nu[i] = float(t["nu"][i])
            for j in range(p):
                out.beta[i * PMAX + j] = float(b[i, j])
        return out


class Opts(ctypes.Structure):
    _fields_ = [("precision", c_int), ("nb", c_int), ("band_tiles", c_int),
                ("tlr_acc", c_double), ("tlr_max_rank", c_int), ("seed", ctypes.c_uint64),
                ("ir_max_iter", c_int), ("ir_tol", c_double)]

    @classmethod
    def make(cls, precision=MVG_FP64, nb=0, band_tiles=0, tlr_acc=0.0, tlr_max_rank=0, seed=0,
             ir_max_iter=0, ir_tol=0.0) -> "Opts":
        return cls(int(precision), int(nb), int(band_tiles), float(tlr_acc), int(tlr_max_rank),
                   int(seed), int(ir_max_iter), float(ir_tol))


_lib = None


def library_path() -> str:
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        raise ImportError("libmvgeo.so is not built (run __graft_entry__.build() or "
                          "python paper_2008_07437_amd/build.py)")
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the gfx950 library needs an MI355X GPU")
    lib = ctypes.CDLL(_SO)
    P = c_void_p
    sig = {
        "morton_order": (c_int, [P, P, c_int64, P, P, P, P]),
        "mvg_trmv": (c_int, [P, P, P, P]),
        "cov_generate": (c_int, [P, P, c_int64, P, P, P, P]),
        "potrf_tiled": (c_int, [P, P, P, P]),
        "loglik": (c_int, [P, P, P, c_int64, P, c_int, P, P, P, P, P, P, P]),
        "tlr_compress": (c_int, [P, P, c_int64, P, P, P, P, P]),
        "cokrige_predict": (c_int, [P, P, P, c_int64, P, P, P]),
        "mloe_mmom": (c_int, [P, P, c_int64, P, P, P, P, c_int64, P, P, P, P, P, P]),
        "loglik_p": (c_int, [P, P, P, c_int64, P, c_int, P, P, P, P, P, P]),
        "mle_fit": (c_int, [P, P, P, c_int64, P, P, P, P, P, P, P, P, P]),
        "cov_generate_p": (c_int, [P, P, c_int64, P, P, P, P]),
        "profile_loglik_p": (c_int, [P, P, P, c_int64, P, P, P, P, P, P, P, P]),
        "mvg_footprint": (ctypes.c_size_t, [c_int64, P]),
        "mvg_dst_band": (c_int, [c_int64, c_int, c_double]),
        "mvg_autotune_nb": (c_int, [P, P, P, c_int64, P, P, P, c_int, P, P, P]),
        "mvg_mat_shape": (c_int, [P, P, P, P, P, P]),
        "mvg_mat_nvar": (c_int, [P]),
        "mvg_mat_gather": (c_int, [P, P, P, c_int64, P, P]),
        "mvg_mat_to_dense": (c_int, [P, P, c_int64, P]),
        "mvg_factor_mat": (P, [P]),
        "mvg_factor_w": (P, [P]),
        "mvg_mat_destroy": (None, [P]),
        "mvg_factor_destroy": (None, [P]),
        "mvg_last_error": (ctypes.c_char_p, []),
        "mvg_prof_enable": (c_int, [c_int]),
        "mvg_prof_read": (c_int, [c_int, P, P, P, P]),
        "mvg_ir_stats": (c_int, [c_int, P, P, P]),
        "loglik_many": (c_int, [P, c_int, P, P, P, P, P]),
        "mvg_mat_loglik": (c_int, [P, P, P, P, P, P]),
        "loglik_many_noalloc": (c_int, [P, c_int, P, P, P, P, P]),
        "mvg_server_create": (P, [ctypes.c_size_t, c_int, P]),
        "mvg_server_add_dataset": (c_int, [P, P, P, P, c_int64]),
        "mvg_server_submit": (c_int64, [P, c_int, c_int, P, P, P, c_int64, P, c_double]),
        "mvg_server_poll": (c_int, [P, P, c_int, c_int]),
        "mvg_server_clock": (c_double, [P]),
        "mvg_server_stats": (c_int, [P, P, P, P, P]),
        "mvg_server_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(fn: str, rc: int):
    if rc != 0:
        raise MvgError(fn, rc, (_load().mvg_last_error() or b"").decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _dev_f64(t, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % name)
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("%s must be contiguous float64" % name)
    return c_void_p(t.data_ptr())


def _opts(opts):
    if opts is None:
        return Opts.make()
    if isinstance(opts, dict):
        return Opts.make(**opts)
    return opts


class Mat:
    """Library-owned tile matrix (freed on garbage collection)."""

    def __init__(self, handle):
        self._h = c_void_p(handle) if not isinstance(handle, c_void_p) else handle

    @property
    def handle(self):
        return self._h

    def shape(self):
        n, nb, T, prec, fac = c_int64(), c_int(), c_int(), c_int(), c_int()
        _check("mvg_mat_shape", _load().mvg_mat_shape(self._h, ctypes.byref(n), ctypes.byref(nb),
                                                     ctypes.byref(T), ctypes.byref(prec),
                                                     ctypes.byref(fac)))
        return {"n_loc": n.value, "nb": nb.value, "ntiles": T.value, "precision": prec.value,
                "factored": bool(fac.value)}

    def gather(self, rows, cols, stream=None) -> torch.Tensor:
        r = torch.as_tensor(np.asarray(rows, dtype=np.int64)).cuda()
        c = torch.as_tensor(np.asarray(cols, dtype=np.int64)).cuda()
        out = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        _check("mvg_mat_gather", _load().mvg_mat_gather(self._h, c_void_p(r.data_ptr()),
                                                       c_void_p(c.data_ptr()), r.numel(),
                                                       c_void_p(out.data_ptr()), _stream(stream)))
        torch.cuda.current_stream().synchronize()
        return out

    def to_dense(self, stream=None) -> torch.Tensor:
        """Lower triangle as a dense (p n, p n) tensor (strict upper part 0)."""
        N = _load().mvg_mat_nvar(self._h) * self.shape()["n_loc"]
        buf = torch.empty((N, N), dtype=torch.float64, device="cuda")  # column-major view
        _check("mvg_mat_to_dense", _load().mvg_mat_to_dense(self._h, c_void_p(buf.data_ptr()), N,
                                                           _stream(stream)))
        torch.cuda.current_stream().synchronize()
        return buf.t()

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None and self._h.value:
            _lib.mvg_mat_destroy(self._h)
            self._h = c_void_p(0)


class Factor:
    """Resident factor from loglik(keep=True); reusable by cokrige_predict."""

    def __init__(self, handle):
        self._h = c_void_p(handle)

    @property
    def handle(self):
        return self._h

    def gather(self, rows, cols, stream=None) -> torch.Tensor:
        """Entries (rows[t], cols[t]), rows >= cols, of the factor L."""
        r = torch.as_tensor(np.asarray(rows, dtype=np.int64)).cuda()
        c = torch.as_tensor(np.asarray(cols, dtype=np.int64)).cuda()
        out = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        mat = c_void_p(_load().mvg_factor_mat(self._h))
        _check("mvg_mat_gather", _load().mvg_mat_gather(mat, c_void_p(r.data_ptr()),
                                                       c_void_p(c.data_ptr()), r.numel(),
                                                       c_void_p(out.data_ptr()), _stream(stream)))
        torch.cuda.current_stream().synchronize()
        return out

    def w(self, n: int) -> torch.Tensor:
        """w = Sigma^-1 Z (first 2n entries), copied out."""
        ptr = _load().mvg_factor_w(self._h)
        out = torch.empty(2 * n, dtype=torch.float64, device="cuda")
        _memcpy_d2d(out.data_ptr(), ptr, 8 * 2 * n)
        return out

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None and self._h.value:
            _lib.mvg_factor_destroy(self._h)
            self._h = c_void_p(0)


_hip = None


def _memcpy_d2d(dst: int, src: int, nbytes: int):
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.restype = c_int
        _hip.hipMemcpy.argtypes = [c_void_p, c_void_p, ctypes.c_size_t, c_int]
    torch.cuda.current_stream().synchronize()
    rc = _hip.hipMemcpy(c_void_p(dst), c_void_p(src), nbytes, 3)  # hipMemcpyDeviceToDevice
    if rc != 0:
        raise RuntimeError("hipMemcpy failed (%d)" % rc)


# ---------------------------------------------------------------- entry points

def morton_order(x: torch.Tensor, y: torch.Tensor, sorted_xy=False, stream=None):
    """Morton permutation; with sorted_xy=True also the reordered (x, y)."""
    n = x.numel()
    perm = torch.empty(n, dtype=torch.int64, device=x.device)
    xs = torch.empty_like(x) if sorted_xy else None
    ys = torch.empty_like(y) if sorted_xy else None
    _check("morton_order", _load().morton_order(
        _dev_f64(x, "x"), _dev_f64(y, "y"), n, c_void_p(perm.data_ptr()),
        c_void_p(xs.data_ptr()) if sorted_xy else None,
        c_void_p(ys.data_ptr()) if sorted_xy else None, _stream(stream)))
    return (perm, xs, ys) if sorted_xy else perm


def mvg_trmv(mat: "Mat", eps: torch.Tensor, stream=None) -> torch.Tensor:
    """Z = L eps on a factored matrix (data simulation)."""
    z = torch.empty_like(eps)
    _check("mvg_trmv", _load().mvg_trmv(mat.handle, _dev_f64(eps, "eps"), c_void_p(z.data_ptr()),
                                       _stream(stream)))
    return z


def mvg_mat_loglik(mat: "Mat", z: torch.Tensor, stream=None) -> dict:
    """Eq. (1) from a factored FP64 matrix and Z (after the factorisation)."""
    ll, ld, q = c_double(), c_double(), c_double()
    _check("mvg_mat_loglik", _load().mvg_mat_loglik(mat.handle, _dev_f64(z, "z"), ctypes.byref(ll),
                                                   ctypes.byref(ld), ctypes.byref(q),
                                                   _stream(stream)))
    return {"loglik": ll.value, "logdet": ld.value, "quad": q.value}


def cov_generate(x, y, theta, opts=None, stream=None) -> Mat:
    h = c_void_p()
    th = Theta.of(theta)
    o = _opts(opts)
    _check("cov_generate", _load().cov_generate(_dev_f64(x, "x"), _dev_f64(y, "y"), x.numel(),
                                               ctypes.byref(th), ctypes.byref(o), ctypes.byref(h),
                                               _stream(stream)))
    return Mat(h)


def cov_generate_p(x, y, theta_p, opts=None, stream=None) -> Mat:
    """Sigma of the p-variate model (Representation I, p x p blocks)."""
    h = c_void_p()
    th = ThetaP.of(theta_p)
    o = _opts(opts)
    _check("cov_generate_p", _load().cov_generate_p(_dev_f64(x, "x"), _dev_f64(y, "y"), x.numel(),
                                                   ctypes.byref(th), ctypes.byref(o),
                                                   ctypes.byref(h), _stream(stream)))
    return Mat(h)


def loglik_p(x, y, z, thetas_p, opts=None, stream=None) -> dict:
    """Eq. (1) for the p-variate model; thetas_p: one theta dict or a list."""
    ths = [thetas_p] if isinstance(thetas_p, (dict, ThetaP)) else list(thetas_p)
    k = len(ths)
    arr = (ThetaP * k)(*[ThetaP.of(t) for t in ths])
    ll, ld, q = np.zeros(k), np.zeros(k), np.zeros(k)
    st = np.zeros(k, dtype=np.int64)
    o = _opts(opts)
    _check("loglik_p", _load().loglik_p(_dev_f64(x, "x"), _dev_f64(y, "y"), _dev_f64(z, "z"),
                                        x.numel(), arr, k, ctypes.byref(o),
                                        ll.ctypes.data_as(c_void_p), ld.ctypes.data_as(c_void_p),
                                        q.ctypes.data_as(c_void_p), st.ctypes.data_as(c_void_p),
                                        _stream(stream)))
    return {"loglik": ll, "logdet": ld, "quad": q, "status": st}


def profile_loglik_p(x, y, z, theta_p, opts=None, stream=None) -> dict:
    """Section 5.2 profile likelihood: sigma_ii^2 = Z_i^T R_ii^-1 Z_i / n, then
    Eq. (1) at those variances (theta_p's own variances are not read)."""
    th = ThetaP.of(theta_p)
    s2 = np.zeros(th.p)
    ll, ld, q = c_double(), c_double(), c_double()
    st = c_int64()
    o = _opts(opts)
    _check("profile_loglik_p", _load().profile_loglik_p(
        _dev_f64(x, "x"), _dev_f64(y, "y"), _dev_f64(z, "z"), x.numel(), ctypes.byref(th),
        ctypes.byref(o), s2.ctypes.data_as(c_void_p), ctypes.byref(ll), ctypes.byref(ld),
        ctypes.byref(q), ctypes.byref(st), _stream(stream)))
    return {"sigma_sq": s2, "loglik": ll.value, "logdet": ld.value, "quad": q.value,
            "status": st.value}


class MleOpts(ctypes.Structure):
    _fields_ = [("max_evals", c_int), ("ftol", c_double), ("xtol", c_double), ("step", c_double)]


def mle_fit(x, y, z, theta0, opts=None, max_evals=0, ftol=0.0, xtol=0.0, step=0.0, stream=None):
    """Nelder-Mead maximum-likelihood estimate of theta from theta0 (host
    driver in the library; every evaluation is the GPU likelihood)."""
    th0 = Theta.of(theta0)
    mo = MleOpts(int(max_evals), float(ftol), float(xtol), float(step))
    out = Theta()
    ll = c_double()
    ev, it, conv = c_int(), c_int(), c_int()
    o = _opts(opts)
    _check("mle_fit", _load().mle_fit(_dev_f64(x, "x"), _dev_f64(y, "y"), _dev_f64(z, "z"),
                                      x.numel(), ctypes.byref(th0), ctypes.byref(o),
                                      ctypes.byref(mo), ctypes.byref(out), ctypes.byref(ll),
                                      ctypes.byref(ev), ctypes.byref(it), ctypes.byref(conv),
                                      _stream(stream)))
    th = (out.sigma11_sq, out.sigma22_sq, out.a, out.nu11, out.nu22, out.beta)
    return {"theta": th, "loglik": ll.value, "evals": ev.value, "iters": it.value,
            "converged": bool(conv.value)}


def potrf_tiled(mat: Mat, opts=None, stream=None) -> int:
    info = c_int64()
    o = _opts(opts)
    _check("potrf_tiled", _load().potrf_tiled(mat.handle, ctypes.byref(o), ctypes.byref(info),
                                             _stream(stream)))
    return int(info.value)


def loglik(x, y, z, thetas, opts=None, keep=False, stream=None):
    """Eq. (1) for one theta (6 numbers) or a batch (k x 6).  Returns a dict of
    numpy arrays {'loglik', 'logdet', 'quad', 'status'} and, with keep=True
    (single theta), the resident Factor as a second value."""
    # mvg_theta is six consecutive doubles: a C-contiguous k x 6 array has its layout
    th = np.ascontiguousarray(np.atleast_2d(np.asarray(thetas, dtype=np.float64)))
    if th.ndim != 2 or th.shape[1] != 6:
        raise ValueError("theta needs 6 entries")
    k = th.shape[0]
    arr = th.ctypes.data_as(c_void_p)
    ll = np.zeros(k)
    ld = np.zeros(k)
    q = np.zeros(k)
    st = np.zeros(k, dtype=np.int64)
    o = _opts(opts)
    fh = c_void_p()
    rc = _load().loglik(_dev_f64(x, "x"), _dev_f64(y, "y"), _dev_f64(z, "z"), x.numel(),
                        arr, k, ctypes.byref(o), ll.ctypes.data_as(c_void_p),
                        ld.ctypes.data_as(c_void_p), q.ctypes.data_as(c_void_p),
                        st.ctypes.data_as(c_void_p), ctypes.byref(fh) if keep else None,
                        _stream(stream))
    _check("loglik", rc)
    res = {"loglik": ll, "logdet": ld, "quad": q, "status": st}
    if keep:
        return res, (Factor(fh.value) if fh.value else None)
    return res


class Task(ctypes.Structure):
    _fields_ = [("x", c_void_p), ("y", c_void_p), ("z", c_void_p), ("n_loc", c_int64),
                ("theta", Theta)]


SMALL_MAX_ROWS = 1024


def loglik_many(tasks, stream=None, noalloc=False):
    """Eq. (1) for many small problems in one persistent launch.  tasks: list
    of (x, y, z, theta) with device float64 tensors (2 n <= 1024).  Returns a
    dict of numpy arrays as loglik does.  noalloc=True calls
    loglik_many_noalloc (the library's fixed scratch array, no allocation)."""
    if noalloc:
        return loglik_many_noalloc(tasks, stream)
    return _loglik_many("loglik_many", tasks, stream)


def loglik_many_noalloc(tasks, stream=None):
    """loglik_many without any device allocation (fixed scratch array)."""
    return _loglik_many("loglik_many_noalloc", tasks, stream)


def _loglik_many(name, tasks, stream):
    k = len(tasks)
    arr = (Task * k)()
    for i, (x, y, z, th) in enumerate(tasks):
        arr[i] = Task(_dev_f64(x, "x"), _dev_f64(y, "y"), _dev_f64(z, "z"), x.numel(),
                      Theta.of(th))
    ll, ld, q = np.zeros(k), np.zeros(k), np.zeros(k)
    st = np.zeros(k, dtype=np.int64)
    _check(name, getattr(_load(), name)(arr, k, ll.ctypes.data_as(c_void_p),
                                        ld.ctypes.data_as(c_void_p), q.ctypes.data_as(c_void_p),
                                        st.ctypes.data_as(c_void_p), _stream(stream)))
    return {"loglik": ll, "logdet": ld, "quad": q, "status": st}


def tlr_compress(x, y, theta, opts=None, stream=None):
    """TLR compression of Sigma(theta); returns (Mat, ranks T x T, -1 = dense)."""
    h = c_void_p()
    th = Theta.of(theta)
    if opts is None or isinstance(opts, dict):
        opts = dict(opts or {})
        opts["precision"] = MVG_TLR
    o = _opts(opts)
    N = 2 * x.numel()
    T = (N + (o.nb or 1200) - 1) // (o.nb or 1200)
    ranks = np.zeros((T, T), dtype=np.int32)
    _check("tlr_compress", _load().tlr_compress(_dev_f64(x, "x"), _dev_f64(y, "y"), x.numel(),
                                               ctypes.byref(th), ctypes.byref(o), ctypes.byref(h),
                                               ranks.ctypes.data_as(c_void_p), _stream(stream)))
    return Mat(h), ranks


def cokrige_predict(factor: Factor, x0, y0, with_mse=False, stream=None):
    m = x0.numel()
    zhat = torch.empty(2 * m, dtype=torch.float64, device=x0.device)
    mse = torch.empty(m, dtype=torch.float64, device=x0.device) if with_mse else None
    _check("cokrige_predict", _load().cokrige_predict(
        factor.handle, _dev_f64(x0, "x0"), _dev_f64(y0, "y0"), m, c_void_p(zhat.data_ptr()),
        c_void_p(mse.data_ptr()) if with_mse else None, _stream(stream)))
    zhat = zhat.view(m, 2)
    return (zhat, mse) if with_mse else zhat


def mloe_mmom(x, y, theta, theta_a, x0, y0, opts=None, stream=None):
    """Section 5.4 (Eq. 5-8, Algorithm 1): prediction efficiency of the model
    theta_a when theta is true, at the m targets (x0, y0).  Returns
    {'mloe', 'mmom', 'loe', 'mom', 'status'}; status 1 / 2 means Sigma(theta) /
    Sigma(theta_a) is not positive definite (means are NaN then)."""
    m = x0.numel()
    th, tha = Theta.of(theta), Theta.of(theta_a)
    loe = torch.empty(m, dtype=torch.float64, device=x0.device)
    mom = torch.empty(m, dtype=torch.float64, device=x0.device)
    a, b = c_double(), c_double()
    o = _opts(opts)
    rc = _load().mloe_mmom(_dev_f64(x, "x"), _dev_f64(y, "y"), x.numel(), ctypes.byref(th),
                           ctypes.byref(tha), _dev_f64(x0, "x0"), _dev_f64(y0, "y0"), m,
                           ctypes.byref(o), ctypes.byref(a), ctypes.byref(b),
                           c_void_p(loe.data_ptr()), c_void_p(mom.data_ptr()), _stream(stream))
    if rc not in (0, 1, 2):
        _check("mloe_mmom", rc)
    return {"mloe": a.value, "mmom": b.value, "loe": loe, "mom": mom, "status": rc}


PROF_KINDS = {"trailing": 0, "gen": 1, "potrf": 2, "solve": 3, "cokrige": 4, "lowp": 5, "ir": 6,
              "syrk": 7, "tlr_gemm": 8, "qr": 9}


def mvg_prof_enable(on: bool = True):
    _check("mvg_prof_enable", _load().mvg_prof_enable(1 if on else 0))


def mvg_prof_read(kind: str) -> dict:
    n, ms, fl, by = c_int64(), c_double(), c_double(), c_double()
    _check("mvg_prof_read", _load().mvg_prof_read(PROF_KINDS[kind], ctypes.byref(n),
                                                 ctypes.byref(ms), ctypes.byref(fl),
                                                 ctypes.byref(by)))
    return {"launches": n.value, "ms": ms.value, "flops": fl.value, "bytes": by.value}


MVG_NB_AUTO = -1


def mvg_autotune_nb(x, y, z, theta, opts=None, candidates=None, stream=None):
    """Tile size by measurement (one timed evaluation per candidate, cached
    per (n_loc, precision, band)).  Returns (nb, {candidate: seconds} or
    None when the choice came from the cache)."""
    th = Theta.of(theta)
    o = _opts(opts)
    cand = None if candidates is None else (c_int * len(candidates))(*candidates)
    k = 4 if candidates is None else len(candidates)
    secs = np.full(k, np.nan)
    best = c_int()
    rc = _load().mvg_autotune_nb(_dev_f64(x, "x"), _dev_f64(y, "y"), _dev_f64(z, "z"), x.numel(),
                                 ctypes.byref(th), ctypes.byref(o), cand,
                                 0 if candidates is None else len(candidates), ctypes.byref(best),
                                 secs.ctypes.data_as(c_void_p), _stream(stream))
    if rc < 0:
        _check("mvg_autotune_nb", rc)
    cands = list(candidates) if candidates is not None else [256, 512, 768, 1024]
    return best.value, (None if rc == 1 else dict(zip(cands, secs.tolist())))


def mvg_dst_band(n_loc: int, nb: int, keep_fraction: float) -> int:
    """Kept tile diagonals of a DST matrix that keeps keep_fraction of the tiles."""
    w = int(_load().mvg_dst_band(int(n_loc), int(nb), float(keep_fraction)))
    if w < 1:
        raise ValueError("mvg_dst_band: bad arguments")
    return w


def mvg_footprint(n_loc: int, opts=None) -> int:
    o = _opts(opts)
    return int(_load().mvg_footprint(int(n_loc), ctypes.byref(o)))


def mvg_ir_stats(i: int = 0) -> dict:
    """Iterative refinement of the last mixed-precision loglik on this thread, theta i."""
    it, rel, conv = c_int(), c_double(), c_int()
    _check("mvg_ir_stats", _load().mvg_ir_stats(int(i), ctypes.byref(it), ctypes.byref(rel),
                                                 ctypes.byref(conv)))
    return {"iters": it.value, "relres": rel.value, "converged": conv.value == 1,
            "fp64_fallback": conv.value == -1}


class Result(ctypes.Structure):
    _fields_ = [("id", c_int64), ("kind", c_int), ("status", c_int), ("n_loc", c_int64),
                ("loglik", c_double), ("logdet", c_double), ("quad", c_double),
                ("t_arrive", c_double), ("t_start", c_double), ("t_end", c_double),
                ("batch", c_int), ("cache_hit", c_int), ("precision", c_int)]


REQ_LOGLIK, REQ_COKRIGE = 0, 1


class Server:
    """Request server of the library (footprint admission, concurrent
    workers, continuous batching of small likelihoods, resident factors).
    Datasets and cokriging buffers must stay alive while requests use them;
    this wrapper keeps references to them."""

    def __init__(self, hbm_budget_bytes: int, n_workers: int = 4, opts=None):
        self._o = _opts(opts)
        h = _load().mvg_server_create(int(hbm_budget_bytes), int(n_workers), ctypes.byref(self._o))
        if not h:
            raise MvgError("mvg_server_create", -1, "bad arguments")
        self._h = c_void_p(h)
        self._keep = []

    def add_dataset(self, x, y, z) -> int:
        r = _load().mvg_server_add_dataset(self._h, _dev_f64(x, "x"), _dev_f64(y, "y"),
                                           _dev_f64(z, "z"), x.numel())
        if r < 0:
            raise MvgError("mvg_server_add_dataset", r, "")
        self._keep.append((x, y, z))
        return r

    def submit(self, kind, dataset, theta, x0=None, y0=None, zhat=None, t_arrive=-1.0) -> int:
        th = Theta.of(theta)
        m = 0 if x0 is None else x0.numel()
        args = (None, None, None) if x0 is None else (_dev_f64(x0, "x0"), _dev_f64(y0, "y0"),
                                                      c_void_p(zhat.data_ptr()))
        if x0 is not None:
            self._keep.append((x0, y0, zhat))
        r = _load().mvg_server_submit(self._h, int(kind), int(dataset), ctypes.byref(th), args[0],
                                      args[1], m, args[2], float(t_arrive))
        if r < 0:
            raise MvgError("mvg_server_submit", int(r), "")
        return int(r)

    def poll(self, max_results=256, wait_ms=100):
        buf = (Result * max_results)()
        k = _load().mvg_server_poll(self._h, buf, max_results, int(wait_ms))
        return [buf[i] for i in range(k)]

    def clock(self) -> float:
        return _load().mvg_server_clock(self._h)

    def stats(self) -> dict:
        h, m, b, c = c_int64(), c_int64(), c_int64(), ctypes.c_size_t()
        _load().mvg_server_stats(self._h, ctypes.byref(h), ctypes.byref(m), ctypes.byref(b),
                                 ctypes.byref(c))
        return {"hits": h.value, "misses": m.value, "batches": b.value, "cached_bytes": c.value}

    def close(self):
        if self._h:
            _load().mvg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
