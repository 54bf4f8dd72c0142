"""Plain FP64 CPU oracle for the bivariate parsimonious-Matern likelihood path.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It never imports
the GPU package and the GPU package never imports it; the two share only the
seeded input generators in ``synthetic/``.

Each function states the passage of the paper it follows:

* ``gamma``, ``bessel_k``, ``matern`` -- the special functions inside Eq. (2)
  (Section 4.2); the paper gives no evaluation method, the methods used are
  named in ``oracle.c``.
* ``theta_scalars`` / ``rho12`` -- Section 4.2, colocated correlation.
* ``cov_dense`` / ``cov_entries`` -- Eq. (2) laid out as Representation I
  (Section 5.2).
* ``potrf`` / ``trsv_lower`` -- the Cholesky factorisation (Section 5.2).
* ``loglik`` -- Eq. (1).
* ``cokrige`` -- Eq. (3)-(4), with the predictor MSE of Eq. (5).
* ``morton_order`` -- the Morton (Z-order) ordering of Section 5.3.
* ``tlr_truncate_tiles`` -- the per-tile SVD truncation of Section 5.3 (dense
  SVD, a library primitive), used to separate compression error from
  factorisation error.
* ``round_to`` -- emulation of FP32 / BF16 round-to-nearest-even, used to size
  the mixed-precision error.
* ``cross_cov_targets`` / ``mloe_mmom`` -- the multivariate prediction
  efficiency criteria of Section 5.4 (Eq. (5)-(8), Algorithm 1).
* ``theta_p_check`` / ``rho_p`` / ``cov_dense_p`` / ``loglik_p`` /
  ``profile_loglik_p`` -- the parsimonious multivariate Matern for p
  variables (Section 4.2, Eq. (1)-(2)) and the profile likelihood of
  Section 5.2.
* ``dst_band`` / ``dst_mask`` -- the Diagonal Super Tile approximation
  (Section 4.4; "DST 40/60" and "DST 70/30" of Experiment 2, Section 6.4.1):
  the tiles far from the diagonal set to zero.
* ``mixed_cholesky_emulated`` -- not in the paper: the mixed-precision tiled
  factorisation (FP64 band, FP32 / BF16 / split-BF16 off the band) emulated
  in FP64 with
  rounding at the operand points, to predict the size of its error (not its
  bits).  Pinned by the defining equations of its rounding points: band
  blocks reproduce S to FP64 rounding, off-band blocks deviate at the
  operand precision's scale, FP64-storage panel tiles solve their Schur
  complement in FP64 (``tests/test_oracle.py``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-fno-fast-math", _SRC, "-o", _SO + ".tmp", "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(_SO + ".tmp", _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build(force=True)
    lib = ctypes.CDLL(_SO)
    D, I64, I = ctypes.c_double, ctypes.c_int64, ctypes.c_int
    P = ctypes.c_void_p
    sig = {
        "orc_rgamma1p": (D, [D]),
        "orc_gamma": (D, [D]),
        "orc_bessel_k": (D, [D, D]),
        "orc_matern": (D, [D, D]),
        "orc_theta_check": (I, [P]),
        "orc_rho12": (D, [P]),
        "orc_cross_cov": (D, [P, I, I, D]),
        "orc_cov_entries": (None, [P, P, P, P, P, I64, P]),
        "orc_cov_dense": (None, [P, P, I64, P, P]),
        "orc_potrf": (I64, [P, I64]),
        "orc_trsv_lower": (None, [P, I64, P]),
        "orc_trsv_lower_trans": (None, [P, I64, P]),
        "orc_loglik": (I64, [P, P, P, I64, P, P]),
        "orc_cokrige": (I64, [P, P, P, I64, P, P, P, I64, P, P]),
        "orc_num_threads": (I, []),
        "orc_bessel_k_vec": (None, [D, P, I64, P]),
        "orc_matern_vec": (None, [D, P, I64, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _theta(theta):
    t = _f64(theta).reshape(-1)
    if t.size != 6:
        raise ValueError("theta must be (sigma11^2, sigma22^2, a, nu11, nu22, beta)")
    return t


def num_threads() -> int:
    return int(_load().orc_num_threads())


# ----------------------------------------------------------- special functions

def rgamma1p(z: float) -> float:
    """1/Gamma(1+z) for |z| <= 1/2."""
    return float(_load().orc_rgamma1p(float(z)))


def gamma(x: float) -> float:
    """Gamma(x), x > 0."""
    return float(_load().orc_gamma(float(x)))


def bessel_k(nu: float, x) -> np.ndarray:
    """Modified Bessel function of the second kind K_nu(x), x > 0."""
    xa = _f64(np.atleast_1d(x))
    out = np.empty_like(xa)
    _load().orc_bessel_k_vec(float(nu), _ptr(xa), xa.size, _ptr(out))
    return out


def matern(x, nu: float) -> np.ndarray:
    """M(x; nu) = x^nu K_nu(x) / (2^(nu-1) Gamma(nu)), M(0; nu) = 1 (Eq. 2)."""
    xa = _f64(np.atleast_1d(x))
    out = np.empty_like(xa)
    _load().orc_matern_vec(float(nu), _ptr(xa), xa.size, _ptr(out))
    return out


# ---------------------------------------------------------------------- theta

def theta_check(theta) -> int:
    """0 if theta is admissible, else -(1-based index of the offending entry)."""
    t = _theta(theta)
    return int(_load().orc_theta_check(_ptr(t)))


def rho12(theta) -> float:
    """Colocated correlation rho_12 (Section 4.2, d = 2)."""
    t = _theta(theta)
    return float(_load().orc_rho12(_ptr(t)))


def cross_cov(theta, i: int, j: int, h: float) -> float:
    """C_ij(h), 0-based i, j (Eq. 2)."""
    t = _theta(theta)
    return float(_load().orc_cross_cov(_ptr(t), int(i), int(j), float(h)))


# ------------------------------------------------------------------ covariance

def cov_dense(x, y, theta) -> np.ndarray:
    """Dense 2n x 2n Sigma in Representation I (Section 5.2)."""
    xa, ya, t = _f64(x), _f64(y), _theta(theta)
    n = xa.size
    S = np.empty((2 * n, 2 * n), dtype=np.float64)
    _load().orc_cov_dense(_ptr(xa), _ptr(ya), n, _ptr(t), _ptr(S))
    return S


def cov_entries(x, y, theta, rows, cols) -> np.ndarray:
    """Sigma[rows[t], cols[t]] one by one (0-based)."""
    xa, ya, t = _f64(x), _f64(y), _theta(theta)
    r = np.ascontiguousarray(rows, dtype=np.int64)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.empty(r.size, dtype=np.float64)
    _load().orc_cov_entries(_ptr(xa), _ptr(ya), _ptr(t), _ptr(r), _ptr(c), r.size, _ptr(out))
    return out


# -------------------------------------------------------------- linear algebra

def potrf(A):
    """Lower Cholesky factor of a dense SPD matrix; returns (L, info)."""
    L = np.array(A, dtype=np.float64, order="C", copy=True)
    info = int(_load().orc_potrf(_ptr(L), L.shape[0]))
    return L, info


def trsv_lower(L, b, trans: bool = False) -> np.ndarray:
    """L^-1 b, or L^-T b with trans=True."""
    La = _f64(L)
    out = _f64(b).copy()
    fn = _load().orc_trsv_lower_trans if trans else _load().orc_trsv_lower
    fn(_ptr(La), La.shape[0], _ptr(out))
    return out


# ------------------------------------------------------------------ likelihood

def loglik(x, y, z, theta) -> dict:
    """Eq. (1): {'loglik', 'logdet', 'quad', 'info'}; loglik = -inf if Sigma is
    not positive definite (info = 1-based first failing pivot)."""
    xa, ya, za, t = _f64(x), _f64(y), _f64(z), _theta(theta)
    n = xa.size
    if za.size != 2 * n:
        raise ValueError("z must have 2n entries (Representation I)")
    out = np.zeros(3, dtype=np.float64)
    info = int(_load().orc_loglik(_ptr(xa), _ptr(ya), _ptr(za), n, _ptr(t), _ptr(out)))
    if info < 0:
        raise ValueError("invalid theta (code %d)" % info)
    return {"loglik": float(out[0]), "logdet": float(out[1]), "quad": float(out[2]),
            "info": info}


def cokrige(x, y, z, theta, x0, y0, with_mse: bool = False):
    """Eq. (3)-(4): predictions (m, 2); with_mse adds the Eq. (5) MSE per target."""
    xa, ya, za, t = _f64(x), _f64(y), _f64(z), _theta(theta)
    x0a, y0a = _f64(x0), _f64(y0)
    n, m = xa.size, x0a.size
    zhat = np.empty(2 * m, dtype=np.float64)
    mse = np.empty(m, dtype=np.float64) if with_mse else None
    info = int(_load().orc_cokrige(_ptr(xa), _ptr(ya), _ptr(za), n, _ptr(t), _ptr(x0a),
                                   _ptr(y0a), m, _ptr(zhat),
                                   _ptr(mse) if with_mse else None))
    if info != 0:
        raise ValueError("cokrige failed (code %d)" % info)
    zhat = zhat.reshape(m, 2)
    return (zhat, mse) if with_mse else zhat


def simulate_z(x, y, theta, eps) -> np.ndarray:
    """Z = L eps with L the oracle Cholesky factor of Sigma(theta) (data
    generation for the likelihood workloads)."""
    L, info = potrf(cov_dense(x, y, theta))
    if info:
        raise ValueError("Sigma(theta) is not positive definite (pivot %d)" % info)
    return L @ _f64(eps)


# --------------------------------------------------------------------- ordering

def morton_keys(x, y) -> np.ndarray:
    """Z-order keys: floor(coord * 2^16) clamped to [0, 2^16 - 1], x bits at even
    and y bits at odd positions (Section 5.3 names the ordering; the
    quantisation is this implementation's reading)."""
    qx = np.clip(np.floor(_f64(x) * 65536.0), 0, 65535).astype(np.uint64)
    qy = np.clip(np.floor(_f64(y) * 65536.0), 0, 65535).astype(np.uint64)
    key = np.zeros(qx.shape, dtype=np.uint64)
    for b in range(16):
        key |= ((qx >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b)
        key |= ((qy >> np.uint64(b)) & np.uint64(1)) << np.uint64(2 * b + 1)
    return key


def morton_order(x, y) -> np.ndarray:
    """Permutation sorting locations by Morton key; ties keep input order."""
    return np.argsort(morton_keys(x, y), kind="stable")


# -------------------------------------------------------------- approximations

def tlr_truncate_tiles(S: np.ndarray, nb: int, acc: float, max_rank: int, rule: str = "2norm"):
    """Section 5.3 TLR compression by per-tile SVD: every off-diagonal tile of
    the (padded) matrix keeps the singular triplets with s_i > acc (absolute
    2-norm rule), or, with rule="frobenius", the fewest leading triplets whose
    discarded tail has Frobenius norm <= acc; a tile whose rank would exceed
    max_rank stays dense.  Returns (S_tilde, ranks) with ranks[I, J] (-1 for
    dense tiles)."""
    N = S.shape[0]
    T = (N + nb - 1) // nb
    St = np.array(S, copy=True)
    ranks = np.full((T, T), -1, dtype=np.int64)
    for J in range(T):
        for I in range(J + 1, T):
            r0, r1 = I * nb, min(N, (I + 1) * nb)
            c0, c1 = J * nb, min(N, (J + 1) * nb)
            U, s, Vt = np.linalg.svd(S[r0:r1, c0:c1], full_matrices=False)
            if rule == "2norm":
                k = int(np.sum(s > acc))
            else:
                tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]  # tail[i] = ||s[i:]||
                k = int(np.sum(tail > acc))
            if k > max_rank:
                continue
            ranks[I, J] = k
            blk = (U[:, :k] * s[:k]) @ Vt[:k, :]
            St[r0:r1, c0:c1] = blk
            St[c0:c1, r0:r1] = blk.T
    return St, ranks


def loglik_from_matrix(S: np.ndarray, z) -> dict:
    """Eq. (1) for an explicitly given covariance matrix (oracle Cholesky)."""
    N = S.shape[0]
    L, info = potrf(S)
    if info:
        return {"loglik": float("-inf"), "logdet": float("nan"), "quad": float("nan"),
                "info": info}
    logdet = 2.0 * float(np.sum(np.log(np.diag(L))))
    yv = trsv_lower(L, z)
    q = float(np.dot(yv, yv))
    return {"loglik": -(N / 2.0) * np.log(2.0 * np.pi) - 0.5 * logdet - 0.5 * q,
            "logdet": logdet, "quad": q, "info": 0}


def round_to(a, fmt: str) -> np.ndarray:
    """Round FP64 values to FP32 or BF16 (round to nearest, ties to even) and
    return them as FP64."""
    a = _f64(a)
    if fmt == "fp32":
        return a.astype(np.float32).astype(np.float64)
    if fmt == "bf16":
        f = a.astype(np.float32)
        u = f.view(np.uint32).astype(np.uint64)
        lsb = (u >> np.uint64(16)) & np.uint64(1)
        u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
        return u.astype(np.uint32).view(np.float32).astype(np.float64)
    raise ValueError(fmt)


def mixed_cholesky_emulated(S: np.ndarray, nb: int, band: int, fmt: str, storage: str = "fp32",
                            _plant: str = ""):
    """Not in the paper.  Right-looking tiled Cholesky of S (padded with an
    identity block to a multiple of nb) where the trailing updates of tiles
    (I, J) with I - J >= band take operands rounded to ``fmt`` ("fp32",
    "bf16", "bf16x3", or "fp64" for no rounding), everything else in FP64.

    "bf16x3" (MVG_MIXED_BF16X3) splits each operand value a into
    a_hi = bf16(fp32(a)) and a_lo = bf16(fp32(a) - a_hi) and forms each product
    as a_hi b_hi + a_hi b_lo + a_lo b_hi (the a_lo b_lo term dropped).

    storage "fp32" (MVG_MIXED_FP32 / BF16): those tiles are stored in FP32:

    * off-band tiles start as S rounded to FP32;
    * diagonal tiles: FP64 Cholesky; W_k = L_kk^-1 (FP64);
    * panel tiles within the band: L_ik = A_ik W_k^T in FP64; off the band:
      round32(A_ik round32(W_k)^T);
    * trailing tiles within the band: A_ij -= L_ik L_jk^T in FP64 (the FP32
      panel values upcast exactly); off the band:
      A_ij = round32(A_ij - op(L_ik) op(L_jk)^T), op = round to fmt.

    storage "fp64" (MVG_MIXED_FP32X): every tile stays FP64 and every panel
    tile is solved in FP64; only the off-band trailing products take rounded
    operands: A_ij -= op(L_ik) op(L_jk)^T.

    Products are formed in FP64 and rounded once, so the result predicts the
    size of the mixed-precision error of an FP32-accumulating implementation,
    not its bits.  Returns (L padded, info) with info the 1-based index of the
    first non-positive pivot (0 if none).

    ``_plant`` exists only for the tests that check the pins of this function
    can fail: "band_operands" rounds the operands of band-target updates too,
    "w32" solves off-band panel tiles against round32(W_k) in FP64 storage.
    "x3_hi_only" keeps only a_hi b_hi of a "bf16x3" product.  All three are
    mistakes; the default "" is the definition above."""
    S = _f64(S)
    N = S.shape[0]
    T = (N + nb - 1) // nb
    Np = T * nb
    A = np.eye(Np)
    A[:N, :N] = S
    A = np.tril(A)

    def blk(I, J):
        return slice(I * nb, (I + 1) * nb), slice(J * nb, (J + 1) * nb)

    def op(a):
        if fmt == "fp64":
            return a
        return round_to(a, "fp32") if fmt == "fp32" else round_to(round_to(a, "fp32"), "bf16")

    def lowp_product(Li, Lj):
        """op(L_i) op(L_j)^T, or the three-term product of the BF16 splits."""
        if fmt != "bf16x3":
            return op(Li) @ op(Lj).T
        fi, fj = round_to(Li, "fp32"), round_to(Lj, "fp32")
        hi_i, hi_j = round_to(fi, "bf16"), round_to(fj, "bf16")
        lo_i, lo_j = round_to(fi - hi_i, "bf16"), round_to(fj - hi_j, "bf16")
        if _plant == "x3_hi_only":
            return hi_i @ hi_j.T
        return hi_i @ hi_j.T + hi_i @ lo_j.T + lo_i @ hi_j.T

    if fmt not in ("fp32", "bf16", "bf16x3", "fp64"):
        raise ValueError(fmt)
    if storage not in ("fp32", "fp64"):
        raise ValueError(storage)
    if _plant not in ("", "band_operands", "w32", "x3_hi_only"):
        raise ValueError(_plant)
    low = storage == "fp32"
    if low:
        for J in range(T):
            for I in range(J + band, T):
                A[blk(I, J)] = round_to(A[blk(I, J)], "fp32")
    for k in range(T):
        d = A[blk(k, k)]
        d = np.tril(d) + np.tril(d, -1).T
        Lkk, info = potrf(d)
        if info:
            return A, k * nb + info
        A[blk(k, k)] = Lkk
        W = np.linalg.solve(Lkk, np.eye(nb))
        for i in range(k + 1, T):
            if _plant == "w32" and not low and i - k >= band:
                A[blk(i, k)] = A[blk(i, k)] @ round_to(W, "fp32").T
            elif i - k < band or not low:
                A[blk(i, k)] = A[blk(i, k)] @ W.T
            else:
                A[blk(i, k)] = round_to(A[blk(i, k)] @ round_to(W, "fp32").T, "fp32")
        for j in range(k + 1, T):
            for i in range(j, T):
                Li, Lj = A[blk(i, k)], A[blk(j, k)]
                if i - j < band and _plant == "band_operands":
                    A[blk(i, j)] = A[blk(i, j)] - lowp_product(Li, Lj)
                elif i - j < band:
                    A[blk(i, j)] = A[blk(i, j)] - Li @ Lj.T
                elif low:
                    A[blk(i, j)] = round_to(A[blk(i, j)] - lowp_product(Li, Lj), "fp32")
                else:
                    A[blk(i, j)] = A[blk(i, j)] - lowp_product(Li, Lj)
    return np.tril(A), 0


def cross_cov_targets(x, y, x0, y0, theta) -> np.ndarray:
    """c0 of Eq. (3)-(4) for every target: a 2n x 2m matrix whose columns
    2l + j hold C_ij(||s_r - s0_l||) at rows 2r + i (Representation I)."""
    xa, ya, x0a, y0a = _f64(x), _f64(y), _f64(x0), _f64(y0)
    h = np.sqrt((xa[:, None] - x0a[None, :]) ** 2 + (ya[:, None] - y0a[None, :]) ** 2)
    t = _theta(theta)
    nu12 = 0.5 * (t[3] + t[4])
    c11 = t[0] * matern(h / t[2], t[3])
    c22 = t[1] * matern(h / t[2], t[4])
    c12 = rho12(theta) * np.sqrt(t[0]) * np.sqrt(t[1]) * matern(h / t[2], nu12)
    n, m = h.shape
    c0 = np.empty((2 * n, 2 * m))
    c0[0::2, 0::2] = c11
    c0[1::2, 0::2] = c12
    c0[0::2, 1::2] = c12
    c0[1::2, 1::2] = c22
    return c0


def mloe_mmom(x, y, theta, theta_a, x0, y0) -> dict:
    """Section 5.4: per target s0, E_t (Eq. 5 with the true theta), E_a (Eq. 5
    with the approximate model's theta_a) and E_{t,a} (Eq. 6), then
    LOE = E_{t,a}/E_t - 1 and MOM = E_a/E_{t,a} - 1 and their means (Eq. 7-8),
    following Algorithm 1 with the oracle's own Cholesky factors and
    triangular solves."""
    S, Sa = cov_dense(x, y, theta), cov_dense(x, y, theta_a)
    L, info = potrf(S)
    La, info_a = potrf(Sa)
    if info or info_a:
        raise ValueError("covariance not positive definite")
    c0t = cross_cov_targets(x, y, x0, y0, theta)
    c0a = cross_cov_targets(x, y, x0, y0, theta_a)
    t, ta = _theta(theta), _theta(theta_a)
    tr_t, tr_a = t[0] + t[1], ta[0] + ta[1]
    m = c0t.shape[1] // 2
    loe, mom = np.empty(m), np.empty(m)
    for l in range(m):
        et = tr_t
        ea = tr_a
        eta = tr_t
        for j in (2 * l, 2 * l + 1):
            ut = trsv_lower(L, c0t[:, j])                    # L^-1 c0_t
            ua = trsv_lower(La, c0a[:, j])                   # L_a^-1 c0_a
            wa = trsv_lower(La, ua, trans=True)              # Sigma_a^-1 c0_a
            et -= float(np.dot(ut, ut))
            ea -= float(np.dot(ua, ua))
            lw = L.T @ wa                                    # L^T w_a
            eta += -2.0 * float(np.dot(c0t[:, j], wa)) + float(np.dot(lw, lw))
        loe[l] = eta / et - 1.0
        mom[l] = ea / eta - 1.0
    return {"mloe": float(np.mean(loe)), "mmom": float(np.mean(mom)), "loe": loe, "mom": mom}


def dst_band(T: int, keep: float) -> int:
    """Section 6.4.1, Experiment 2: "DST 40/60" keeps the 40 % of the tiles
    nearest the diagonal.  Reading: of the T x T tiles, those with
    |I - J| < w are kept, w the smallest band whose tile count reaches
    keep * T * T (counted tile by tile)."""
    need = keep * T * T
    kept = 0
    for w in range(1, T + 1):
        d = w - 1                      # tile diagonal |I - J| = d joins the band
        kept += T if d == 0 else 2 * (T - d)
        if kept >= need:
            return w
    return T


def dst_mask(S: np.ndarray, nb: int, band: int) -> np.ndarray:
    """Section 4.4: the DST matrix, entries of the nb x nb tiles (I, J) with
    |I - J| >= band annihilated."""
    out = np.array(S, dtype=np.float64, copy=True)
    N = out.shape[0]
    for r in range(N):
        for c in range(N):
            if abs(r // nb - c // nb) >= band:
                out[r, c] = 0.0
    return out


# ------------------------------------------------------------ p variables

def _theta_p(th):
    sig = np.asarray(th["sigma_sq"], dtype=np.float64).ravel()
    p = sig.size
    nu = np.asarray(th["nu"], dtype=np.float64).ravel()
    beta = np.asarray(th["beta"], dtype=np.float64).reshape(p, p)
    return p, sig, float(th["a"]), nu, beta


def theta_p_check(th) -> int:
    """Section 4.2: sigma_ii^2 > 0, a > 0, nu_ii > 0 (<= 5 as for p = 2) and
    (beta_ij) a symmetric positive definite correlation matrix.  0 or a
    negative code (-1 p, -2 variances, -3 range, -4 smoothness, -5 beta)."""
    p, sig, a, nu, beta = _theta_p(th)
    if not 1 <= p <= 4 or nu.size != p:
        return -1
    if not np.all(sig > 0):
        return -2
    if not a > 0:
        return -3
    if not np.all((nu > 0) & (nu <= 5)):
        return -4
    if not np.array_equal(beta, beta.T) or not np.all(np.diag(beta) == 1.0):
        return -5
    if np.min(np.linalg.eigvalsh(beta)) <= 0:
        return -5
    return 0


def rho_p(th) -> np.ndarray:
    """Colocated correlations rho_ij of Section 4.2 for d = 2, from the Gamma
    function itself (the third factor read without the square root, as for
    p = 2); rho_ii = 1."""
    p, sig, a, nu, beta = _theta_p(th)
    r = np.empty((p, p))
    for i in range(p):
        for j in range(p):
            nij = 0.5 * (nu[i] + nu[j])
            r[i, j] = (beta[i, j] * np.sqrt(gamma(nu[i] + 1.0) / gamma(nu[i]))
                       * np.sqrt(gamma(nu[j] + 1.0) / gamma(nu[j])) * gamma(nij) / gamma(nij + 1.0))
    return r


def cov_dense_p(x, y, th) -> np.ndarray:
    """Sigma of the p-variate model in Representation I (Section 5.2):
    entry (p l + i, p r + j) = rho_ij sigma_i sigma_j M(||s_l - s_r|| / a; nu_ij)."""
    if theta_p_check(th):
        raise ValueError("invalid theta_p")
    p, sig, a, nu, beta = _theta_p(th)
    xa, ya = _f64(x), _f64(y)
    n = xa.size
    h = np.sqrt((xa[:, None] - xa[None, :]) ** 2 + (ya[:, None] - ya[None, :]) ** 2)
    rho = rho_p(th)
    S = np.empty((p * n, p * n))
    for i in range(p):
        for j in range(p):
            M = matern(h.ravel() / a, 0.5 * (nu[i] + nu[j])).reshape(n, n)
            S[i::p, j::p] = rho[i, j] * np.sqrt(sig[i]) * np.sqrt(sig[j]) * M
    return S


def loglik_p(x, y, z, th) -> dict:
    """Eq. (1) for p variables (-(p n / 2) log 2 pi - log|Sigma| / 2 - q / 2)."""
    return loglik_from_matrix(cov_dense_p(x, y, th), z)


def profile_loglik_p(x, y, z, th) -> dict:
    """Section 5.2: sigma_ii^2 = n^-1 Z_i^T R_ii^-1 Z_i with R_ii the
    correlation matrix of variable i alone (unit variance, nu_ii, a), then
    Eq. (1) at theta with those variances."""
    p, sig, a, nu, beta = _theta_p(th)
    za = _f64(z)
    n = za.size // p
    s_hat = np.empty(p)
    for i in range(p):
        R = cov_dense_p(x, y, {"sigma_sq": [1.0], "a": a, "nu": [nu[i]], "beta": [[1.0]]})
        L, info = potrf(R)
        if info:
            raise ValueError("R_%d%d not positive definite" % (i + 1, i + 1))
        u = trsv_lower(L, za[i::p])
        s_hat[i] = float(np.dot(u, u)) / n
    full = dict(th)
    full["sigma_sq"] = list(s_hat)
    out = loglik_p(x, y, z, full)
    out["sigma_sq"] = s_hat
    return out
