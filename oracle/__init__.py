"""CPU oracle for block orthonormalization -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the GPU library and never imports it.

Python front end over ``oracle.c`` (plain C, gcc, binary128 and Dekker
double-double).  See the C file's header for what each routine computes and
which part of the paper (Sec. 4.2) it follows.

Functions (all arrays row-major float64 numpy arrays):

* gram_q(A, B)            exact A^T B (binary128 sums) as (hi, lo)
* gram_dot2(A, B)         A^T B by Ogita-Rump-Oishi Dot2 as (hi, lo)
* gram_f64(A, B)          A^T B in binary64, fixed row-block partition
* chol_q(G_hi, G_lo)      binary128 Cholesky -> (R_hi, R_lo, info)
* trinv_q(R_hi, R_lo)     binary128 inverse of upper-triangular R
* update_q(X, Z, Y, C)    (X - Y C) Z in binary128, rounded once
* qr_q(X, Y)              exact thin QR of (I - Y Y^T) X  (O1)
* cholqr_steps(X, Y, ...) the paper's steps in binary64 / DD      (O2)
* iterate(X, Y, ...)      the iterated scheme (Cholesky / SVQB)   (O2)
* kappa_true(X, Y)        kappa from the exact Gram matrix        (O1)
* svqb_q(M_hi, M_lo)      M^{-1/2} by binary128 Jacobi
* metrics(Q, X, R, Y, C)  omega, rho, omega_Y, ||X||_F
* gram_split_bf16(X32)    split-BF16 Gram model
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB = _HERE / "_liboracle.so"
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64 = ctypes.c_int64
_int = ctypes.c_int


def build(force: bool = True) -> Path:
    """Compile oracle.c into _liboracle.so (gcc, no fast-math, no contraction)."""
    if force or not _LIB.exists():
        tmp = _LIB.with_suffix(".so.tmp")
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", str(tmp), str(_SRC), "-lquadmath", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
            build(force=True)
        lib = ctypes.CDLL(str(_LIB))
        sig = {
            "or_num_threads": ([], _int),
            "or_set_num_threads": ([_int], None),
            "or_gram_q": ([_i64, _int, _dp, _i64, _int, _dp, _i64, _dp, _dp], _int),
            "or_gram_dot2": ([_i64, _int, _dp, _i64, _int, _dp, _i64, _dp, _dp], _int),
            "or_gram_f64": ([_i64, _int, _dp, _i64, _int, _dp, _i64, _dp], _int),
            "or_gram_w_q": ([_i64, _int, _dp, _i64, _int, _dp, _i64, _dp, _dp, _dp], _int),
            "or_chol_q": ([_int, _dp, _dp, _dp, _dp], _int),
            "or_trinv_q": ([_int, _dp, _dp, _dp, _dp], _int),
            "or_update_q": ([_i64, _int, _dp, _i64, _int, _dp, _i64, _dp, _dp, _dp,
                             _dp, _i64], _int),
            "or_qr_q": ([_i64, _int, _dp, _i64, _int, _dp, _i64, _dp, _i64, _dp, _dp,
                         _dp, _dp], _int),
            "or_svqb_q": ([_int, _dp, _dp, _dp, _dp], _int),
            "or_cholqr_steps": ([_i64, _int, _dp, _i64, _int, _dp, _i64, _int, _int, _int,
                                 _int, _dp, _i64, _dp, _dp, _dp, _dp], _int),
            "or_iterate": ([_i64, _int, _dp, _i64, _int, _dp, _i64, _int, _int, _int,
                            ctypes.c_double, _int, _dp, _i64, _dp, _dp, _dp, _dp, _dp], _int),
            "or_metrics": ([_i64, _int, _dp, _i64, _dp, _i64, _int, _dp, _i64, _dp,
                            _dp, _dp, _dp], _int),
            "or_gram_split_bf16": ([_i64, _int, _fp, _i64, _i64, _dp], _int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _c(a, dtype=np.float64):
    a = np.asarray(a, dtype=dtype)
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    return np.ascontiguousarray(a)


def _p(a):
    return None if a is None else a.ctypes.data_as(_dp)


def num_threads() -> int:
    return _load().or_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (its results do not depend on
    the count: every sum runs over a fixed row-block partition)."""
    _load().or_set_num_threads(int(n))


def gram_q(A, B=None):
    """Exact A^T B: binary128 accumulation, returned as (hi, lo) float64."""
    A = _c(A)
    B = A if B is None else _c(B)
    m, ka = A.shape
    kb = B.shape[1]
    hi = np.empty((ka, kb))
    lo = np.empty((ka, kb))
    _load().or_gram_q(m, ka, _p(A), ka, kb, _p(B), kb, _p(hi), _p(lo))
    return hi, lo


def gram_w_q(A, w, B=None):
    """Exact A^T diag(w) B (B-inner products): binary128 accumulation, as
    (hi, lo) float64."""
    A = _c(A)
    B = A if B is None else _c(B)
    w = _c(np.asarray(w, dtype=np.float64).reshape(-1))
    m, ka = A.shape
    kb = B.shape[1]
    if w.shape[0] != m or B.shape[0] != m:
        raise ValueError("row counts differ")
    ghi = np.zeros((ka, kb))
    glo = np.zeros((ka, kb))
    _load().or_gram_w_q(m, ka, _p(A), ka, kb, _p(B), kb, _p(w), _p(ghi), _p(glo))
    return ghi, glo


def metrics_b(Q, X, R, w, Y=None, C=None):
    """B-inner-product measures, B = diag(w): omega_B = ||Q^T B Q - I||_F,
    omega_Y = ||Y^T B Q||_F (binary128 Gram matrices), rho as in metrics."""
    k = Q.shape[1]
    ghi, glo = gram_w_q(Q, w)
    om = float(np.linalg.norm((ghi - np.eye(k)) + glo))
    omy = 0.0
    if Y is not None and Y.shape[1] > 0:
        yhi, ylo = gram_w_q(Y, w, Q)
        omy = float(np.linalg.norm(yhi + ylo))
    rho = metrics(Q, X, R, Y, C)["rho"]
    return {"omega": om, "omega_y": omy, "rho": rho}


def gram_dot2(A, B=None):
    """A^T B by Dot2 (Dekker TwoProduct + TwoSum), as (hi, lo)."""
    A = _c(A)
    B = A if B is None else _c(B)
    m, ka = A.shape
    kb = B.shape[1]
    hi = np.empty((ka, kb))
    lo = np.empty((ka, kb))
    _load().or_gram_dot2(m, ka, _p(A), ka, kb, _p(B), kb, _p(hi), _p(lo))
    return hi, lo


def gram_f64(A, B=None):
    A = _c(A)
    B = A if B is None else _c(B)
    m, ka = A.shape
    kb = B.shape[1]
    g = np.empty((ka, kb))
    _load().or_gram_f64(m, ka, _p(A), ka, kb, _p(B), kb, _p(g))
    return g


def chol_q(ghi, glo=None):
    """binary128 Cholesky G = R^T R (R upper).  Returns (R_hi, R_lo, info)."""
    ghi = _c(ghi)
    k = ghi.shape[0]
    glo = None if glo is None else _c(glo)
    rhi = np.zeros((k, k))
    rlo = np.zeros((k, k))
    info = _load().or_chol_q(k, _p(ghi), _p(glo), _p(rhi), _p(rlo))
    return rhi, rlo, info


def trinv_q(rhi, rlo=None):
    rhi = _c(rhi)
    k = rhi.shape[0]
    rlo = None if rlo is None else _c(rlo)
    zhi = np.zeros((k, k))
    zlo = np.zeros((k, k))
    info = _load().or_trinv_q(k, _p(rhi), _p(rlo), _p(zhi), _p(zlo))
    if info:
        raise ZeroDivisionError(f"zero diagonal at {info}")
    return zhi, zlo


def update_q(X, Z, Y=None, C_hi=None, C_lo=None):
    """(X - Y C) Z evaluated in binary128, rounded once to float64."""
    X = _c(X)
    Z = _c(Z)
    m, k = X.shape
    ky = 0 if Y is None else Y.shape[1]
    Yc = _c(Y) if ky else np.zeros((1, 1))
    ch = _c(C_hi) if ky else np.zeros((1, 1))
    cl = None if (C_lo is None or not ky) else _c(C_lo)
    Q = np.empty((m, k))
    _load().or_update_q(m, k, _p(X), k, ky, _p(Yc), max(ky, 1), _p(ch), _p(cl), _p(Z),
                        _p(Q), k)
    return Q


def qr_q(X, Y=None, want_gram=False):
    """O1: exact thin QR of Xt = (I - Y Y^T) X.

    Returns dict(Q, R, C, info[, G_hi, G_lo]).  R has a positive diagonal."""
    X = _c(X)
    m, k = X.shape
    ky = 0 if Y is None else Y.shape[1]
    Yc = _c(Y) if ky else np.zeros((1, 1))
    Q = np.zeros((m, k))
    R = np.zeros((k, k))
    C = np.zeros((max(ky, 1), k))
    ghi = np.zeros((k, k)) if want_gram else None
    glo = np.zeros((k, k)) if want_gram else None
    info = _load().or_qr_q(m, k, _p(X), k, ky, _p(Yc), max(ky, 1), _p(Q), k, _p(R),
                           _p(C), _p(ghi), _p(glo))
    out = dict(Q=Q, R=R, C=C[:ky], info=info)
    if want_gram:
        out["G_hi"] = ghi
        out["G_lo"] = glo
    return out


def cholqr_steps(X, Y=None, *, dd_first=False, passes=2, project_each_pass=True,
                 dd_corrected=False, exact_gram=False):
    """O2: the paper's two-phase steps, first pass in DD if ``dd_first``
    (``dd_corrected``: with the projection coefficients D = 2C - S C, S = Y^T Y,
    which remove the part in span(Y) to second order in ||S - I||).
    ``exact_gram`` (binary64 first pass only): that pass is given the
    binary128 Gram matrix rounded once to binary64 instead of a binary64 sum.

    Returns dict(Q, R_hi, R_lo, C_hi, C_lo, info) with X = Y C + Q R;
    info = 100*(pass+1) + pivot on Cholesky breakdown, else 0."""
    X = _c(X)
    m, k = X.shape
    ky = 0 if Y is None else Y.shape[1]
    Yc = _c(Y) if ky else np.zeros((1, 1))
    Q = np.zeros((m, k))
    rhi = np.zeros((k, k))
    rlo = np.zeros((k, k))
    chi = np.zeros((max(ky, 1), k))
    clo = np.zeros((max(ky, 1), k))
    info = _load().or_cholqr_steps(m, k, _p(X), k, ky, _p(Yc), max(ky, 1),
                                   2 if (exact_gram and not dd_first) else int(bool(dd_first)),
                                   int(bool(dd_corrected)), int(passes),
                                   int(bool(project_each_pass)), _p(Q), k, _p(rhi),
                                   _p(rlo), _p(chi), _p(clo))
    return dict(Q=Q, R_hi=rhi, R_lo=rlo, C_hi=chi[:ky], C_lo=clo[:ky], info=info)


def iterate(X, Y=None, *, gram="f64", fact="chol", eps=1e-10, max_iter=5, fused=False):
    """O2 iterated scheme: passes of projection against Y and Cholesky or
    symmetric-SVQB orthonormalization (binary64, or DD Gram and factor),
    until ||C_j||_F <= eps and ||R_j - I||_F <= eps or max_iter passes.
    ``fused``: each pass takes M from the Gram matrix of [Y | S] of one sweep
    (M = S^T S - C^T (2 C - Y^T Y C)), the fused operations, instead of the
    Gram matrix of the projected block.

    Returns dict(Q, R_hi, R_lo, C_hi, C_lo, passes, converged, c_norm, r_dev,
    info) with X = Y C + Q R; info = 100*pass + pivot on a breakdown, else 0."""
    X = _c(X)
    m, k = X.shape
    ky = 0 if Y is None else Y.shape[1]
    Yc = _c(Y) if ky else np.zeros((1, 1))
    Q = np.zeros((m, k))
    rhi = np.zeros((k, k))
    rlo = np.zeros((k, k))
    chi = np.zeros((max(ky, 1), k))
    clo = np.zeros((max(ky, 1), k))
    out = np.zeros(4)
    info = _load().or_iterate(m, k, _p(X), k, ky, _p(Yc), max(ky, 1), 1 if gram == "dd" else 0,
                              1 if fact == "svqb" else 0, int(bool(fused)), float(eps),
                              int(max_iter), _p(Q), k,
                              _p(rhi), _p(rlo), _p(chi), _p(clo), _p(out))
    return dict(Q=Q, R_hi=rhi, R_lo=rlo, C_hi=chi[:ky], C_lo=clo[:ky], passes=int(out[0]),
                converged=bool(out[1]), c_norm=float(out[2]), r_dev=float(out[3]), info=info)


def kappa_true(X, Y=None):
    """kappa of the (projected) block from its exact Gram matrix:
    sqrt(lambda_max / lambda_min) of the binary128 Gram matrix of
    Xt = X - Y (Y^T X), eigenvalues by binary128 Jacobi."""
    o = qr_q(X, Y, want_gram=True)
    _, lam, info = svqb_q(o["G_hi"], o["G_lo"])
    if info or not lam[0] > 0:
        return float("inf")
    return float(np.sqrt(lam[-1] / lam[0]))


def svqb_q(mhi, mlo=None):
    """Symmetric SVQB transform Z = M^{-1/2} (binary128 Jacobi).

    Returns (Z, eigenvalues ascending, info)."""
    mhi = _c(mhi)
    k = mhi.shape[0]
    mlo = None if mlo is None else _c(mlo)
    Z = np.zeros((k, k))
    lam = np.zeros(k)
    info = _load().or_svqb_q(k, _p(mhi), _p(mlo), _p(Z), _p(lam))
    return Z, lam, info


def metrics(Q, X, R, Y=None, C=None, want_E=False):
    """omega = ||Q^T Q - I||_F, rho = ||X - Y C - Q R||_F / ||X||_F,
    omega_Y = ||Y^T Q||_F, normX = ||X||_F, all accurate to ~u^2."""
    Q = _c(Q)
    X = _c(X)
    R = _c(R)
    m, k = Q.shape
    ky = 0 if Y is None else Y.shape[1]
    Yc = _c(Y) if ky else np.zeros((1, 1))
    Cc = _c(C) if ky else np.zeros((1, 1))
    out = np.zeros(4)
    E = np.zeros((k, k)) if want_E else None
    _load().or_metrics(m, k, _p(Q), k, _p(X), k, ky, _p(Yc), max(ky, 1), _p(R), _p(Cc),
                       _p(out), _p(E))
    res = dict(omega=out[0], rho=out[1], omega_y=out[2], norm_x=out[3])
    if want_E:
        res["E"] = E
    return res


def gram_split_bf16(X32, chunk=256):
    """Model of the split-BF16 Gram (see oracle.c), float64 result."""
    X32 = np.ascontiguousarray(np.asarray(X32, dtype=np.float32))
    m, k = X32.shape
    G = np.zeros((k, k))
    _load().or_gram_split_bf16(m, k, X32.ctypes.data_as(_fp), k, int(chunk), _p(G))
    return G
