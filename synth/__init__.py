"""Seeded synthetic inputs for block orthonormalization.

This module only *draws* matrices; it holds none of the orthonormalization
arithmetic.  Both the CPU oracle and the GPU path are fed from here, so the
same seed gives the same bytes to both sides.

The paper (Sec. 4.2, Fig. 7 and Fig. 8) uses synthetic X with a prescribed
condition number but does not say how they are built.  The recipe used here:

* U (m x k) and V (k x k) are Haar-distributed orthonormal matrices: a seeded
  Gaussian matrix is factored with LAPACK's Householder QR and each column is
  multiplied by the sign of the matching diagonal entry of R (Mezzadri 2007).
* sigma_i = kappa ** (-(i-1)/(k-1)), i = 1..k (log-spaced from 1 down to 1/kappa).
* X = U diag(sigma) V^T, formed in float64 (optionally rounded to float32).
* The locked basis Y is another Haar matrix, drawn independently.

For the full-size benchmark blocks (tens of GB) the same recipe runs on the
GPU with torch's seeded Philox generator (``svd_matrix_device``): same
distribution, different random stream from the numpy one, so those inputs are
checked through properties (orthogonality, residual) rather than against the
oracle element by element.

Exact families (Sylvester-Hadamard columns) are provided for bitwise tests:
with m = 4**j rows, column c of the normalized Hadamard matrix has entries
(-1)**popcount(i & c) * 2**-j, which are exactly orthonormal in binary64.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar",
    "sigma_logspace",
    "svd_matrix",
    "locked_basis",
    "hadamard_columns",
    "hadamard_scaled",
    "hadamard_near_parallel",
    "batch_table",
    "projected_pair",
    "svd_matrix_device",
    "locked_basis_device",
    "projected_pair_device",
    "b_weighted_pair",
]


def haar(rng: np.random.Generator, m: int, k: int) -> np.ndarray:
    """Haar-distributed m x k matrix with orthonormal columns (m >= k)."""
    if k == 0:
        return np.zeros((m, 0))
    g = rng.standard_normal((m, k))
    q, r = np.linalg.qr(g, mode="reduced")
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    q *= s[None, :]
    return np.ascontiguousarray(q)


def sigma_logspace(k: int, kappa: float) -> np.ndarray:
    if k == 1:
        return np.ones(1)
    i = np.arange(k, dtype=np.float64)
    return np.power(float(kappa), -i / (k - 1))


def svd_matrix(m: int, k: int, kappa: float, seed: int,
               dtype=np.float64) -> np.ndarray:
    """X = U diag(sigma) V^T with Haar U (m x k), Haar V (k x k).

    U is drawn first, then V, from ``numpy.random.default_rng(seed)``.
    """
    rng = np.random.default_rng(seed)
    u = haar(rng, m, k)
    v = haar(rng, k, k)
    x = (u * sigma_logspace(k, kappa)[None, :]) @ v.T
    del u
    x = np.ascontiguousarray(x)
    if dtype != np.float64:
        x = np.ascontiguousarray(x.astype(dtype))
    return x


def locked_basis(m: int, ky: int, seed: int) -> np.ndarray:
    """Orthonormal m x ky locked basis Y (Haar), seeded independently of X."""
    rng = np.random.default_rng(seed)
    return haar(rng, m, ky)


def hadamard_columns(j: int, cols) -> np.ndarray:
    """Columns ``cols`` of the normalized Sylvester-Hadamard matrix of order 4**j.

    Entry (i, c) = (-1)**popcount(i & c) * 2**-j; exact in binary64.
    """
    m = 4 ** j
    i = np.arange(m, dtype=np.uint64)[:, None]
    c = np.asarray(cols, dtype=np.uint64)[None, :]
    v = i & c
    # popcount parity
    par = np.zeros(v.shape, dtype=np.uint64)
    while np.any(v):
        par ^= v & np.uint64(1)
        v = v >> np.uint64(1)
    out = np.where(par == 1, -1.0, 1.0) * np.ldexp(1.0, -j)
    return np.ascontiguousarray(out)


def hadamard_scaled(j: int, exps, first_col: int = 1) -> np.ndarray:
    """X = H[:, cols] diag(2**e_c): exact QR is Q = H[:, cols], R = diag(2**e_c)."""
    exps = np.asarray(exps, dtype=np.int64)
    k = exps.size
    h = hadamard_columns(j, range(first_col, first_col + k))
    return np.ascontiguousarray(h * np.ldexp(1.0, exps)[None, :])


def hadamard_near_parallel(j: int, k: int, delta_exp: int = 40,
                           first_col: int = 1) -> np.ndarray:
    """Columns x_0 = h_0, x_i = h_0 + 2**-delta_exp h_i (i >= 1).

    Exact thin QR: Q = [h_0 .. h_{k-1}], R = [[1, 1, ..., 1],
    [0, d, 0, ...], [0, 0, d, ...] ...] with d = 2**-delta_exp.  The Gram
    matrix has entries 1 and 1 + d**2 that binary64 cannot hold.
    """
    h = hadamard_columns(j, range(first_col, first_col + k))
    x = h.copy()
    d = np.ldexp(1.0, -delta_exp)
    for i in range(1, k):
        x[:, i] = h[:, 0] + d * h[:, i]
    return np.ascontiguousarray(x)


def projected_pair(m: int, k: int, ky: int, kappa_x: float, kappa_xy: float,
                   seed: int):
    """Y (m x ky, orthonormal) and X with a prescribed kappa(X) and closeness to
    span(Y): X = Y A + P B with P orthonormal, P^T Y = 0, A Gaussian normalized
    to spectral norm 1, B = U_B diag(sigma) V_B^T with sigma log-spaced from
    1/kappa_xy * ... down so that sigma_min(B) = 1/kappa_xy and
    sigma_max(B)/sigma_min(B) = kappa_x.
    """
    rng = np.random.default_rng(seed)
    yp = haar(rng, m, ky + k)
    y = np.ascontiguousarray(yp[:, :ky])
    p = yp[:, ky:]
    a = rng.standard_normal((ky, k))
    a /= np.linalg.norm(a, 2)
    vb = haar(rng, k, k)
    smin = 1.0 / kappa_xy
    sig = smin * kappa_x * sigma_logspace(k, kappa_x)
    b = (vb * sig[None, :]) @ haar(rng, k, k).T
    x = y @ a + p @ b
    return np.ascontiguousarray(x), y


def batch_table(nblocks: int = 256, seed: int = 5000, m_lo: int = 10_000,
                m_hi: int = 1_000_000, widths=(8, 16, 32, 64),
                log_kappa=(3.0, 10.0)):
    """Block table of the batched workload: rows uniform in [m_lo, m_hi],
    width uniform over ``widths``, kappa log-uniform, seed per block."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=nblocks)
    ks = rng.choice(np.asarray(widths), size=nblocks)
    kap = np.power(10.0, rng.uniform(log_kappa[0], log_kappa[1], size=nblocks))
    return [dict(m=int(ms[b]), k=int(ks[b]), kappa=float(kap[b]),
                 seed=int(seed + 1 + b)) for b in range(nblocks)]


def _haar_device(torch, gen, m: int, k: int, device):
    g = torch.randn((m, k), generator=gen, dtype=torch.float64, device=device)
    q, r = torch.linalg.qr(g, mode="reduced")
    s = torch.sign(torch.diagonal(r))
    s[s == 0] = 1.0
    return (q * s[None, :]).contiguous()


def svd_matrix_device(m: int, k: int, kappa: float, seed: int, device="cuda", dtype=None):
    """X = U diag(sigma) V^T drawn on the device (torch Philox stream seeded
    with ``seed``; U first, then V).  Same recipe as ``svd_matrix``."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    u = _haar_device(torch, gen, m, k, device)
    v = _haar_device(torch, gen, k, k, device)
    sig = torch.from_numpy(sigma_logspace(k, kappa)).to(device)
    x = (u * sig[None, :]) @ v.t().contiguous()
    del u
    if dtype is not None:
        x = x.to(dtype)
    return x.contiguous()


def locked_basis_device(m: int, ky: int, seed: int, device="cuda"):
    """Haar m x ky locked basis drawn on the device (seeded Philox stream)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    return _haar_device(torch, gen, m, ky, device)


def projected_pair_device(m: int, k: int, ky: int, kappa_x: float, kappa_xy: float,
                          seed: int, device="cuda"):
    """``projected_pair`` drawn on the device (torch Philox stream seeded with
    ``seed``): Y (m x ky) and X = Y A + P B with P orthonormal and P^T Y = 0."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    yp = _haar_device(torch, gen, m, ky + k, device)
    y = yp[:, :ky].contiguous()
    p = yp[:, ky:]
    a = torch.randn((ky, k), generator=gen, dtype=torch.float64, device=device)
    a /= torch.linalg.matrix_norm(a, ord=2)
    vb = _haar_device(torch, gen, k, k, device)
    wb = _haar_device(torch, gen, k, k, device)
    sig = (1.0 / kappa_xy) * kappa_x * torch.from_numpy(sigma_logspace(k, kappa_x)).to(device)
    b = (vb * sig[None, :]) @ wb.t().contiguous()
    x = y @ a + p @ b
    return x.contiguous(), y


def b_weighted_pair(m: int, k: int, ky: int, kappa_x: float, kappa_xy: float, kappa_b: float,
                    seed: int):
    """Inputs for a B-inner product, B = diag(w) with w log-uniform in
    [kappa_b^-1/2, kappa_b^1/2]: (X, Y, w) = (W^-1/2 X0, W^-1/2 Y0, w) with
    (X0, Y0) from ``projected_pair``, so Y^T B Y = I and X has the
    B-condition and B-closeness to span(Y) of X0."""
    if ky:
        X0, Y0 = projected_pair(m, k, ky, kappa_x, kappa_xy, seed)
    else:
        X0, Y0 = svd_matrix(m, k, kappa_x, seed), np.zeros((m, 0))
    rng = np.random.default_rng(seed + 99)
    lw = rng.uniform(-0.5, 0.5, size=m) * np.log(kappa_b)
    w = np.exp(lw)
    s = 1.0 / np.sqrt(w)
    return (np.ascontiguousarray(X0 * s[:, None]), np.ascontiguousarray(Y0 * s[:, None]),
            np.ascontiguousarray(w))
