"""GPU tests of the iterated scheme in a B-inner product (Sec. 4.2: the
technique carries over to B-inner products), B = diag(w) with kappa(B) up to
1e4: Q^T B Q = I, Y^T B Q = 0 and X = Y C + Q R, measured by the oracle's
binary128 B-weighted Gram matrices."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import U64, dev, host, lib, note, torch_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,k,ky,gram,fact,strided", [
    (30011, 4, 20, "dd", "chol", False),   # narrow, fused weighted Gram columns (DD)
    (30011, 2, 10, "f64", "svqb", False),  # narrow, fused (binary64)
    (30011, 8, 0, "dd", "svqb", False),    # no Y
    (30011, 16, 12, "dd", "chol", False),  # wide: weighted [Y | S]^T B S sweeps, MFMA update
    (20000, 3, 7, "f64", "chol", False),   # odd ky: separate weighted sweeps, narrow update
    (20000, 2, 12, "dd", "chol", True),    # strided Y
])
def test_b_inner_iterated(m, k, ky, gram, fact, strided):
    borth = lib()
    torch = torch_gpu()
    kx, kxy = (1e4, 1e8) if gram == "dd" else (1e3, 1e3)
    if fact == "chol" and gram == "f64":
        kx, kxy = 1e2, 1e2
    X, Y, w = synth.b_weighted_pair(m, k, ky, kx, kxy, 1e4, 2100 + k + ky)
    Yd = None
    if ky:
        Yd = dev(np.hstack([Y, np.zeros((m, 3))]))[:, :ky] if strided else dev(Y)
    Q, R, C, it, info = borth.orthonormalize_iter(dev(X), Yd, gram=gram, fact=fact, eps=1e-10,
                                                  max_iter=8, B=dev(w))
    note("B-inner", m, k, ky, gram, fact, strided, it)
    assert info.status == 0 and it.converged
    Qh = host(Q)
    met = oracle.metrics_b(Qh, X, host(R), w, Y if ky else None, host(C) if ky else None)
    note("  metrics", met)
    svqb64 = fact == "svqb" and gram == "f64"
    assert met["omega"] <= (20 * k * U64 if svqb64 else 1e-14)
    # binary64 SVQB's residual carries k kappa u times the norm of the part
    # it factors (kappa(X) / kappa(X, Y) of X's scale when Y is present)
    svqb_rho = 10 * k * kx * U64 * (kx / kxy if ky else 1.0)
    assert met["rho"] <= (max(1e-14, svqb_rho) if svqb64 else 1e-14)
    if ky:
        assert met["omega_y"] <= 1e-14
        # exact B-projection coefficients (Y^T B Y)^{-1} Y^T B X
        shi, slo = oracle.gram_w_q(Y, w)
        chi, clo = oracle.gram_w_q(Y, w, X)
        cex = np.linalg.solve(shi + slo, chi + clo)
        assert np.max(np.abs(host(C) - cex)) <= 1e-13 * max(1.0, np.max(np.abs(cex)))
    # the Euclidean orthogonality is not what was asked for: with kappa(B) =
    # 1e4 it is far from the identity
    assert np.linalg.norm(Qh.T @ Qh - np.eye(k)) > 1e-3


def test_b_inner_identity_weights_match_plain():
    """B = I through the weighted kernels reaches the plain scheme's levels
    and its passes."""
    borth = lib()
    X, Y = synth.projected_pair(40_000, 4, 16, 1e6, 1e10, 2200)
    w = np.ones(X.shape[0])
    r1 = borth.orthonormalize_iter(dev(X), dev(Y), gram="dd", fact="chol", eps=1e-10,
                                   max_iter=8, B=dev(w))
    r0 = borth.orthonormalize_iter(dev(X), dev(Y), gram="dd", fact="chol", eps=1e-10,
                                   max_iter=8)
    assert r1[3].converged and r0[3].converged and r1[3].passes_run == r0[3].passes_run
    for r in (r0, r1):
        met = oracle.metrics(host(r[0]), X, host(r[1]), Y, host(r[2]))
        assert met["omega"] <= 1e-14 and met["omega_y"] <= 1e-14 and met["rho"] <= 1e-14
    # the same method; the weighted sweeps stage their row panels in
    # registers and the unweighted first sweep by direct transfers to LDS,
    # with panels of other heights, so the DD Gram matrices differ in their
    # last bits (~1e-31 relative) and the results agree to rounding level
    assert np.max(np.abs(host(r0[0]) - host(r1[0]))) <= 1e-14


def test_b_inner_errors():
    borth = lib()
    torch = torch_gpu()
    X, Y, w = synth.b_weighted_pair(5000, 2, 4, 10.0, 10.0, 10.0, 2300)
    with pytest.raises(ValueError):
        borth.orthonormalize_iter(dev(X), dev(Y), B=dev(w[:-1]))
    with pytest.raises(ValueError):
        borth.orthonormalize_iter(dev(X), dev(Y), B=dev(w.astype(np.float32)))
