"""GPU tests of the double-double result (borth_orthonormalize_dd: one DD
pass, Q returned as Q + Q_lo), on the shape of the paper's accuracy
experiment (Sec. 4.2, Fig. 7: n = 1000, k_y = 20, n_b = 4).  The levels of
the DD result are measured by the oracle's binary128 Gram matrix of
[Y | Q | Q_lo]."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import U64, dev, host, lib, note

pytestmark = pytest.mark.gpu

N, KY, K = 1000, 20, 4


def dd_levels(Qh, Ql, Y=None):
    """omega = ||(Qh + Ql)^T (Qh + Ql) - I||_F and omega_Y = ||Y^T (Qh + Ql)||_F
    from the binary128 Gram of [Y | Qh | Ql] (its hi + lo words carry ~106
    bits, so levels down to ~1e-31 are resolved)."""
    k = Qh.shape[1]
    ky = 0 if Y is None else Y.shape[1]
    V = np.hstack(([Y] if ky else []) + [Qh, Ql])
    hi, lo = oracle.gram_q(V)
    H, L = slice(ky, ky + k), slice(ky + k, ky + 2 * k)
    D = ((hi[H, H] - np.eye(k)) + lo[H, H]) + ((hi[H, L] + hi[L, H]) + (lo[H, L] + lo[L, H])) + hi[L, L]
    om = float(np.linalg.norm(D))
    omy = 0.0
    if ky:
        E = (hi[:ky, H] + hi[:ky, L]) + (lo[:ky, H] + lo[:ky, L])
        omy = float(np.linalg.norm(E))
    return om, omy


@pytest.mark.parametrize("kx,kxy,dot2", [(1.0, 1.0, False), (1.0, 1e3, False), (1e3, 1e3, False),
                                         (1.0, 1e6, True), (1e3, 1e6, True)])
def test_dd_result_levels(kx, kxy, dot2):
    """The DD result is orthonormal far below binary64 rounding: omega and
    omega_Y of Q + Q_lo at the DD pass's own error level (about u_DD kappa^2
    with kappa = max(kappa(X), kappa(X, Y)) and the Gram's error), while Q
    alone sits at the rounding level ~1e-17."""
    borth = lib()
    X, Y = synth.projected_pair(N, K, KY, kx, kxy, 7900 + int(np.log10(kx * kxy)))
    Q, Ql, R, C, info = borth.orthonormalize_dd(dev(X), dev(Y), dot2=dot2)
    assert info.status == 0
    Qh, Qlh = host(Q), host(Ql)
    om, omy = dd_levels(Qh, Qlh, Y)
    met = oracle.metrics(Qh, X, host(R), Y, host(C))
    note("dd result", kx, kxy, dot2, om, omy, "binary64 Q:", met["omega"], met["omega_y"])
    kap = max(kx, kxy)
    assert om <= 1e-29 * kap ** 2 and omy <= 1e-29 * kap ** 2
    if kap <= 1e3:
        assert om <= 1e-3 * met["omega"]
    # the low words are those of a normalized DD pair
    assert np.all(np.abs(Qlh) <= np.spacing(np.abs(Qh)) / 2)


def test_dd_result_hi_word_is_the_dd_pass():
    """Q alone is bit for bit what the one-pass DD orthonormalization returns."""
    borth = lib()
    X, Y = synth.projected_pair(N, K, KY, 10.0, 1e4, 7950)
    Q, Ql, R, C, _ = borth.orthonormalize_dd(dev(X), dev(Y))
    Q1, R1, C1, _ = borth.orthonormalize(dev(X), dev(Y), gram="dd", passes=1)
    assert np.array_equal(host(Q), host(Q1)) and np.array_equal(host(R), host(R1))
    assert np.array_equal(host(C), host(C1))


def test_dd_result_exact_hadamard():
    """X = H diag(2^e): the exact Q = H is representable, so Q_lo = 0."""
    borth = lib()
    X = synth.hadamard_scaled(6, [0, -3, 7, -20])
    H = synth.hadamard_columns(6, range(1, 5))
    Q, Ql, R, _, info = borth.orthonormalize_dd(dev(X))
    assert info.status == 0
    assert np.array_equal(host(Q), H) and not np.any(host(Ql))


def test_dd_result_argument_checks():
    borth = lib()
    X = dev(synth.svd_matrix(2000, 16, 10.0, 7960))
    with pytest.raises(Exception):  # k > 8
        borth.orthonormalize_dd(X)
    X4 = dev(synth.svd_matrix(2000, 4, 10.0, 7961))
    with pytest.raises(Exception):  # Q_lo aliasing X
        borth.orthonormalize_dd(X4, out_lo=X4)


@pytest.mark.parametrize("ky", [20, 0])
def test_dd_input(ky):
    """A DD input X + X_lo (|X_lo| up to ulp(X)/2): the result is orthonormal
    at the DD level only if both the Gram (its [X | X_lo] and [Y | X_lo]
    blocks) and the update see X_lo -- leaving it out of either would leave
    an error of about |X_lo| / |X| ~ 1e-16 in omega or omega_Y."""
    borth = lib()
    X, Y = synth.projected_pair(N, K, KY, 10.0, 10.0, 7970)
    rng = np.random.default_rng(7971)
    Xl = (rng.random(X.shape) - 0.5) * np.spacing(np.abs(X))
    Yd = dev(Y) if ky else None
    Q, Ql, R, C, info = borth.orthonormalize_dd(dev(X), Yd, X_lo=dev(Xl), dot2=True)
    assert info.status == 0
    om, omy = dd_levels(host(Q), host(Ql), Y if ky else None)
    note("dd input", ky, om, omy)
    assert om <= 1e-27 and omy <= 1e-27
    # the same X without its low words gives a different DD result
    Q0, Ql0, _, _, _ = borth.orthonormalize_dd(dev(X), Yd, dot2=True)
    d = np.max(np.abs((host(Q) - host(Q0)) + (host(Ql) - host(Ql0))))
    assert 1e-20 < d < 1e-14
