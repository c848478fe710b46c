"""GPU tests of the double-double result (borth_orthonormalize_dd: one DD
pass, Q returned as Q + Q_lo), on the shape of the paper's accuracy
experiment (Sec. 4.2, Fig. 7: n = 1000, k_y = 20, n_b = 4) and on blocks of
up to 64 columns.  The levels of the DD result are measured by the oracle's
binary128 Gram matrix of [Y | Q | Q_lo]; its binary64 words are compared
with the oracle's DD pass."""
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
    X = dev(synth.svd_matrix(2000, 65, 10.0, 7960))
    with pytest.raises(Exception):  # k > 64
        borth.orthonormalize_dd(X)
    X40 = synth.svd_matrix(2000, 40, 10.0, 7962)
    with pytest.raises(Exception):  # a DD input needs k <= 32
        borth.orthonormalize_dd(dev(X40), X_lo=dev(np.zeros_like(X40)))
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


@pytest.mark.parametrize("k,fact,dot2", [(12, "chol", False), (16, "chol", True), (32, "chol", False),
                                         (64, "chol", False), (24, "svqb", False),
                                         (64, "svqb", True)])
def test_dd_result_wide(k, fact, dot2):
    """Blocks of 9 to 64 columns (the DD update kernel for wide blocks): the
    DD result is orthonormal and orthogonal to Y at the DD pass's level
    (binary128 Gram of [Y | Q | Q_lo]), its low words are normalized, and
    for Cholesky its binary64 words agree with the oracle's DD pass."""
    borth = lib()
    n, ky, kx, kxy = 3000, 20, 10.0, 1e3
    X, Y = synth.projected_pair(n, k, ky, kx, kxy, 8100 + k)
    Q, Ql, R, C, info = borth.orthonormalize_dd(dev(X), dev(Y), fact=fact, dot2=dot2)
    assert info.status == 0
    Qh, Qlh = host(Q), host(Ql)
    om, omy = dd_levels(Qh, Qlh, Y)
    note("dd result wide", k, fact, dot2, om, omy)
    assert om <= 1e-28 * kxy ** 2 and omy <= 1e-28 * kxy ** 2
    assert np.all(np.abs(Qlh) <= np.spacing(np.abs(Qh)) / 2)
    if fact == "chol":
        o = oracle.cholqr_steps(X, Y, dd_first=True, dd_corrected=True, passes=1)
        assert o["info"] == 0
        dq = np.max(np.abs(Qh - o["Q"])) / np.max(np.abs(o["Q"]))
        note("  vs oracle DD pass", dq)
        assert dq <= 8 * U64


def test_dd_input_wide():
    """A DD input X + X_lo on a 16-column block with 20 locked columns."""
    borth = lib()
    X, Y = synth.projected_pair(N, 16, KY, 10.0, 10.0, 8170)
    rng = np.random.default_rng(8171)
    Xl = (rng.random(X.shape) - 0.5) * np.spacing(np.abs(X))
    Q, Ql, R, C, info = borth.orthonormalize_dd(dev(X), dev(Y), X_lo=dev(Xl), dot2=True)
    assert info.status == 0
    om, omy = dd_levels(host(Q), host(Ql), Y)
    note("dd input wide", om, omy)
    assert om <= 1e-27 and omy <= 1e-27
