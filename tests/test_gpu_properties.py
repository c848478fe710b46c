"""Property tests on the GPU (hypothesis, derandomized so every run draws the
same cases): orthonormalization and Gram sweeps over random shapes, leading
dimensions, conditioning, locked-basis widths, precisions and in-place calls,
each checked against the oracle's binary128 measures and bounds."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
import synth
from gpu_common import U64, dev, host, lib, note, rel_fro, torch_gpu

SETTINGS = dict(deadline=None, derandomize=True, database=None,
                suppress_health_check=list(HealthCheck))


def gamma(n):
    return n * U64 / (1 - n * U64)


def chain(m):
    # summation chain of the sweeps: per-lane rows plus the fixed-order reductions
    return m // 4 + 1100


@pytest.mark.gpu
@settings(max_examples=40, **SETTINGS)
@given(k=st.integers(1, 64), ky=st.sampled_from([0, 1, 5, 16]),
       extra=st.one_of(st.integers(8, 300), st.integers(300, 30_000)),
       padx=st.integers(0, 3), padq=st.integers(0, 2), log_kappa=st.sampled_from([0, 3, 6, 10]),
       gram=st.sampled_from(["f64", "dd"]), inplace=st.booleans(),
       seed=st.integers(0, 2 ** 31 - 1))
def test_orthonormalize_properties(k, ky, extra, padx, padq, log_kappa, gram, inplace, seed):
    borth = lib()
    torch = torch_gpu()
    if gram == "f64":
        log_kappa = min(log_kappa, 6)  # binary64 CholQR2 needs u kappa^2 < 1
    m = k + ky + extra
    note("props: orthonormalize", dict(m=m, k=k, ky=ky, padx=padx, padq=padq,
                                       log_kappa=log_kappa, gram=gram, inplace=inplace, seed=seed))
    X = synth.svd_matrix(m, k, 10.0 ** log_kappa, seed)
    Y = synth.locked_basis(m, ky, seed + 1) if ky else None
    xbuf = torch.zeros((m, k + padx), dtype=torch.float64, device="cuda")
    xbuf[:, :k] = dev(X)
    Xd = xbuf[:, :k]
    if inplace:
        out, qbuf = Xd, xbuf
    else:
        qbuf = torch.zeros((m, k + padq), dtype=torch.float64, device="cuda")
        out = qbuf[:, :k]
    Q, R, C, info = borth.orthonormalize(Xd, None if Y is None else dev(Y), gram=gram, out=out)
    assert info.status == 0, info
    met = oracle.metrics(host(Q), X, host(R), Y, None if C is None else host(C))
    assert met["omega"] <= 1e-14 and met["rho"] <= 1e-14, met
    if ky:
        assert met["omega_y"] <= 1e-14, met
    # columns beyond k of the padded buffers are never written
    assert torch.count_nonzero(qbuf[:, k:]).item() == 0
    if not inplace:
        assert torch.count_nonzero(xbuf[:, k:]).item() == 0
        assert np.array_equal(host(Xd), X)  # the input is left as it was


@pytest.mark.gpu
@settings(max_examples=30, **SETTINGS)
@given(m=st.one_of(st.integers(1, 200), st.integers(200, 60_000)), k=st.integers(1, 64),
       ky=st.integers(0, 64), pad=st.integers(0, 3), prec=st.sampled_from(["f64", "dd", "dd_dot2"]),
       seed=st.integers(0, 2 ** 31 - 1))
def test_gram_properties(m, k, ky, pad, prec, seed):
    borth = lib()
    torch = torch_gpu()
    note("props: gram", dict(m=m, k=k, ky=ky, pad=pad, prec=prec, seed=seed))
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((m, k)) * np.ldexp(1.0, rng.integers(-4, 4, (1, k)))
    Y = rng.standard_normal((m, ky)) if ky else None
    xbuf = torch.zeros((m, k + pad), dtype=torch.float64, device="cuda")
    xbuf[:, :k] = dev(X)
    ghi, glo = borth.gram(xbuf[:, :k], None if Y is None else dev(Y), prec=prec)
    ghi = host(ghi)
    glo = host(glo) if glo is not None else np.zeros_like(ghi)
    V = X if Y is None else np.hstack([Y, X])
    ex_hi, ex_lo = oracle.gram_q(V)
    absg = np.abs(V).T @ np.abs(V)
    err = np.abs((ghi - ex_hi) + (glo - ex_lo))
    if prec == "f64":
        assert np.all(err <= gamma(chain(m)) * absg + 1e-300)
        assert rel_fro(ghi, ex_hi + ex_lo) <= 1e-14
    else:
        assert np.all(err <= gamma(chain(m)) ** 2 * absg + 4 * U64 ** 2 * np.abs(ex_hi))
    assert np.array_equal(ghi, ghi.T) and np.array_equal(glo, glo.T)
