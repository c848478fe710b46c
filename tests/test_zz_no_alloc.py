"""The allocation-free entry point (borth_orthonormalize_noalloc) against
borth_orthonormalize, through the C ABI: the same kernels with the same
launch shapes, so the results must agree bit for bit.  Two calls in a row
share the device scratch array, the second on a smaller input (whatever the
first left there must not leak into it); the outputs are also judged by the
oracle's measures.  The per-device scratch address is taken at context
creation (hipGetSymbolAddress); the call allocates nothing."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import dev, host, lib, note, torch_gpu

pytestmark = pytest.mark.gpu


def _pair(borth, X, Y, **kw):
    torch = torch_gpu()
    Xd = dev(X)
    Yd = dev(Y) if Y is not None else None
    Q0, R0, C0, i0 = borth.orthonormalize(Xd, Yd, **kw)
    Q1, R1, C1, i1 = borth.orthonormalize_noalloc(Xd, Yd, **kw)
    torch.cuda.synchronize()
    assert i0.status == 0 and i1.status == 0, (i0, i1)
    assert i1.passes_run == i0.passes_run
    assert torch.equal(Q0, Q1) and torch.equal(R0, R1)
    if Y is not None:
        assert torch.equal(C0, C1)
    met = oracle.metrics(host(Q1), X, host(R1), Y, None if Y is None else host(C1))
    note("  noalloc metrics", {k: float(v) for k, v in met.items()})
    return met


def test_noalloc_matches_regular_two_calls():
    borth = lib()
    # first call: a taller, wider block (DD CholQR2, recompute schedule)
    note("noalloc call 1: 300000 x 32, kappa 1e12, DD CholQR2")
    X = synth.svd_matrix(300_000, 32, 1e12, 901)
    met = _pair(borth, X, None, gram="dd", passes=2)
    assert met["omega"] <= 1e-14 and met["rho"] <= 1e-14
    # second call, smaller, with a locked basis (P,C,P,C)
    note("noalloc call 2: 50000 x 16 with Y 50000 x 8, kappa 1e9, DD CholQR2")
    X = synth.svd_matrix(50_000, 16, 1e9, 902)
    Y = synth.locked_basis(50_000, 8, 903)
    met = _pair(borth, X, Y, gram="dd", passes=2)
    assert met["omega"] <= 1e-14 and met["rho"] <= 1e-14 and met["omega_y"] <= 1e-14


def test_noalloc_other_modes_and_async():
    borth = lib()
    torch = torch_gpu()
    note("noalloc: binary64 CholQR2 materialized 100000 x 64, then plain CholQR 20000 x 8")
    X = synth.svd_matrix(100_000, 64, 1e6, 904)
    _pair(borth, X, None, gram="f64", passes=2, sched="materialize")
    X = synth.svd_matrix(20_000, 8, 1e4, 905)
    _pair(borth, X, None, gram="f64", passes=1)
    note("noalloc: split-BF16 + 2 binary64 passes, 100000 x 64 fp32")
    X32 = synth.svd_matrix(100_000, 64, 1e6, 906).astype(np.float32)
    Xd = dev(X32)
    Q0, R0, _, _ = borth.orthonormalize(Xd, gram="split", passes=3)
    Q1, R1, _, _ = borth.orthonormalize_noalloc(Xd, gram="split", passes=3)
    assert torch.equal(Q0, Q1) and torch.equal(R0, R1)
    # asynchronous call (no info): the same result once the stream is done
    note("noalloc: asynchronous call")
    X = synth.svd_matrix(40_000, 32, 1e10, 907)
    Xd = dev(X)
    Q0, R0, _, _ = borth.orthonormalize(Xd, gram="dd")
    Q1 = torch.full_like(Q0, float("nan"))
    R1 = torch.full_like(R0, float("nan"))
    borth.orthonormalize_noalloc(Xd, gram="dd", out=Q1, R=R1, sync=False)
    torch.cuda.synchronize()
    assert torch.equal(Q0, Q1) and torch.equal(R0, R1)
    # what the call refuses before anything is enqueued
    with pytest.raises(borth.BorthError):
        borth.orthonormalize_noalloc(dev(np.zeros((3, 5))))  # m < k
