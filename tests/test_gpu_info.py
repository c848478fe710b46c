"""GPU tests of what a call reports besides its result: the estimates in
borth_info (orth_est, kappa_est), the automatic escalation after a
breakdown, and the BORTH_LOG trace.  Exact values on the Hadamard family
(every factor is exact there), properties elsewhere."""
import os
import subprocess
import sys
from pathlib import Path

import numpy as np
import pytest

import oracle
import synth
from gpu_common import U64, dev, host, lib, note

pytestmark = pytest.mark.gpu

ROOT = Path(__file__).resolve().parents[1]


@pytest.mark.parametrize("gram,fact", [("f64", "chol"), ("dd", "chol"), ("f64", "svqb"),
                                       ("dd", "svqb")])
def test_estimates_exact_on_hadamard(gram, fact):
    """X = H diag(2^e): R_1 = diag(2^e) exactly, so kappa_est = 2^(max e - min
    e) and, after one pass, orth_est = ||diag(2^e) - I||_F; a second pass
    sees Q_1 = H exactly: orth_est = 0."""
    borth = lib()
    exps = [0, -3, 7, -9, 11, -5, 2, -12] if fact == "svqb" else [0, -3, 7, -20, 11, -35, 2, -50]
    X = synth.hadamard_scaled(7, exps)
    d = np.ldexp(1.0, exps)
    _, _, _, i1 = borth.orthonormalize(dev(X), gram=gram, fact=fact, passes=1)
    note("hadamard estimates", gram, fact, i1)
    assert i1.kappa_est == 2.0 ** (max(exps) - min(exps))
    assert abs(i1.orth_est - np.linalg.norm(d - 1.0)) <= 4 * U64 * np.linalg.norm(d)
    _, _, _, i2 = borth.orthonormalize(dev(X), gram=gram, fact=fact, passes=2)
    assert i2.orth_est == 0.0 and i2.kappa_est == i1.kappa_est and i2.escalation == 0


@pytest.mark.parametrize("fact", ["chol", "svqb"])
def test_estimates_against_the_oracle(fact):
    """kappa(X) = 1e6: the Cholesky diagonal ratio is a lower bound on kappa
    (R_ii lies between sigma_min and sigma_max), the SVQB estimate is
    sqrt(lambda_max / lambda_min) of the Gram (accurate to u kappa^2 here);
    orth_est of CholQR2 is ||R_2 - I||_F of the exact Cholesky of Q_1^T Q_1."""
    borth = lib()
    k, kappa = 8, 1e6
    X = synth.svd_matrix(20000, k, kappa, 6100)
    _, _, _, inf = borth.orthonormalize(dev(X), gram="f64", fact=fact, passes=2)
    note("estimates", fact, inf)
    if fact == "chol":
        assert kappa / 1e3 <= inf.kappa_est <= kappa * (1 + 1e-6)
    else:
        assert abs(inf.kappa_est / kappa - 1) <= 1e-3
    # the second pass's input, recomputed by one pass of the same kind
    Q1, _, _, _ = borth.orthonormalize(dev(X), gram="f64", fact=fact, passes=1)
    hi, lo = oracle.gram_q(host(Q1))
    G = hi + lo
    if fact == "chol":
        dev2 = np.linalg.norm(np.linalg.cholesky(G).T - np.eye(k))
    else:
        w, V = np.linalg.eigh(G)
        dev2 = np.linalg.norm(V @ np.diag(np.sqrt(w)) @ V.T - np.eye(k))
    note("  orth_est", inf.orth_est, "reference", dev2)
    assert 1e-12 <= dev2 and abs(inf.orth_est - dev2) <= 0.05 * dev2


def test_escalation_to_dd():
    """Exact Gram [[1, 1], [1, 1 + 2^-80]] (Hadamard columns, one tilted by
    2^-40): the binary64 Gram holds [[1, 1], [1, 1]] and its Cholesky breaks
    down at pivot 2; the DD retry returns the exact Q within a few ulps."""
    borth = lib()
    X = synth.hadamard_near_parallel(7, 4, 40)
    H = synth.hadamard_columns(7, range(1, 5))
    _, _, _, inf0 = borth.orthonormalize(dev(X), gram="f64", passes=2, check=False)
    note("no escalation", inf0)
    assert inf0.status == 4 and inf0.escalation == 0
    Q, R, _, inf = borth.orthonormalize(dev(X), gram="f64", passes=2, escalate=True, check=False)
    note("escalation", inf)
    assert inf.status == 0 and inf.escalation == 1
    assert np.max(np.abs(host(Q) - H)) <= 8 * U64 * np.abs(H).max()


def test_escalation_shifted_on_dependent_columns():
    """Two exactly equal columns (scaled Sylvester-Hadamard columns: the Gram
    matrix and the pivots are exact, so the DD Cholesky meets an exactly zero
    fourth pivot and breaks down).  The escalation then runs the shifted
    attempt: its first pass factors M + s I and succeeds; X has rank k - 1,
    so a binary64 pass after it may still meet a non-positive pivot.  The
    call must either return an orthonormal Q with X = Q R (the dependency a
    tiny R_ii) or report the breakdown of a later pass; both are
    deterministic for this input."""
    borth = lib()
    X = synth.hadamard_columns(6, [1, 2, 3, 2, 5, 6]) * np.ldexp(1.0, [0, -3, 2, 1, -1, 4])[None, :]
    _, _, _, inf0 = borth.orthonormalize(dev(X), gram="dd", passes=2, check=False)
    assert inf0.status == 4 and inf0.failed_pass == 1 and inf0.failed_pivot == 4
    Q, R, _, inf = borth.orthonormalize(dev(X), gram="dd", passes=2, escalate=True, check=False)
    note("shifted", inf)
    assert inf.escalation == 2
    if inf.status == 0:
        assert inf.passes_run == 3
        met = oracle.metrics(host(Q), X, host(R))
        note("  metrics", met)
        assert met["omega"] <= 1e-13 and met["rho"] <= 1e-13
        d = np.abs(np.diag(host(R)))
        assert d.min() <= 1e-8 * d.max()
    else:
        assert inf.status == 4 and inf.failed_pass >= 2


def test_escalation_rejects_in_place_and_fp32():
    borth = lib()
    X = dev(synth.svd_matrix(3000, 4, 10.0, 6400))
    with pytest.raises(Exception):
        borth.orthonormalize(X, out=X, sched="materialize", escalate=True)
    with pytest.raises(Exception):
        borth.orthonormalize(X.float(), gram="split", escalate=True)


def test_log_line():
    """BORTH_LOG=1 prints one line per call with the status and estimates."""
    code = ("import sys; sys.path.insert(0, %r); import torch, synth; "
            "import paper_1806_01036_amd as b; "
            "X = torch.from_numpy(synth.hadamard_scaled(5, [0, 3, -2])).cuda(); "
            "b.orthonormalize(X, gram='dd', passes=2)" % str(ROOT))
    env = dict(os.environ, BORTH_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stderr.splitlines() if l.startswith("borth: orthonormalize")]
    note("log", lines)
    assert len(lines) == 1 and "status=0" in lines[0] and "kappa_est=3.200e+01" in lines[0]


def test_profiling_mask():
    """Event timing per kernel kind: only the kinds in the mask are timed."""
    borth = lib()
    ctx = borth.default_context()
    X = dev(synth.svd_matrix(100_000, 16, 1e3, 6500))
    ctx.set_profiling(True, kinds=(0,))
    for _ in range(3):
        borth.orthonormalize(X, gram="dd", passes=2, ctx=ctx)
    g_ms, g_n = ctx.kernel_time(0)
    u_ms, u_n = ctx.kernel_time(1)
    ctx.set_profiling(False)
    assert g_n == 3 and g_ms > 0.0 and u_n == 0
    ctx.set_profiling(True)
    borth.orthonormalize(X, gram="dd", passes=2, ctx=ctx)
    g_ms, g_n = ctx.kernel_time(0)
    u_ms, u_n = ctx.kernel_time(1)
    ctx.set_profiling(False)
    assert g_n == 1 and u_n == 2 and u_ms > 0.0


def test_update_clears_the_estimates():
    """borth_update stages its C where a path call leaves its estimates; the
    info read after it reports no estimates instead of entries of C."""
    borth = lib()
    ctx = borth.default_context(0)
    X = synth.svd_matrix(4000, 8, 1e3, 11)
    _, _, _, i1 = borth.orthonormalize(dev(X), gram="f64", passes=1, ctx=ctx)
    assert i1.kappa_est > 1.0 and ctx.info().kappa_est == i1.kappa_est
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((4000, 4))
    C = np.full((4, 8), 123.0)
    borth.update(dev(X), dev(np.triu(rng.standard_normal((8, 8)))), dev(Y), dev(C), ctx=ctx)
    inf = ctx.info()
    assert inf.orth_est == 0.0 and inf.kappa_est == 0.0
