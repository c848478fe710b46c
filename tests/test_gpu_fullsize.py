"""Parity at the workloads' full sizes, judged by the CPU oracle.

The smaller parity tests cover every kernel element by element; these run
the configurations the measurements are quoted on, at their real shapes and
launch configurations, and judge the outputs with the oracle's binary128-
accurate measures (orthogonality loss omega = ||Q^T Q - I||_F, residual
rho = ||X - Y C - Q R||_F / ||X||_F, omega_Y = ||Y^T Q||_F) and, where the
oracle can afford it, its exact Gram matrix:

* 4,000,000 x 32 binary64, kappa in {1e8, 1e12, 1e15}: DD-Gram CholQR2
  reaches omega, rho <= 1e-14; the binary64 CholQR2 comparator on the same
  input breaks down or stays far from orthogonal at kappa >= 1e12; at
  kappa = 1e12 the DD Gram sweep (many panels per workgroup) against the
  exact Gram matrix;
* 10,000,000 x {32, 64} binary64, kappa = 1e6: binary64 CholQR2;
* 16,777,216 x 64 fp32, kappa = 1e6: the split-BF16 Gram (stage 1) against
  the exact Gram of the widened X, then omega after one and two binary64
  passes (stages 2 and 3) and rho;
* the eight tallest blocks of the 256-block batch, at full height with their
  16-column locked bases, in one batched call.

Inputs are drawn on the device with the seeded generator of the same recipe
(synth.*_device) and copied to the host for the oracle.  The oracle's
measures run on the host's cores (a few seconds to a minute per case).
"""
import re

import numpy as np
import pytest

import oracle
import synth
from gpu_common import U64, host, lib, note, torch_gpu

pytestmark = pytest.mark.gpu

_cache = {}


def _svd_x(m, k, kappa, seed, dtype=None):
    key = (m, k, kappa, seed, dtype)
    if key not in _cache:
        _cache.clear()  # one large input at a time
        torch = torch_gpu()
        note(f"generate X {m} x {k} kappa={kappa:g} seed={seed}")
        Xd = synth.svd_matrix_device(m, k, kappa, seed, dtype=dtype)
        torch.cuda.synchronize()
        _cache[key] = (Xd, host(Xd))
    return _cache[key]


def _metrics(Q, X, R, Y=None, C=None):
    met = oracle.metrics(host(Q), X, host(R), Y, C)
    note("  oracle metrics", {k: float(v) for k, v in met.items()})
    return met


@pytest.mark.parametrize("kappa,seed", [(1e8, 301), (1e12, 302), (1e15, 303)])
def test_c3_dd_cholqr2_full(kappa, seed):
    borth = lib()
    torch = torch_gpu()
    m, k = 4_000_000, 32
    Xd, X = _svd_x(m, k, kappa, seed)
    note(f"DD CholQR2 {m} x {k} kappa={kappa:g}")
    Q, R, _, info = borth.orthonormalize(Xd, gram="dd", passes=2)
    assert info.status == 0, info
    met = _metrics(Q, X, R)
    assert met["omega"] <= 1e-14 and met["rho"] <= 1e-14, met
    del Q
    note(f"binary64 CholQR2 {m} x {k} kappa={kappa:g}")
    Qf, Rf, _, inf = borth.orthonormalize(Xd, gram="f64", passes=2, check=False)
    torch.cuda.synchronize()
    if inf.status == 0:
        mf = _metrics(Qf, X, Rf)
        if kappa >= 1e12:
            assert mf["omega"] > 1e-14, mf
    else:
        note("  binary64 CholQR2 status", inf.status, "pass", inf.failed_pass,
             "pivot", inf.failed_pivot)
        assert kappa >= 1e8 and inf.status == 4
    del Qf


def test_c3_dd_gram_full_vs_exact():
    """The DD Gram sweep of the 4,000,000 x 32 headline input in its timed
    launch configuration (each workgroup folds many row panels) against the
    binary128 Gram matrix: max |dG_ij| <= 2e-30 sqrt(G_ii G_jj), normwise
    <= 1e-28."""
    borth = lib()
    Xd, X = _svd_x(4_000_000, 32, 1e12, 302)
    note("DD Gram 4,000,000 x 32")
    ghi, glo = borth.gram(Xd, prec="dd")
    ex_hi, ex_lo = oracle.gram_q(X)
    err = np.abs((host(ghi) - ex_hi) + (host(glo) - ex_lo))
    d = np.sqrt(np.diag(ex_hi))
    rel = err / np.outer(d, d)
    note("  max", rel.max(), "normwise", np.linalg.norm(err) / np.linalg.norm(ex_hi))
    assert rel.max() <= 2e-30
    assert np.linalg.norm(err) <= 1e-28 * np.linalg.norm(ex_hi)


def test_fig8_dot2_gram_full_sampled():
    """The first Gram sweep of the iterated DD scheme at the paper's runtime
    shape (n = 8e6 rows, [Y | X] with k_y = 40 and n_b = 4, kappa(X) = 1e6,
    kappa(X, Y) = 1e12): Dot2 sums on LDS-staged panels, each workgroup
    folding many panels, against entries of the binary128 Gram matrix taken
    one column pair at a time (Y^T Y, Y^T X and X^T X entries, on and off the
    diagonal): |dG_ij| <= 2e-30 sqrt(G_ii G_jj) (measured up to 1.9e-31)."""
    borth = lib()
    torch_gpu()
    Xd, Yd = synth.projected_pair_device(8_000_000, 4, 40, 1e6, 1e12, 8101)
    note("Dot2 Gram 8,000,000 x [40 | 4]")
    ghi, glo = borth.gram(Xd, Yd, prec="dd_dot2")
    ghi, glo = host(ghi), host(glo)
    Y, X = host(Yd), host(Xd)
    for i, j in [(0, 0), (3, 17), (39, 39), (5, 40), (39, 43), (40, 40), (41, 43), (43, 43)]:
        a = Y[:, i] if i < 40 else X[:, i - 40]
        b = Y[:, j] if j < 40 else X[:, j - 40]
        ex_hi, ex_lo = oracle.gram_q(np.ascontiguousarray(np.stack([a, b], axis=1)))
        d = np.sqrt(ex_hi[0, 0] * ex_hi[1, 1])
        e = abs((ghi[i, j] - ex_hi[0, 1]) + (glo[i, j] - ex_lo[0, 1])) / d
        note("  entry", i, j, e)
        assert e <= 2e-30


@pytest.mark.parametrize("gram,fact,max_passes,bq,by",
                         [("dd", "chol", 3, 1e-16, 1e-17), ("dd", "svqb", 3, 1e-16, 1e-17),
                          ("f64", "svqb", 4, 1e-14, 1e-15)])
def test_fig8_iterated_full_sampled(gram, fact, max_passes, bq, by):
    """The iterated scheme, fused, to convergence (eps 1e-10) at the paper's
    runtime shape (n = 8e6, k_y = 40, n_b = 4, kappa(X) = 1e6, kappa(X, Y) =
    1e12), judged by binary128 entries of [Y | Q]^T Q taken one column pair
    at a time: every entry of Q^T Q - I and sampled entries of Y^T Q (measured
    2.0e-18 / 4.2e-20 for DD Cholesky, 1.5e-19 / 3.2e-20 for DD SVQB,
    7.2e-16 / 9.0e-18 for binary64 SVQB), in at most 3 passes with DD sums and
    4 with binary64 ones (the passes the paper's DD variant saves)."""
    borth = lib()
    torch = torch_gpu()
    Xd, Yd = synth.projected_pair_device(8_000_000, 4, 40, 1e6, 1e12, 7404)
    Q = torch.empty_like(Xd)
    note("iterated", gram, fact, "8,000,000 x [40 | 4]")
    it = borth.orthonormalize_iter(Xd, Yd, gram=gram, fact=fact, eps=1e-10, max_iter=10, out=Q,
                                   fuse=True)[3]
    note("  passes", it.passes_run, "converged", it.converged)
    assert it.converged and it.passes_run <= max_passes
    Qh, Y = host(Q), host(Yd)
    for i in range(4):
        for j in range(i, 4):
            ex_hi, ex_lo = oracle.gram_q(np.ascontiguousarray(np.stack([Qh[:, i], Qh[:, j]], axis=1)))
            v = abs((ex_hi[0, 1] - (1.0 if i == j else 0.0)) + ex_lo[0, 1])
            note("  Q^T Q - I", i, j, v)
            assert v <= bq
    for i in (0, 7, 19, 33, 39):
        for j in range(4):
            ex_hi, ex_lo = oracle.gram_q(np.ascontiguousarray(np.stack([Y[:, i], Qh[:, j]], axis=1)))
            assert abs(ex_hi[0, 1] + ex_lo[0, 1]) <= by


@pytest.mark.parametrize("gram,max_passes,bq,by", [("dd", 3, 1e-16, 1e-17), ("f64", 4, 1e-14, 1e-15)])
def test_binner_iterated_full_sampled(gram, max_passes, bq, by):
    """B-inner products at the runtime experiment's size: B = diag(w), w
    log-uniform with kappa(B) = 1e4, n = 8e6, k_y = 20, n_b = 4, the inputs
    scaled so that Y^T B Y = I; the iterated scheme with SVQB to convergence,
    judged by binary128 entries of [Y | Q]^T B Q taken one column pair at a
    time: every entry of Q^T B Q - I and sampled entries of Y^T B Q (measured
    1.2e-19 / 3.8e-20 with DD sums, 8.9e-16 / 9.8e-18 with binary64 ones)."""
    borth = lib()
    torch = torch_gpu()
    n, ky, k = 8_000_000, 20, 4
    X0, Y0 = synth.projected_pair_device(n, k, ky, 1e6, 1e12, 7000 + 10 * ky + k)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(8000 + ky + k)
    w = torch.exp((torch.rand(n, generator=gen, dtype=torch.float64, device="cuda") - 0.5)
                  * np.log(1e4))
    s = torch.rsqrt(w)[:, None]
    X = (X0 * s).contiguous()
    Y = (Y0 * s).contiguous()
    del X0, Y0
    Q = torch.empty_like(X)
    note("B-inner iterated", gram, "8,000,000 x [20 | 4]")
    it = borth.orthonormalize_iter(X, Y, gram=gram, fact="svqb", eps=1e-10, max_iter=10, out=Q,
                                   B=w)[3]
    note("  passes", it.passes_run, "converged", it.converged)
    assert it.converged and it.passes_run <= max_passes
    Qh, Yh, wh = host(Q), host(Y), host(w)
    for i in range(k):
        for j in range(i, k):
            hi, lo = oracle.gram_w_q(np.ascontiguousarray(np.stack([Qh[:, i], Qh[:, j]], axis=1)), wh)
            assert abs((hi[0, 1] - (1.0 if i == j else 0.0)) + lo[0, 1]) <= bq
    for i in (0, 5, 11, 19):
        for j in range(k):
            hi, lo = oracle.gram_w_q(np.ascontiguousarray(np.stack([Yh[:, i], Qh[:, j]], axis=1)), wh)
            assert abs(hi[0, 1] + lo[0, 1]) <= by


@pytest.mark.parametrize("fact", ["chol", "svqb"])
def test_dd_result_full_sampled(fact):
    """One DD pass returning Q + Q_lo (the DD update for wide blocks) at
    4,000,000 x [16 | 32], kappa(X) = 10, kappa(X, Y) = 1e3, judged by
    binary128 Gram entries of [q_i, q_i_lo, q_j, q_j_lo] (and [y_i, q_j,
    q_j_lo]): entries of (Q + Q_lo)^T (Q + Q_lo) - I within 1e-25 and sampled
    entries of Y^T (Q + Q_lo) within 1e-27 (measured 5.6e-27 / 4.8e-30 with
    Cholesky, 3.0e-27 / 4.7e-30 with SVQB), far below any binary64 result."""
    borth = lib()
    torch_gpu()
    Xd, Yd = synth.projected_pair_device(4_000_000, 32, 16, 10.0, 1e3, 8200)
    note("DD result", fact, "4,000,000 x [16 | 32]")
    Q, Ql, R, C, info = borth.orthonormalize_dd(Xd, Yd, fact=fact)
    assert info.status == 0
    Qh, Qlh, Y = host(Q), host(Ql), host(Yd)

    def gram(*cols):
        return oracle.gram_q(np.ascontiguousarray(np.stack(cols, axis=1)))

    for i, j in [(0, 0), (0, 1), (5, 17), (31, 31), (30, 31), (12, 12)]:
        hi, lo = gram(Qh[:, i], Qlh[:, i], Qh[:, j], Qlh[:, j])
        v = (((hi[0, 2] - (1.0 if i == j else 0.0)) + lo[0, 2]) + (hi[0, 3] + hi[1, 2])
             + (lo[0, 3] + lo[1, 2]) + hi[1, 3])
        note("  (Q + Q_lo)^T (Q + Q_lo) - I", i, j, v)
        assert abs(v) <= 1e-25
    for i in (0, 9, 15):
        for j in (0, 13, 31):
            hi, lo = gram(Y[:, i], Qh[:, j], Qlh[:, j])
            assert abs((hi[0, 1] + hi[0, 2]) + (lo[0, 1] + lo[0, 2])) <= 1e-27


@pytest.mark.parametrize("gram", ["f64", "dd"])
def test_rank_revealing_full_sampled(gram):
    """SVQB with rank revelation at the runtime experiment's size (n = 8e6,
    k_y = 10, n_b = 4, kappa(X) = kappa(X, Y) = 1e3) with column 3 set to
    column 0 plus column 1: rank 3, the last column of Q zero, the first
    three orthonormal and orthogonal to Y by binary128 entries taken one
    column pair at a time, and X = Y C + Q R to the binary64 level."""
    borth = lib()
    torch = torch_gpu()
    Xd, Yd = synth.projected_pair_device(8_000_000, 4, 10, 1e3, 1e3, 3104)
    Xd[:, 3] = Xd[:, 0] + Xd[:, 1]
    note("rank revealing", gram, "8,000,000 x [10 | 4]")
    Q, R, C, it, info = borth.orthonormalize_iter(Xd, Yd, gram=gram, fact="svqb", eps=1e-10,
                                                  max_iter=8, rank_reveal=True)
    note("  ", it)
    assert info.status == 0 and it.converged and it.rank == 3
    Qh, Y = host(Q), host(Yd)
    assert np.all(Qh[:, 3] == 0.0)
    for i in range(3):
        for j in range(i, 3):
            hi, lo = oracle.gram_q(np.ascontiguousarray(np.stack([Qh[:, i], Qh[:, j]], axis=1)))
            assert abs((hi[0, 1] - (1.0 if i == j else 0.0)) + lo[0, 1]) <= 20 * 4 * U64
    for i in (0, 4, 9):
        for j in range(3):
            hi, lo = oracle.gram_q(np.ascontiguousarray(np.stack([Y[:, i], Qh[:, j]], axis=1)))
            assert abs(hi[0, 1] + lo[0, 1]) <= 1e-14
    res = Xd - Yd @ C - Q @ R
    assert float(torch.linalg.norm(res)) <= 1e3 * 4 * U64 * float(torch.linalg.norm(Xd))


@pytest.mark.parametrize("k", [32, 64])
def test_c2_f64_cholqr2_full(k):
    borth = lib()
    m = 10_000_000
    Xd, X = _svd_x(m, k, 1e6, 200 + k)
    note(f"binary64 CholQR2 {m} x {k}")
    Q, R, _, info = borth.orthonormalize(Xd, gram="f64", passes=2)
    assert info.status == 0, info
    met = _metrics(Q, X, R)
    assert met["omega"] <= 1e-14 and met["rho"] <= 1e-14, met


def _c4():
    import torch
    return _svd_x(16_777_216, 64, 1e6, 401, dtype=torch.float32)


def test_c4_split_gram_full():
    """Stage 1: the split-BF16 Gram matrix of the fp32 X against the exact
    Gram matrix of its binary64 widening (oracle Dot2 sums, error ~u^2):
    elementwise within 4 * 2^-16 (|X|^T |X|)_ij, as the two-term split
    leaves the lo*lo term and the remainder below bf16."""
    borth = lib()
    Xd, X32 = _c4()
    X = X32.astype(np.float64)
    note("split Gram 16,777,216 x 64")
    ghi, _ = borth.gram(Xd, prec="split")
    ex_hi, ex_lo = oracle.gram_dot2(X)
    g = host(ghi)
    absg = np.abs(X).T @ np.abs(X)
    rel = np.abs((g - ex_hi) - ex_lo) / absg
    note("  max elementwise", rel.max(), "normwise",
         np.linalg.norm((g - ex_hi) - ex_lo) / np.linalg.norm(ex_hi))
    assert rel.max() <= 4 * 2.0 ** -16


@pytest.mark.parametrize("passes", [2, 3])
def test_c4_split_refinement_full(passes):
    """Stages 2 and 3: after the shifted split pass, one binary64 pass leaves
    omega_1 ~ kappa(Q_1)^2 u (kappa(Q_1) about sqrt(shift) / sigma_min:
    gated at 1e-6), a second one omega_2 <= 1e-14; rho <= 1e-14 for both."""
    borth = lib()
    Xd, X32 = _c4()
    note(f"split + {passes - 1} binary64 pass(es), 16,777,216 x 64")
    Q, R, _, info = borth.orthonormalize(Xd, gram="split", passes=passes)
    assert info.status == 0, info
    met = _metrics(Q, X32.astype(np.float64), R)
    assert met["rho"] <= 1e-14, met
    assert met["omega"] <= (1e-6 if passes == 2 else 1e-14), met


@pytest.mark.parametrize("persistent", [False, True])
def test_c5_tallest_blocks_full(persistent, monkeypatch, capfd):
    """The eight tallest blocks of the 256-block batch (rows up to 1e6,
    widths from {8, 16, 32, 64}, kappa log-uniform in [1e3, 1e10]) with
    their 16-column locked bases, one batched DD CholQR2 call (P,C,P,C),
    with one launch per phase or as the single persistent launch: per block
    omega, rho and omega_Y <= 1e-14."""
    monkeypatch.setenv("BORTH_LOG", "1")
    borth = lib()
    torch = torch_gpu()
    table = synth.batch_table(256, seed=5000)
    tall = sorted(table, key=lambda t: -t["m"])[:8]
    ky = 16
    blocks, hostb = [], []
    for t in tall:
        note(f"block m={t['m']} k={t['k']} kappa={t['kappa']:.3g} seed={t['seed']}")
        X = synth.svd_matrix_device(t["m"], t["k"], t["kappa"], t["seed"])
        Y = synth.locked_basis_device(t["m"], ky, t["seed"] + 100_000)
        blocks.append({"X": X, "Y": Y})
    torch.cuda.synchronize()
    note("batched DD CholQR2 of 8 full-height blocks, persistent =", persistent)
    capfd.readouterr()
    outs, infos = borth.batch_orthonormalize(blocks, gram="dd", passes=2, persistent=persistent)
    drivers = [int(x) for x in re.findall(r"borth: batch .*persistent=(\d)", capfd.readouterr().err)]
    assert drivers == [int(persistent)]
    for t, b, (Q, R, C), inf in zip(tall, blocks, outs, infos):
        assert inf.status == 0, (t, inf)
        met = oracle.metrics(host(Q), host(b["X"]), host(R), host(b["Y"]), host(C))
        note("  block", t["m"], t["k"], {k: float(v) for k, v in met.items()})
        assert met["omega"] <= 1e-14 and met["rho"] <= 1e-14 and met["omega_y"] <= 1e-14, (t, met)
