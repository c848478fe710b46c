"""GPU tests of the iterated two-phase scheme (projection against Y and
orthonormalization alternated until a pass changes nothing, Sec. 4.2), on
the shape of the paper's runtime experiment (Fig. 8: few columns, a locked
basis of 10-40 vectors, kappa(X) = 1e6, X within 1e-12 of span(Y))."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import U64, dev, host, lib, note, torch_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,ky", [(1, 10), (2, 20), (4, 40)])
@pytest.mark.parametrize("gram,fact,kxy", [("f64", "svqb", 1e12), ("dd", "chol", 1e12),
                                           ("dd", "svqb", 1e12), ("f64", "chol", 1e4)])
def test_iterated_scheme_converges(k, ky, gram, fact, kxy):
    """binary64 Cholesky is run at kappa(X, Y) = 1e4 only: at 1e12 the
    projected Gram matrix (smallest eigenvalue ~1e-24 against an absolute
    binary64 error ~1e-16) is not positive definite and an unshifted
    Cholesky must break down -- the paper's binary64 variant uses SVQB."""
    borth = lib()
    m = 100_000
    X, Y = synth.projected_pair(m, k, ky, 1e6, kxy, 800 + 10 * k + ky)
    Q, R, C, it, info = borth.orthonormalize_iter(dev(X), dev(Y), gram=gram, fact=fact,
                                                  eps=1e-10, max_iter=8)
    note("iter", k, ky, gram, fact, it)
    assert info.status == 0 and it.converged and it.c_norm <= 1e-10 and it.r_dev <= 1e-10
    met = oracle.metrics(host(Q), X, host(R), Y, host(C))
    note("  metrics", met)
    assert met["rho"] <= 1e-14
    assert met["omega"] <= (20 * k * U64 if fact == "svqb" and gram == "f64" else 1e-14)
    assert met["omega_y"] <= 1e-14
    o1 = oracle.qr_q(X, Y)
    assert np.max(np.abs(host(C) - o1["C"])) <= 1e-13
    # The oracle's iterated scheme with the same steps: the same precision,
    # factor and stop test, and M from the Gram matrix of [Y | S] of one
    # sweep (the fused operations; its cancellation near span(Y) sets how
    # good the first pass is and so the number of passes).  The pass counts
    # agree unless a stop-test norm sits within a decade of eps at the pass
    # where they part.  kappa(X, Y) = ||X||_2 / sigma_min(Xt) is the paper's
    # kappa(X, W) (sigma_min from the exact Gram matrix of Xt via kappa_true).
    o2 = oracle.iterate(X, Y, gram=gram, fact=fact, eps=1e-10, max_iter=8, fused=True)
    Xt = X - Y @ (Y.T @ X)
    kxy = np.linalg.norm(X, 2) * oracle.kappa_true(X, Y) / np.linalg.norm(Xt, 2)
    Qg = host(Q)
    dq = np.max(np.abs(Qg - o2["Q"]))
    sin_max = np.linalg.norm(Qg - o2["Q"] @ (o2["Q"].T @ Qg), 2)  # largest principal angle
    note("  oracle passes", o2["passes"], "gpu", it.passes_run, "kappa(X, Y)", kxy, "max |dQ|", dq,
         "sin angle", sin_max)
    assert o2["info"] == 0 and o2["converged"]
    if it.passes_run != o2["passes"]:
        p = min(it.passes_run, o2["passes"])
        ob = oracle.iterate(X, Y, gram=gram, fact=fact, eps=1e-10, max_iter=p, fused=True)
        worst = max(ob["c_norm"], ob["r_dev"])
        note("  pass counts differ; oracle norms at pass", p, ob["c_norm"], ob["r_dev"])
        assert abs(it.passes_run - o2["passes"]) == 1 and 1e-11 <= worst <= 1e-9
    if gram == "f64" and fact == "svqb" and kxy ** 2 * U64 > 1e-6:
        # binary64 symmetric SVQB near span(Y): the first pass's M is
        # dominated by cancellation, the later passes' symmetric transforms
        # multiply to a non-symmetric one, and the result is another
        # orthonormal basis of the same span, known to ~u kappa(X, Y)
        assert sin_max <= 100 * kxy * U64
    else:
        # the thin QR factor is unique, and so is the symmetric SVQB result
        # when M is accurate: the same Q to the ~u kappa(X, Y) a binary64
        # projection leaves in Xt
        assert dq <= 100 * kxy * U64
    m2 = oracle.metrics(o2["Q"], X, o2["R_hi"] + o2["R_lo"], Y, o2["C_hi"] + o2["C_lo"])
    assert m2["omega_y"] <= 1e-14 and m2["omega"] <= 1e-14


@pytest.mark.parametrize("m,k,ky,strided", [(30011, 8, 0, False), (30011, 3, 7, False),
                                           (30011, 5, 59, False), (30011, 8, 60, False),
                                           (30011, 2, 12, True), (20000, 1, 63, False),
                                           (1000, 4, 16, False)])
@pytest.mark.parametrize("gram,fact", [("f64", "svqb"), ("dd", "chol")])
def test_iterated_scheme_layouts(m, k, ky, strided, gram, fact):
    """Narrow blocks with Y dense and ky even take the update with the Gram
    columns fused in; odd ky, ky + k > 64 and a strided Y take the separate
    sweep over [Y | X]^T X; ky = 0 is iterated CholQR / SVQB.  All reach the
    same levels."""
    borth = lib()
    torch = torch_gpu()
    X, Y = synth.projected_pair(m, k, ky, 1e6, 1e10, 1900 + 7 * k + ky) if ky else \
        (synth.svd_matrix(m, k, 1e6, 1900 + k), None)
    Yd = None
    if ky:
        Yd = dev(np.hstack([Y, np.zeros((m, 3))]))[:, :ky] if strided else dev(Y)
    Q, R, C, it, info = borth.orthonormalize_iter(dev(X), Yd, gram=gram, fact=fact, eps=1e-10,
                                                  max_iter=8)
    note("iter layouts", m, k, ky, strided, gram, fact, it)
    assert info.status == 0 and it.converged
    met = oracle.metrics(host(Q), X, host(R), Y, host(C) if ky else None)
    note("  metrics", met)
    # binary64 SVQB applies the dense symmetric Z as a product: its residual
    # carries k kappa u times the norm of the part it factors (CholQR's
    # triangular factor keeps it O(u)): kappa = 1e6 and, with Y present, the
    # part outside span(Y) has norm kappa(X) / kappa(X, Y) = 1e-4
    svqb_rho = 4 * k * 1e6 * U64 * (1e-4 if ky else 1.0)
    assert met["rho"] <= (max(1e-14, svqb_rho) if fact == "svqb" else 1e-14)
    assert met["omega"] <= (20 * k * U64 if fact == "svqb" else 1e-14)
    if ky:
        assert met["omega_y"] <= 1e-14
        assert np.max(np.abs(host(C) - oracle.qr_q(X, Y)["C"])) <= 1e-13


@pytest.mark.parametrize("gram,fact", [("f64", "svqb"), ("dd", "chol")])
def test_iterated_scheme_fused_matches_unfused(gram, fact):
    """Gram columns accumulated by the update (fused) and a full Gram sweep
    per pass (unfused) are the same arithmetic up to summation order: same
    passes, R and C agree to rounding, both reach the same levels."""
    borth = lib()
    X, Y = synth.projected_pair(60_000, 2, 20, 1e6, 1e12, 951)
    out = {}
    for fuse in (True, False):
        Q, R, C, it, info = borth.orthonormalize_iter(dev(X), dev(Y), gram=gram, fact=fact,
                                                      eps=1e-10, max_iter=8, fuse=fuse)
        assert info.status == 0 and it.converged
        met = oracle.metrics(host(Q), X, host(R), Y, host(C))
        note("fuse", fuse, gram, fact, it, met)
        assert met["rho"] <= 1e-14 and met["omega_y"] <= 1e-14
        assert met["omega"] <= (20 * 2 * U64 if fact == "svqb" else 1e-14)
        out[fuse] = (it.passes_run, host(R), host(C))
    assert out[True][0] == out[False][0]
    # R factors the part outside span(Y), kappa = 1e6: two valid roundings
    # differ by up to ~kappa u relative
    assert np.max(np.abs(out[True][1] - out[False][1])) <= 1e3 * 1e6 * U64 * np.max(np.abs(out[False][1]))
    assert np.max(np.abs(out[True][2] - out[False][2])) <= 1e-13


def test_iterated_scheme_dd_needs_fewer_passes():
    """The point of the paper's DD variant: the DD projection resolves X's
    tiny component outside span(Y) in one pass, so the scheme converges in
    fewer passes than in binary64."""
    borth = lib()
    X, Y = synth.projected_pair(100_000, 4, 20, 1e6, 1e12, 901)
    *_, it64, _ = borth.orthonormalize_iter(dev(X), dev(Y), gram="f64", fact="svqb", eps=1e-10,
                                            max_iter=10)
    *_, itdd, _ = borth.orthonormalize_iter(dev(X), dev(Y), gram="dd", fact="chol", eps=1e-10,
                                            max_iter=10)
    note("passes binary64", it64.passes_run, "DD", itdd.passes_run)
    assert it64.converged and itdd.converged
    assert itdd.passes_run < it64.passes_run


def test_iterated_scheme_limits_and_errors():
    borth = lib()
    X, Y = synth.projected_pair(50_000, 2, 10, 1e6, 1e12, 902)
    # one pass only, unreachable tolerance: reported as not converged
    Q, R, C, it, info = borth.orthonormalize_iter(dev(X), dev(Y), gram="dd", eps=0.0, max_iter=1)
    assert info.status == 0 and not it.converged and it.passes_run == 1
    # in place
    Xd = dev(X)
    Q, R, C, it, info = borth.orthonormalize_iter(Xd, dev(Y), gram="dd", out=Xd, max_iter=6)
    assert it.converged
    met = oracle.metrics(host(Xd), X, host(R), Y, host(C))
    assert met["rho"] <= 1e-14 and met["omega"] <= 1e-14 and met["omega_y"] <= 1e-14
    with pytest.raises(borth.BorthError):
        borth.orthonormalize_iter(dev(X), dev(Y), gram="split")
    with pytest.raises(borth.BorthError):
        borth.orthonormalize_iter(dev(X), dev(Y), max_iter=0)


@pytest.mark.parametrize("gram", ["f64", "dd"])
@pytest.mark.parametrize("k,ky,deps", [(4, 10, [(3, (0, 1))]), (8, 0, [(2, (0, 5)), (6, (1, 3))]),
                                       (3, 0, [])])
def test_iterated_scheme_rank_revealing(gram, k, ky, deps):
    """SVQB with rank revelation on blocks whose columns are exact linear
    combinations of others (each (j, (a, b)) sets column j to column a plus
    column b): the rank is k minus the number of dependent columns, the first
    rank columns of Q are orthonormal (and orthogonal to Y), the others are
    zero, X = Y C + Q R still holds, and the stop test converges."""
    borth = lib()
    m = 20011
    X, Y = (synth.projected_pair(m, k, ky, 1e3, 1e3, 3100 + k) if ky
            else (synth.svd_matrix(m, k, 1e3, 3100 + k), None))
    X = X.copy()
    for j, (a, b) in deps:
        X[:, j] = X[:, a] + X[:, b]
    Q, R, C, it, info = borth.orthonormalize_iter(dev(X), None if Y is None else dev(Y), gram=gram,
                                                  fact="svqb", eps=1e-10, max_iter=8,
                                                  rank_reveal=True)
    r = k - len(deps)
    note("rank revealing", gram, k, ky, deps, it)
    assert info.status == 0 and it.converged and it.rank == r
    Qh = host(Q)
    assert np.all(Qh[:, r:] == 0.0)
    Qr = Qh[:, :r].copy()
    g = oracle.gram_q(Qr)
    assert np.linalg.norm(g[0] - np.eye(r) + g[1]) <= 20 * k * U64
    if ky:
        gy = oracle.gram_q(Y, Qr)
        assert np.linalg.norm(gy[0] + gy[1]) <= 1e-14
    Rh = host(R)
    res = X - (Y @ host(C) if ky else 0) - Qh @ Rh
    assert np.linalg.norm(res) <= 1e3 * k * U64 * np.linalg.norm(X)
