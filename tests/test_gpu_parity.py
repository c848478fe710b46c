"""GPU parity tests: every step of the HIP path against the CPU oracle.

Tolerances (derived from the arithmetic, stated per test):
* binary64 Gram: elementwise |dG_ij| <= gamma_n (|X|^T|X|)_ij with n the
  longest serial accumulation chain of the kernels (rows per accumulator plus
  the fixed reduction tree), and normwise ||dG||_F / ||G||_F <= 1e-14.
* DD Gram: elementwise |dG_ij| <= gamma_n^2 (|X|^T|X|)_ij + 4u^2 |G_ij| (the
  Dot2 bound, which the biased accumulation's per-panel bound
  (n_p + n_p^2) u^2 sigma also meets at these sizes) and normwise <= 1e-28;
  at a million rows, max |dG_ij| <= 2e-30 sqrt(G_ii G_jj).
* update: |dQ_ij| <= (2(k + ky) + 2) u ((|X| + |Y||C|)|Z|)_ij.
* end to end: reconstruction rho and orthogonality omega <= 1e-14 where the
  method guarantees it; bitwise equality on the exact Hadamard families.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import U64, dev, host, lib, note, rel_fro, torch_gpu

pytestmark = pytest.mark.gpu


def gamma(n):
    return n * U64 / (1 - n * U64)


def chain(m):
    return m // 4 + 1100


# ---------------------------------------------------------------------------
# a2: Gram sweeps

@pytest.mark.parametrize("m,k,ky", [(5003, 4, 0), (5003, 8, 0), (5003, 16, 0), (5003, 20, 0),
                                    (7001, 32, 0), (7001, 64, 0), (5003, 8, 5), (6007, 32, 16),
                                    (3001, 64, 16), (1, 3, 0), (17, 1, 0), (4001, 3, 2),
                                    (100_003, 8, 0), (100_003, 4, 0), (150_001, 4, 40),
                                    (5, 4, 2), (300, 2, 0)])
@pytest.mark.parametrize("prec", ["f64", "dd", "dd_dot2"])
def test_gram_vs_oracle(m, k, ky, prec):
    borth = lib()
    note("gram", m, k, ky, prec)
    rng = np.random.default_rng(1000 + m + k + ky)
    X = rng.standard_normal((m, k)) * np.ldexp(1.0, rng.integers(-3, 3, (1, k)))
    Y = rng.standard_normal((m, ky)) if ky else None
    V = X if Y is None else np.hstack([Y, X])
    ghi, glo = borth.gram(dev(X), None if Y is None else dev(Y), prec=prec)
    ghi = host(ghi)
    glo = host(glo) if glo is not None else np.zeros_like(ghi)
    ex_hi, ex_lo = oracle.gram_q(V)
    absg = np.abs(V).T @ np.abs(V)
    err = np.abs((ghi - ex_hi) + (glo - ex_lo))
    if prec == "f64":
        assert np.all(err <= gamma(chain(m)) * absg + 1e-300)
        assert rel_fro(ghi, ex_hi + ex_lo) <= 1e-14
    else:
        assert np.all(err <= gamma(chain(m)) ** 2 * absg + 4 * U64 ** 2 * np.abs(ex_hi))
        assert np.linalg.norm(err) <= 1e-28 * np.linalg.norm(ex_hi)
    assert np.array_equal(ghi, ghi.T)


def test_gram_strided_and_deterministic():
    borth = lib()
    torch = torch_gpu()
    rng = np.random.default_rng(7)
    big = rng.standard_normal((9000, 40))
    Xd = dev(big)[:, 3:35]  # ld = 40, k = 32
    g1, l1 = borth.gram(Xd, prec="dd")
    g2, l2 = borth.gram(Xd, prec="dd")
    torch.cuda.synchronize()
    assert torch.equal(g1, g2) and torch.equal(l1, l2)
    ex_hi, ex_lo = oracle.gram_q(big[:, 3:35])
    assert np.linalg.norm(host(g1) - ex_hi + host(l1) - ex_lo) <= 1e-28 * np.linalg.norm(ex_hi)


def test_gram_near_parallel_dd_exact():
    """Exact Gram [[1,1],[1,1+2^-80]]: the DD sweep must return it exactly;
    a contracted TwoSum would lose the 2^-80."""
    borth = lib()
    X = synth.hadamard_near_parallel(8, 4, 40)
    ghi, glo = borth.gram(dev(X), prec="dd")
    ex_hi, ex_lo = oracle.gram_q(X)
    assert np.array_equal(host(ghi), ex_hi) and np.array_equal(host(glo), ex_lo)


@pytest.mark.parametrize("m,k,ky", [(1_000_000, 32, 0), (400_000, 4, 40), (250_000, 64, 0)])
def test_gram_dd_accuracy_large(m, k, ky):
    """The DD sweep at sizes where every thread folds many panels (biased
    accumulation, one to many row phases): the error against the exact Gram
    stays at the double-double level, max |dG_ij| <= 2e-30 sqrt(G_ii G_jj)
    (measured 2.6e-31 at most, Dot2 about 5e-32), columns graded by 1e-5."""
    borth = lib()
    note("gram dd large", m, k, ky)
    rng = np.random.default_rng(4100 + k + ky)
    V = rng.standard_normal((m, ky + k))
    V[:, 1::3] *= 1e-5
    Y = V[:, :ky] if ky else None
    ghi, glo = borth.gram(dev(V[:, ky:]), None if Y is None else dev(Y), prec="dd")
    ex_hi, ex_lo = oracle.gram_q(V)
    err = np.abs((host(ghi) - ex_hi) + (host(glo) - ex_lo))
    d = np.sqrt(np.diag(ex_hi))
    rel = err / np.outer(d, d)
    note("  max", rel.max(), "rms", np.sqrt(np.mean(rel ** 2)))
    assert rel.max() <= 2e-30
    assert np.sqrt(np.mean(rel ** 2)) <= 2e-31


@pytest.mark.parametrize("kxy", [1e9, 1e12])
def test_gram_dd_accumulations_near_span(kxy):
    """X close to span(Y) on the paper's accuracy-experiment shape (1000 x
    [20 | 4]): few panels are summed, so the per-panel error of the biased
    accumulation shows.  Against the exact Gram: Dot2 stays at a few u^2
    (measured 2.5e-32 relative to sqrt(G_ii G_jj)), the biased sums at the
    rows x u^2 sigma level (measured 5e-31)."""
    borth = lib()
    for rep in range(3):
        X, Y = synth.projected_pair(1000, 4, 20, 1.0, kxy, 7700 + rep)
        V = np.hstack([Y, X])
        ex_hi, ex_lo = oracle.gram_q(V)
        d = np.sqrt(np.diag(ex_hi))
        for prec, bound in (("dd_dot2", 2e-31), ("dd", 4e-30)):
            ghi, glo = borth.gram(dev(X), dev(Y), prec=prec)
            rel = np.abs((host(ghi) - ex_hi) + (host(glo) - ex_lo)) / np.outer(d, d)
            note("near span", kxy, rep, prec, rel.max())
            assert rel.max() <= bound


def test_gram_split_bf16_vs_oracle():
    """Split-BF16 Gram: within 3 * 2^-16 (dropped l*l term and unsplit remainder)
    of the exact Gram, and within fp32-accumulation noise of the oracle's
    split model."""
    borth = lib()
    torch = torch_gpu()
    m, k = 40000, 64
    X = synth.svd_matrix(m, k, 1e3, 401).astype(np.float32)
    X64 = X.astype(np.float64)
    ghi, _ = borth.gram(dev(X), prec="split")
    g = host(ghi)
    ex = oracle.gram_q(X64)[0]
    absg = np.abs(X64).T @ np.abs(X64)
    assert np.all(np.abs(g - ex) <= 4 * 2.0 ** -16 * absg)
    model = oracle.gram_split_bf16(X, chunk=32)
    assert np.all(np.abs(g - model) <= (96 + 32) * 2.0 ** -24 * absg)
    # not the plain product: a missing cross term would be ~2^-8 off
    assert np.max(np.abs(g - ex) / absg) > 1e-9


# ---------------------------------------------------------------------------
# a3: small factorization

@pytest.mark.parametrize("k,ky,kappa,dd", [(8, 0, 1e3, False), (32, 0, 1e3, False),
                                           (64, 0, 1e3, False), (32, 0, 1e12, True),
                                           (64, 0, 1e14, True), (20, 16, 1e6, True),
                                           (33, 7, 1e4, False)])
def test_factor_vs_oracle(k, ky, kappa, dd):
    borth = lib()
    note("factor", k, ky, kappa, dd)
    m = 4000
    X = synth.svd_matrix(m, k, kappa, 300 + k)
    Y = synth.locked_basis(m, ky, 99) if ky else None
    V = X if Y is None else np.hstack([Y, X])
    ghi, glo = oracle.gram_q(V)
    Z, R, C, info = borth.factor(dev(ghi), dev(glo) if dd else None, ky=ky)
    assert info.status == 0
    Z, R, C = host(Z), host(R), host(C)
    # oracle: exact M = Xt^T Xt of the projected block, its Cholesky and inverse
    o = oracle.qr_q(X, Y, want_gram=True)
    rex, _, inf2 = oracle.chol_q(o["G_hi"], o["G_lo"])
    assert inf2 == 0
    zex, _ = oracle.trinv_q(rex)
    # backward error of the returned R (binary64 words): ||R^T R - M|| / ||M||
    # <= 2 (k + 1) sqrt(k) u  (Cholesky backward stability + output rounding)
    rtr_hi, rtr_lo = oracle.gram_q(R)
    bw = np.linalg.norm(rtr_hi - o["G_hi"] + (rtr_lo - o["G_lo"])) / np.linalg.norm(o["G_hi"])
    assert bw <= 2 * (k + 1) * np.sqrt(k) * U64, bw
    # forward errors: worst case kappa(M) times the working precision
    uw = 2.0 ** -104 if dd else U64
    tol = 10 * k * (U64 + kappa ** 2 * uw)
    assert rel_fro(R, rex) <= tol, rel_fro(R, rex)
    assert rel_fro(Z, zex) <= tol * kappa, rel_fro(Z, zex)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.tril(Z, -1) == 0)
    if ky:
        assert np.array_equal(C, (ghi + glo)[:ky, ky:]) or rel_fro(C, ghi[:ky, ky:]) <= 1e-15


def test_factor_breakdown_pivot():
    borth = lib()
    G = np.array([[4.0, 2.0, 1.0], [2.0, 1.0, 3.0], [1.0, 3.0, 9.0]])
    _, _, _, info = borth.factor(dev(G), None, check=False)
    assert info.status == 4 and info.failed_pivot == 2
    G2 = G.copy()
    G2[0, 0] = np.nan
    _, _, _, info = borth.factor(dev(G2), None, check=False)
    assert info.status == 5


def test_factor_svqb_vs_oracle():
    borth = lib()
    m, k = 3000, 16
    X = synth.svd_matrix(m, k, 1e4, 55)
    ghi, glo = oracle.gram_q(X)
    Z, R, _, info = borth.factor(dev(ghi + glo), None, fact="svqb")
    assert info.status == 0
    zex, lam, _ = oracle.svqb_q(ghi, glo)
    assert rel_fro(host(Z), zex) <= 1e-15 * 1e8 * 10  # kappa(M) u
    assert np.allclose(host(Z), host(Z).T, rtol=0, atol=1e-12 * np.abs(zex).max())


@pytest.mark.parametrize("k,kappa,ky", [(4, 1e6, 0), (16, 1e10, 0), (33, 1e6, 0), (8, 1e5, 12),
                                         (64, 1e3, 0)])
def test_factor_svqb_dd_vs_oracle(k, kappa, ky):
    """DD SVQB: Jacobi, Z = M^{-1/2} and R = M^{1/2} in DD from the DD Gram
    of [Y | X].  The oracle's binary128 Jacobi on the same M (formed in
    binary128 from the same Gram) gives the same Z to a few ulps: the DD
    transform carries kappa(M) u_DD (below binary64 rounding up to
    kappa(M) ~ 1e16), where binary64 SVQB is off by kappa(M) u."""
    borth = lib()
    m = 3000
    X = synth.svd_matrix(m, k, kappa, 56 + k)
    if ky:
        Y = synth.locked_basis(m, ky, 57)
        X = X + Y @ np.random.default_rng(58).standard_normal((ky, k))
        ghi, glo = oracle.gram_q(np.hstack([Y, X]))
    else:
        ghi, glo = oracle.gram_q(X)
    Z, R, C, info = borth.factor(dev(ghi), dev(glo), ky=ky, fact="svqb")
    assert info.status == 0
    # the oracle's M: the exact projected Gram (binary128), as hi/lo
    if ky:
        Xt = X - Y @ oracle.qr_q(X, Y)["C"]
        mhi, mlo = oracle.gram_q(Xt)
        # binary128 Gram of the rounded Xt differs from the projected Gram by
        # rounding of Xt: compare at that level instead of ulps
        zex, lam, _ = oracle.svqb_q(mhi, mlo)
        tol = 1e3 * U64 * kappa
    else:
        zex, lam, _ = oracle.svqb_q(ghi, glo)
        # the DD rotations carry u_DD |M|, i.e. kappa(M) u_DD relative to
        # the smallest eigenvalue (kappa(M) = kappa^2)
        tol = 8 * U64 + 100 * kappa ** 2 * 2.0 ** -106
    Zh = host(Z)
    note(" dd svqb", k, kappa, ky, rel_fro(Zh, zex))
    assert rel_fro(Zh, zex) <= tol
    assert np.max(np.abs(Zh - Zh.T)) <= 2 * U64 * np.max(np.abs(Zh))


def test_factor_svqb_near_identity_k64():
    """Second-pass shape: M = Q_1^T Q_1 with ||M - I|| ~ 1e-10 at k = 64
    (2016 rotations per sweep).  Z must stay within O(k u) of the exact
    M^{-1/2} (binary128 Jacobi of the oracle): sweeps over off-diagonal
    entries at rounding level must not keep rotating and feed noise into V."""
    borth = lib()
    rng = np.random.default_rng(64)
    X = synth.svd_matrix(20000, 64, 1.0, 65) + 1e-10 * rng.standard_normal((20000, 64))
    ghi, glo = oracle.gram_q(X)
    M = ghi + glo
    Z, _, _, info = borth.factor(dev(M), None, fact="svqb")
    assert info.status == 0
    zex, lam, _ = oracle.svqb_q(ghi, glo)
    Zh = host(Z)
    note(" svqb k=64 near identity:", rel_fro(Zh, zex))
    assert rel_fro(Zh, zex) <= 10 * 64 * U64
    assert np.linalg.norm(Zh.T @ M @ Zh - np.eye(64)) <= 20 * 64 * U64


# ---------------------------------------------------------------------------
# a4: update sweep

@pytest.mark.parametrize("m,k,ky,dense", [(5003, 4, 0, False), (5003, 8, 3, False),
                                          (7001, 16, 16, False), (7001, 32, 0, False),
                                          (3001, 64, 16, False), (4099, 20, 5, True),
                                          (6007, 64, 0, False), (6007, 48, 0, True),
                                          (5003, 37, 0, False), (17, 64, 0, False),
                                          (6007, 64, 10, True), (4093, 50, 6, False),
                                          (4093, 64, 7, False), (23, 64, 16, False),
                                          (6007, 32, 16, False), (5003, 24, 10, True),
                                          (4093, 32, 7, False), (29, 32, 16, False),
                                          (1, 5, 0, False)])
def test_update_vs_oracle(m, k, ky, dense):
    borth = lib()
    note("update", m, k, ky, dense)
    rng = np.random.default_rng(2000 + m + k)
    X = rng.standard_normal((m, k))
    Y = rng.standard_normal((m, ky)) if ky else None
    C = rng.standard_normal((ky, k)) if ky else None
    Z = rng.standard_normal((k, k))
    if not dense:
        Z = np.triu(Z)
    Q = host(borth.update(dev(X), dev(Z), None if Y is None else dev(Y),
                          None if C is None else dev(C), dense=dense))
    ex = oracle.update_q(X, Z, Y, C)
    mag = np.abs(X) + (np.abs(Y) @ np.abs(C) if ky else 0)
    bound = (2 * (k + ky) + 2) * U64 * (mag @ np.abs(Z)) + U64 * np.abs(ex)
    assert np.all(np.abs(Q - ex) <= bound)


@pytest.mark.parametrize("m,k,ky,dense,strided", [
    (5003, 1, 10, False, False), (5003, 2, 20, True, False), (5003, 4, 40, False, False),
    (4099, 3, 17, False, False), (4099, 5, 33, True, False), (4099, 8, 64, False, False),
    (4099, 1, 0, False, False), (4099, 4, 1, False, False), (4099, 2, 63, False, True),
    (130, 4, 16, True, True), (65, 1, 64, False, False), (63, 8, 7, False, True),
    (64, 4, 40, False, False), (1, 1, 0, False, False)])
def test_update_narrow_vs_oracle(m, k, ky, dense, strided):
    """Narrow blocks (k <= 8, any ky <= 64) take the vector-ALU stream kernel:
    ragged panels, every Y width class, odd widths, and row strides larger
    than the widths (then the flat loads of a panel are not contiguous)."""
    borth = lib()
    torch = torch_gpu()
    note("update narrow", m, k, ky, dense, strided)
    rng = np.random.default_rng(3000 + m + 7 * k + ky)
    X = rng.standard_normal((m, k))
    Y = rng.standard_normal((m, ky)) if ky else None
    C = rng.standard_normal((ky, k)) if ky else None
    Z = rng.standard_normal((k, k))
    if not dense:
        Z = np.triu(Z)

    def place(A, extra):
        if A is None or not strided:
            return None if A is None else dev(A)
        W = dev(np.hstack([A, np.full((A.shape[0], extra), np.nan)]))
        return W[:, :A.shape[1]]

    Xd, Yd = place(X, 3), place(Y, 5)
    out = torch.full((m, k + (2 if strided else 0)), np.nan, dtype=torch.float64,
                     device="cuda")[:, :k]
    Q = host(borth.update(Xd, dev(Z), Yd, None if C is None else dev(C), dense=dense, out=out))
    ex = oracle.update_q(X, Z, Y, C)
    mag = np.abs(X) + (np.abs(Y) @ np.abs(C) if ky else 0)
    bound = (2 * (k + ky) + 2) * U64 * (mag @ np.abs(Z)) + U64 * np.abs(ex)
    assert np.all(np.abs(Q - ex) <= bound)
    if strided:  # nothing written outside the k columns
        assert torch.isnan(out.as_strided((m, 2), (k + 2, 1), out.storage_offset() + k)).all()


def test_update_inplace_and_fp32():
    borth = lib()
    torch = torch_gpu()
    rng = np.random.default_rng(5)
    X = rng.standard_normal((3001, 32))
    Z = np.triu(rng.standard_normal((32, 32)))
    Xd = dev(X)
    borth.update(Xd, dev(Z), out=Xd)
    ex = oracle.update_q(X, Z)
    assert np.max(np.abs(host(Xd) - ex)) <= 100 * U64 * np.max(np.abs(X) @ np.abs(Z))
    X32 = X.astype(np.float32)
    Q = borth.update(dev(X32), dev(Z))
    ex32 = oracle.update_q(X32.astype(np.float64), Z)
    assert np.max(np.abs(host(Q) - ex32)) <= 100 * U64 * np.max(np.abs(X) @ np.abs(Z))


@pytest.mark.parametrize("k", [64, 40, 42])
def test_update_wide_inplace_and_fp32(k):
    """Padded width 64 without Y: panels by direct transfers into one buffer
    per wave (binary64 rows with even k, fp32 rows with k a multiple of 4),
    the other widths by loads; in place, out of place, fp32 input, and a
    ragged last panel."""
    borth = lib()
    rng = np.random.default_rng(70 + k)
    m = 4093
    X = rng.standard_normal((m, k))
    Z = np.triu(rng.standard_normal((k, k)))
    ex = oracle.update_q(X, Z)
    tol = 100 * U64 * np.max(np.abs(X) @ np.abs(Z))
    Q = host(borth.update(dev(X), dev(Z)))
    assert np.max(np.abs(Q - ex)) <= tol
    Xd = dev(X)
    borth.update(Xd, dev(Z), out=Xd)
    assert np.max(np.abs(host(Xd) - ex)) <= tol
    X32 = X.astype(np.float32)
    Q = borth.update(dev(X32), dev(Z))
    ex32 = oracle.update_q(X32.astype(np.float64), Z)
    assert np.max(np.abs(host(Q) - ex32)) <= tol


# ---------------------------------------------------------------------------
# a5: the whole path

@pytest.mark.parametrize("gram,passes,sched,fact", [
    ("f64", 1, "auto", "chol"), ("f64", 2, "recompute", "chol"), ("f64", 2, "materialize", "chol"),
    ("dd", 1, "auto", "chol"), ("dd", 2, "recompute", "chol"), ("dd", 2, "materialize", "chol"),
    ("dd", 3, "materialize", "chol"), ("f64", 2, "materialize", "svqb"), ("f64", 1, "auto", "svqb")])
def test_hadamard_bitwise(gram, passes, sched, fact):
    """X = H diag(2^e): exact Q = H, R = diag(2^e); every unshifted mode must
    return them bitwise (all sums, square roots and inverses are exact)."""
    borth = lib()
    # SVQB lifts eigenvalues below 2^-52 lambda_max (rank rule): keep the
    # scale range inside it for SVQB; Cholesky takes the full 2^61 range.
    exps = [0, -3, 7, -20, 11, -35, 2, -50] if fact == "chol" else [0, -3, 7, -9, 11, -5, 2, -12]
    X = synth.hadamard_scaled(7, exps)
    H = synth.hadamard_columns(7, range(1, 1 + len(exps)))
    Q, R, _, info = borth.orthonormalize(dev(X), gram=gram, passes=passes, sched=sched, fact=fact)
    assert info.status == 0
    assert np.array_equal(host(Q), H)
    assert np.array_equal(host(R), np.diag(np.ldexp(1.0, exps)))


def test_hadamard_projection_bitwise():
    borth = lib()
    j = 6
    Y = synth.hadamard_columns(j, [40, 41, 42, 43])
    H = synth.hadamard_columns(j, [1, 2, 3])
    Cex = np.array([[1.0, -2.0, 0.5], [0.25, 3.0, 0.0], [1.0, 1.0, 1.0], [0.0, -4.0, 2.0]])
    X = H * 8.0 + Y @ Cex
    for gram in ("f64", "dd"):
        Q, R, C, info = borth.orthonormalize(dev(X), dev(Y), gram=gram)
        assert info.status == 0
        assert np.array_equal(host(Q), H) and np.array_equal(host(R), 8.0 * np.eye(3))
        assert np.array_equal(host(C), Cex)


def test_near_parallel_dd_vs_f64():
    """kappa ~ 2^41: DD CholQR2 returns the exact Q within a few ulps; the
    binary64 Gram cannot hold 1 + 2^-80, so plain CholQR breaks down or is
    far from orthogonal."""
    borth = lib()
    X = synth.hadamard_near_parallel(7, 4, 40)
    H = synth.hadamard_columns(7, range(1, 5))
    Q, R, _, info = borth.orthonormalize(dev(X), gram="dd", passes=2)
    assert info.status == 0
    assert np.max(np.abs(host(Q) - H)) <= 8 * U64 * np.abs(H).max()
    Q2, R2, _, info2 = borth.orthonormalize(dev(X), gram="f64", passes=1, check=False)
    if info2.status == 0:
        assert oracle.metrics(host(Q2), X, host(R2))["omega"] > 1e-6
    else:
        assert info2.status == 4 and info2.failed_pass == 1


def _check_qr(X, Q, R, Y=None, C=None, omega=1e-14, rho=1e-14):
    met = oracle.metrics(Q, X, R, Y, C)
    note(" metrics", met)
    assert met["rho"] <= rho, met
    assert met["omega"] <= omega, met
    if Y is not None:
        assert met["omega_y"] <= omega, met
    return met


def test_cholqr_plain_c1_shape():
    """Plain binary64 CholQR at the 20000 x 8 workload (kappa = 1e4, and
    1e3 for the slope), against the oracle.  One pass loses about
    c kappa^2 times the relative rounding error of the Gram matrix plus that
    of the Cholesky factor (the published c kappa^2 u law).  The oracle
    brackets the loss by two binary64 passes that differ only in the Gram
    matrix: summed in binary64 over row blocks in order, and the binary128
    Gram matrix rounded once.  The GPU's Gram matrix (short chains combined
    by fixed trees) must be at least as accurate as the oracle's binary64
    sum, and its loss must lie in that bracket widened by 4 on each side."""
    borth = lib()
    for seed in (101, 102, 103):
        om = {}
        for kappa in (1e3, 1e4):
            X = synth.svd_matrix(20000, 8, kappa, seed)
            note("plain CholQR", seed, kappa)
            Q, R, _, info = borth.orthonormalize(dev(X), gram="f64", passes=1)
            assert info.status == 0
            met = _check_qr(X, host(Q), host(R), omega=1.0)
            o_f = oracle.cholqr_steps(X, passes=1)
            o_e = oracle.cholqr_steps(X, passes=1, exact_gram=True)
            om_f = oracle.metrics(o_f["Q"], X, o_f["R_hi"])["omega"]
            om_e = oracle.metrics(o_e["Q"], X, o_e["R_hi"])["omega"]
            ghi, _ = borth.gram(dev(X), prec="f64")
            ex_hi, ex_lo = oracle.gram_q(X)
            nrm = np.linalg.norm(ex_hi)
            e_gpu = np.linalg.norm((host(ghi) - ex_hi) - ex_lo) / nrm
            e_o2 = np.linalg.norm((oracle.gram_f64(X) - ex_hi) - ex_lo) / nrm
            note("  omega gpu", met["omega"], "oracle binary64 Gram", om_f,
                 "oracle rounded exact Gram", om_e, "Gram error gpu", e_gpu, "oracle", e_o2)
            assert e_gpu <= max(2.0 * e_o2, U64)
            assert om_e / 4 <= met["omega"] <= 4 * om_f
            om[kappa] = met["omega"]
        assert 10 <= om[1e4] / om[1e3] <= 1000  # kappa^2 predicts 100
    X = synth.svd_matrix(20000, 8, 1e4, 101)
    Q, R, _, info = borth.orthonormalize(dev(X), gram="f64", passes=1)
    o1 = oracle.qr_q(X)
    assert rel_fro(host(R), o1["R"]) <= 1e-14 * 1e4


@pytest.mark.parametrize("k", [4, 8, 16, 32, 64])
def test_cholqr2_f64_kappa_1e6(k):
    borth = lib()
    X = synth.svd_matrix(60000, k, 1e6, 200 + k)
    for sched in ("recompute", "materialize"):
        Q, R, _, info = borth.orthonormalize(dev(X), gram="f64", passes=2, sched=sched)
        assert info.status == 0
        _check_qr(X, host(Q), host(R))


@pytest.mark.parametrize("kappa", [1e8, 1e12, 1e15])
def test_cholqr2_dd_high_kappa(kappa):
    borth = lib()
    X = synth.svd_matrix(50000, 32, kappa, 301)
    Q, R, _, info = borth.orthonormalize(dev(X), gram="dd", passes=2)
    assert info.status == 0
    _check_qr(X, host(Q), host(R))
    # the binary64 comparator on the same input
    Qf, Rf, _, inf = borth.orthonormalize(dev(X), gram="f64", passes=2, check=False)
    if kappa >= 1e12:
        if inf.status == 0:
            assert oracle.metrics(host(Qf), X, host(Rf))["omega"] > 1e-14
        else:
            assert inf.status == 4


@pytest.mark.parametrize("k,kappa,project_once", [(8, 1e3, False), (32, 1e9, False),
                                                  (16, 1e6, True), (64, 1e5, False)])
def test_projection_dd_cholqr2(k, kappa, project_once):
    borth = lib()
    m = 40000
    X = synth.svd_matrix(m, k, kappa, 500 + k)
    Y = synth.locked_basis(m, 16, 600 + k)
    Q, R, C, info = borth.orthonormalize(dev(X), dev(Y), gram="dd", passes=2,
                                         project_once=project_once)
    assert info.status == 0
    om = 1e-13 if project_once else 1e-14  # P,C,C: Y^T Q grows by ||R^{-1}|| u
    met = oracle.metrics(host(Q), X, host(R), Y, host(C))
    note(" metrics", met)
    assert met["rho"] <= 1e-14 and met["omega"] <= 1e-14
    if not project_once:
        assert met["omega_y"] <= om
    o1 = oracle.qr_q(X, Y)
    # C_tot = C_1 + C_2 R_1 carries ~u ||R_1|| = u sigma_max(X) (sigma_max = 1 here)
    assert np.max(np.abs(host(C) - o1["C"])) <= 1e-13


def test_split_bf16_refinement_c4_shape():
    """fp32 X, split-BF16 Gram, shifted Cholesky, then binary64 passes:
    per-stage tolerance -- after one refinement pass omega <= 1e-6
    (kappa(Q_1)^2 u with kappa(Q_1) ~ sqrt(shift)/sigma_min), after two <= 1e-14."""
    borth = lib()
    m, k = 200000, 64
    X = synth.svd_matrix(m, k, 1e6, 401).astype(np.float32)
    X64 = X.astype(np.float64)
    Q, R, _, info = borth.orthonormalize(dev(X), gram="split", passes=2)
    assert info.status == 0
    met = oracle.metrics(host(Q), X64, host(R))
    note(" split 2 passes", met)
    assert met["rho"] <= 1e-14 and met["omega"] <= 1e-6
    Q, R, _, info = borth.orthonormalize(dev(X), gram="split", passes=3)
    assert info.status == 0
    _check_qr(X64, host(Q), host(R))


# ---------------------------------------------------------------------------
# edge cases

def test_edges():
    borth = lib()
    torch = torch_gpu()
    # square and tiny
    X = synth.svd_matrix(8, 8, 10.0, 1)
    Q, R, _, info = borth.orthonormalize(dev(X), gram="dd")
    _check_qr(X, host(Q), host(R))
    # k = 1, ragged m
    X = np.random.default_rng(3).standard_normal((1001, 1))
    Q, R, _, info = borth.orthonormalize(dev(X))
    _check_qr(X, host(Q), host(R))
    # odd width and strided input
    big = np.random.default_rng(4).standard_normal((3003, 70))
    Xd = dev(big)[:, 2:65]
    Q, R, _, info = borth.orthonormalize(Xd, gram="dd")
    _check_qr(big[:, 2:65], host(Q), host(R))
    # in place
    X = synth.svd_matrix(5000, 16, 1e5, 9)
    Xd = dev(X)
    Q, R, _, info = borth.orthonormalize(Xd, out=Xd, sched="materialize")
    _check_qr(X, host(Xd), host(R))
    # rank deficient -> breakdown with the pivot of the duplicate column
    # (Hadamard columns: the Gram matrix and the pivots are exact, pivot 5 is 0)
    X = synth.hadamard_columns(6, [1, 2, 3, 4, 2, 5])
    for gram in ("f64", "dd"):
        _, _, _, info = borth.orthonormalize(dev(X), gram=gram, passes=1, check=False)
        assert info.status == 4 and info.failed_pass == 1 and info.failed_pivot == 5
    # non-finite input
    X = np.random.default_rng(6).standard_normal((4000, 6))
    X[17, 2] = np.nan
    _, _, _, info = borth.orthonormalize(dev(X), gram="dd", check=False)
    assert info.status == 5
    # argument errors before any launch
    with pytest.raises(borth.BorthError):
        borth.orthonormalize(dev(np.zeros((3, 5))))  # m < k
    with pytest.raises(borth.BorthError):
        borth.orthonormalize(dev(np.zeros((300, 65))))  # k > 64
    for bad in (float("nan"), float("inf")):
        with pytest.raises(borth.BorthError):
            borth.orthonormalize(dev(np.eye(300, 6)), shift=bad)
        with pytest.raises(borth.BorthError):
            borth.factor(dev(np.eye(6)), shift=bad)
    # tensors the binding rejects before any pointer reaches the library
    Xd = dev(np.eye(300, 6))
    bad_calls = [
        lambda: borth.orthonormalize(torch.zeros((300, 6), dtype=torch.float64)),  # host tensor
        lambda: borth.orthonormalize(Xd, out=dev(np.zeros((299, 6)))),  # short Q
        lambda: borth.orthonormalize(Xd, R=dev(np.zeros((6, 5)))),  # wrong R shape
        lambda: borth.orthonormalize(Xd, R=dev(np.zeros((6, 12)))[:, :6]),  # strided R
        lambda: borth.orthonormalize(Xd, dev(np.zeros((200, 2)))),  # Y rows != m
        lambda: borth.orthonormalize(Xd.to(torch.float16)),  # dtype
        lambda: borth.update(Xd, dev(np.eye(5))),  # Z shape
        lambda: borth.gram(Xd, dev(np.zeros((100, 2)))),  # A rows != m
        lambda: borth.batch_orthonormalize([{"X": Xd, "R": dev(np.zeros((5, 5)))}]),
        lambda: borth.orthonormalize(Xd, dev(np.zeros((2, 300))).t()),  # column-major Y
    ]
    for i, call in enumerate(bad_calls):
        with pytest.raises(borth.ArgumentError):
            call()


def test_deterministic_and_graph_replay():
    borth = lib()
    torch = torch_gpu()
    X = synth.svd_matrix(30000, 32, 1e10, 77)
    Xd = dev(X)
    Q1, R1, _, _ = borth.orthonormalize(Xd, gram="dd")
    Q2, R2, _, _ = borth.orthonormalize(Xd, gram="dd")
    assert torch.equal(Q1, Q2) and torch.equal(R1, R2)
    Qg = torch.empty_like(Q1)
    Rg = torch.empty_like(R1)
    for rep in range(4):
        Qg.fill_(0.0)
        borth.orthonormalize(Xd, gram="dd", graph=True, out=Qg, R=Rg)
        torch.cuda.synchronize()
        junk = torch.randn(1000, 1000, device="cuda", dtype=torch.float64).sum()  # eager work
        torch.cuda.synchronize()
        assert torch.equal(Qg, Q1) and torch.equal(Rg, R1), rep
        del junk
