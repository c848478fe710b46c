"""Pins for the CPU oracle: checks against things other than the oracle itself.

* brute force in exact rational arithmetic (Gram, LDL^T, inverse, update);
* exact worked families (Sylvester-Hadamard columns) whose QR is known;
* LAPACK Householder QR / Cholesky on well-conditioned inputs;
* closed forms of the generator (eigenvalues sigma^2, SVQB = polar factor);
* published error laws (plain CholQR ~ kappa^2 u, breakdown near 1e8;
  CholQR2 ~ u; Dot2 error bound) and Fig. 7's plotted levels.

Each pin is also run against a deliberately wrong result ("planted mistake")
to show that it would catch a dropped term, a sign error or a transposed
operand in the oracle.
"""
from fractions import Fraction
from pathlib import Path

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth
from _exact import F, dd_value, gram_exact, ldlt_exact

U64 = 2.0 ** -53
GOLDEN = Path(__file__).resolve().parent / "golden"


def _rand_exp_matrix(rng, m, k, spread=20):
    """Entries with widely varying exponents and signs."""
    return rng.standard_normal((m, k)) * np.ldexp(1.0, rng.integers(-spread, spread, (m, k)))


# --------------------------------------------------------------------------
# Gram products against exact rational sums

def gram_dd_err(hi, lo, A, B):
    """max_ij |(hi+lo)_ij - exact_ij| / (|A|^T |B|)_ij  (exact rationals)."""
    ex = gram_exact(A, B)
    absg = np.abs(A).T @ np.abs(B)
    worst = 0.0
    for i in range(hi.shape[0]):
        for j in range(hi.shape[1]):
            e = abs(dd_value(hi[i, j], None if lo is None else lo[i, j]) - ex[i][j])
            if absg[i, j] > 0:
                worst = max(worst, float(e / F(absg[i, j])))
    return worst


@pytest.mark.parametrize("m,ka,kb,seed", [(1, 1, 1, 0), (7, 3, 2, 1), (64, 4, 4, 2),
                                          (333, 5, 3, 3)])
def test_gram_q_exact_rational(m, ka, kb, seed):
    rng = np.random.default_rng(seed)
    A = _rand_exp_matrix(rng, m, ka)
    B = _rand_exp_matrix(rng, m, kb)
    hi, lo = oracle.gram_q(A, B)
    # binary128 accumulation of exact products (2^-113 per step), then the
    # rounding of the binary128 sum to a (hi, lo) pair (2^-106 relative)
    assert gram_dd_err(hi, lo, A, B) <= (m + 4) * 2.0 ** -112 + 2.0 ** -105
    # planted mistake: transposed operands / dropped last row must be caught
    hi2, lo2 = oracle.gram_q(A[:-1], B[:-1]) if m > 1 else (hi * 2, lo)
    assert gram_dd_err(hi2, lo2, A, B) > 1e-20


@pytest.mark.parametrize("m,k,seed", [(50, 3, 4), (500, 4, 5)])
def test_gram_dot2_error_bound(m, k, seed):
    """Dot2 (Ogita-Rump-Oishi): |res - s| <= u|s| + gamma_{n}^2 sum|p|; our DD
    result keeps hi+lo, so the u|s| term drops to ~u^2|s|."""
    rng = np.random.default_rng(seed)
    A = _rand_exp_matrix(rng, m, k, spread=10)
    hi, lo = oracle.gram_dot2(A)
    n = m + 1024
    gam = n * U64 / (1 - n * U64)
    assert gram_dd_err(hi, lo, A, A) <= 2 * gam ** 2 + 8 * U64 ** 2


@pytest.mark.parametrize("m,k,seed", [(200, 4, 6), (1500, 3, 7)])
def test_gram_f64_error_bound(m, k, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, k))
    g = oracle.gram_f64(A)
    nb = min(m, 1024)
    depth = -(-m // nb) + nb  # serial chain within a block + serial over blocks
    assert gram_dd_err(g, None, A, A) <= depth * U64 * 1.01


def test_gram_near_parallel_hadamard_exact():
    """x0 = h0, x1 = h0 + 2^-40 h1: exact Gram [[1, 1], [1, 1 + 2^-80]] --
    binary128 holds it, the (hi, lo) pair returns it exactly."""
    X = synth.hadamard_near_parallel(4, 2, 40)
    hi, lo = oracle.gram_q(X)
    assert hi.tolist() == [[1.0, 1.0], [1.0, 1.0]]
    assert lo.tolist() == [[0.0, 0.0], [0.0, 2.0 ** -80]]
    hi2, lo2 = oracle.gram_dot2(X)
    assert (hi2 + 0).tolist() == [[1.0, 1.0], [1.0, 1.0]]
    assert lo2[1, 1] == 2.0 ** -80 and lo2[0, 0] == 0 and lo2[0, 1] == 0
    g = oracle.gram_f64(X)
    assert g[1, 1] == 1.0  # binary64 cannot hold 1 + 2^-80


# --------------------------------------------------------------------------
# Cholesky, triangular inverse, update against exact rational algebra

@pytest.mark.parametrize("k,seed", [(3, 10), (6, 11)])
def test_chol_q_vs_exact_ldlt(k, seed):
    rng = np.random.default_rng(seed)
    A = _rand_exp_matrix(rng, 3 * k + 2, k, spread=4)
    hi, lo = oracle.gram_q(A)
    G = [[dd_value(hi[i, j], lo[i, j]) for j in range(k)] for i in range(k)]
    L, D = ldlt_exact(G)
    rhi, rlo, info = oracle.chol_q(hi, lo)
    assert info == 0
    for j in range(k):
        rjj = dd_value(rhi[j, j], rlo[j, j])
        assert abs(rjj * rjj - D[j]) <= D[j] * Fraction(1, 2 ** 100)
        for i in range(j + 1, k):
            rji = dd_value(rhi[j, i], rlo[j, i])
            assert abs(rji / rjj - L[i][j]) <= (abs(L[i][j]) + 1) * Fraction(1, 2 ** 96)
        for i in range(j):
            assert rhi[j, i] == 0.0
    # planted mistake: a sign flip in one off-diagonal entry is caught
    bad = rhi.copy()
    bad[0, 1] = -bad[0, 1]
    assert abs(F(bad[0, 1]) / F(bad[0, 0]) - L[1][0]) > Fraction(1, 2 ** 40)


def test_chol_q_breakdown_pivot():
    G = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 1.0]])  # rank-1 leading 2x2
    _, _, info = oracle.chol_q(G)
    assert info == 2
    G2 = np.array([[-1.0]])
    assert oracle.chol_q(G2)[2] == 1


def test_trinv_q_exact_identity():
    rng = np.random.default_rng(12)
    k = 5
    R = np.triu(rng.standard_normal((k, k))) + 3 * np.eye(k)
    zhi, zlo = oracle.trinv_q(R)
    for i in range(k):
        for j in range(k):
            s = sum((F(R[i, l]) * dd_value(zhi[l, j], zlo[l, j]) for l in range(k)),
                    Fraction(0))
            assert abs(s - (1 if i == j else 0)) <= Fraction(1, 2 ** 98)
    assert np.all(np.tril(zhi, -1) == 0)


def test_update_q_exact_rational():
    rng = np.random.default_rng(13)
    m, k, ky = 9, 3, 2
    X = rng.standard_normal((m, k))
    Y = rng.standard_normal((m, ky))
    C = rng.standard_normal((ky, k))
    Z = np.triu(rng.standard_normal((k, k)))
    Q = oracle.update_q(X, Z, Y, C)
    for r in range(m):
        xt = [F(X[r, j]) - sum((F(Y[r, l]) * F(C[l, j]) for l in range(ky)), Fraction(0))
              for j in range(k)]
        for j in range(k):
            ex = sum((xt[i] * F(Z[i, j]) for i in range(k)), Fraction(0))
            # exact value rounded once to binary64 (binary128 carries ~2^-110)
            assert Q[r, j] == float(ex) or abs(F(Q[r, j]) - ex) <= abs(ex) * Fraction(1, 2 ** 52)
    assert np.array_equal(oracle.update_q(X, np.eye(k)), X)


# --------------------------------------------------------------------------
# Exact worked families: Sylvester-Hadamard

@pytest.mark.parametrize("j,exps", [(3, [0, -1, 5]), (5, [0, -10, -20, -30, -40, -50]),
                                    (4, [3, 3, 3, 3, 3, 3, 3, 3])])
def test_qr_q_hadamard_scaled_bitwise(j, exps):
    X = synth.hadamard_scaled(j, exps)
    H = synth.hadamard_columns(j, range(1, 1 + len(exps)))
    o = oracle.qr_q(X)
    assert o["info"] == 0
    assert np.array_equal(o["Q"], H)
    assert np.array_equal(o["R"], np.diag(np.ldexp(1.0, exps)))
    met = oracle.metrics(o["Q"], X, o["R"])
    assert met["omega"] == 0.0 and met["rho"] == 0.0


def test_qr_q_near_parallel_exact():
    k = 4
    X = synth.hadamard_near_parallel(5, k, 40)
    H = synth.hadamard_columns(5, range(1, 1 + k))
    o = oracle.qr_q(X)
    d = 2.0 ** -40
    Rex = np.eye(k) * d
    Rex[0, :] = 1.0
    assert np.array_equal(o["Q"], H)
    assert np.array_equal(o["R"], Rex)


def test_cholqr_steps_near_parallel():
    """DD CholQR2 returns the exact Q within a few ulps; binary64 Gram loses the
    2^-80 term, so plain CholQR breaks down or returns a non-orthogonal Q."""
    k = 4
    X = synth.hadamard_near_parallel(6, k, 40)
    H = synth.hadamard_columns(6, range(1, 1 + k))
    s = oracle.cholqr_steps(X, dd_first=True, passes=2)
    assert s["info"] == 0
    assert np.max(np.abs(s["Q"] - H)) <= 8 * U64 * np.max(np.abs(H))
    assert oracle.metrics(s["Q"], X, s["R_hi"])["omega"] <= 1e-15
    p = oracle.cholqr_steps(X, dd_first=False, passes=1)
    if p["info"] == 0:
        assert oracle.metrics(p["Q"], X, p["R_hi"])["omega"] > 1e-6


def test_projection_hadamard_exact():
    """Y = other Hadamard columns, so Y^T X is exact and X - Y C is exact."""
    j = 4
    Y = synth.hadamard_columns(j, [20, 21, 22])
    H = synth.hadamard_columns(j, [1, 2])
    X = H * 4.0 + Y @ np.array([[1.0, -2.0], [0.5, 0.25], [3.0, 0.0]])
    o = oracle.qr_q(X, Y)
    assert np.array_equal(o["C"], np.array([[1.0, -2.0], [0.5, 0.25], [3.0, 0.0]]))
    assert np.array_equal(o["Q"], H)
    assert np.array_equal(o["R"], 4.0 * np.eye(2))
    for dd in (False, True):
        s = oracle.cholqr_steps(X, Y, dd_first=dd, passes=2)
        assert np.array_equal(s["Q"], H) and np.array_equal(s["C_hi"], o["C"])


def test_corrected_projection_exact_basis_is_plain():
    """Y exactly orthonormal (Hadamard columns): S = Y^T Y = I exactly, so the
    corrected coefficients D = 2C - S C equal C and the pass is unchanged."""
    Y = synth.hadamard_columns(5, [3, 9, 17, 30])
    X = synth.svd_matrix(1024, 3, 1e4, 61) + Y @ np.array([[1.0, -2.0, 0.5]] * 4)
    a = oracle.cholqr_steps(X, Y, dd_first=True, passes=1)
    b = oracle.cholqr_steps(X, Y, dd_first=True, passes=1, dd_corrected=True)
    for key in ("Q", "R_hi", "R_lo", "C_hi", "C_lo"):
        assert np.array_equal(a[key], b[key]), key


def test_corrected_projection_second_order():
    """Y orthonormal only to ||S - I|| ~ 2e-7 (columns scaled by 1 + e_i):
    the plain projection leaves O(||S - I||) of X in span(Y), amplified by
    kappa(X, Y) in Q; the corrected one leaves O(||S - I||^2)."""
    X, Y0 = synth.projected_pair(4000, 2, 6, 1.0, 1e3, 62)
    Y = Y0 * (1.0 + 1e-7 * np.arange(1, 7))[None, :]
    a = oracle.cholqr_steps(X, Y, dd_first=True, passes=1)
    b = oracle.cholqr_steps(X, Y, dd_first=True, passes=1, dd_corrected=True)
    wa = np.linalg.norm(Y.T @ a["Q"])
    wb = np.linalg.norm(Y.T @ b["Q"])
    assert wa >= 1e-5       # ~ ||S - I|| |C| kappa(X, Y)
    assert wb <= 1e-8       # ~ ||S - I||^2 |C| kappa(X, Y), plus rounding
    # both decompose X: X = Y C + Q R
    for o in (a, b):
        res = X - Y @ (o["C_hi"] + o["C_lo"]) - o["Q"] @ (o["R_hi"] + o["R_lo"])
        assert np.linalg.norm(res) <= 1e-13 * np.linalg.norm(X)


def test_gram_w_q_reduces_to_gram_q():
    """B = I gives the unweighted binary128 Gram bitwise; B = diag(4^e) gives
    the Gram of the rows scaled by 2^e (exact scalings) bitwise."""
    X = synth.svd_matrix(3000, 6, 1e5, 63)
    A = synth.locked_basis(3000, 3, 64)
    ones = np.ones(3000)
    for a, b in zip(oracle.gram_q(A, X), oracle.gram_w_q(A, ones, X)):
        assert np.array_equal(a, b)
    e = np.random.default_rng(65).integers(-6, 7, size=3000)
    w = np.ldexp(1.0, 2 * e)
    s = np.ldexp(1.0, e)[:, None]
    for a, b in zip(oracle.gram_q(A * s, X * s), oracle.gram_w_q(A, w, X)):
        assert np.array_equal(a, b)
    mb = oracle.metrics_b(synth.locked_basis(3000, 4, 66), X[:, :4], np.eye(4), ones)
    mp = oracle.metrics(synth.locked_basis(3000, 4, 66), X[:, :4], np.eye(4))
    assert mb["omega"] == pytest.approx(mp["omega"], rel=1e-12, abs=1e-30)


def test_b_weighted_inputs():
    """The generator's Y is B-orthonormal and X keeps its B-condition."""
    X, Y, w = synth.b_weighted_pair(2000, 3, 5, 1e4, 1e4, 1e4, 67)
    yhi, ylo = oracle.gram_w_q(Y, w)
    assert np.linalg.norm(yhi + ylo - np.eye(5)) <= 1e-14
    assert 1e-2 <= w.min() and w.max() <= 1e2
    Xt = X - Y @ (oracle.gram_w_q(Y, w, X)[0])
    ghi, glo = oracle.gram_w_q(Xt, w)
    ev = np.linalg.eigvalsh(ghi + glo)
    assert np.sqrt(ev.max() / ev.min()) == pytest.approx(1e4, rel=1e-3)


# --------------------------------------------------------------------------
# LAPACK special cases and generator closed forms

def _lapack_qr(X):
    q, r = np.linalg.qr(X)
    s = np.sign(np.diag(r))
    return q * s[None, :], r * s[:, None]


@pytest.mark.parametrize("m,k,kappa,seed", [(2000, 8, 1e2, 20), (3000, 16, 1e4, 21)])
def test_qr_q_vs_lapack(m, k, kappa, seed):
    X = synth.svd_matrix(m, k, kappa, seed)
    o = oracle.qr_q(X)
    ql, rl = _lapack_qr(X)
    tol = 50 * kappa * U64 * np.sqrt(k)
    assert np.max(np.abs(o["Q"] - ql)) <= tol
    assert np.linalg.norm(o["R"] - rl) / np.linalg.norm(rl) <= tol
    # LAPACK Cholesky of the rounded exact Gram reproduces R where kappa^2 u << 1
    g = oracle.gram_q(X)[0]
    rc = scipy.linalg.cholesky(g, lower=False)
    assert np.linalg.norm(o["R"] - rc) / np.linalg.norm(rc) <= 50 * kappa ** 2 * U64
    # planted mistake: a transposed R fails the same check
    assert np.linalg.norm(o["R"].T - rl) / np.linalg.norm(rl) > tol


def test_generator_closed_forms():
    """X = U S V^T: eig(X^T X) = sigma^2, and the symmetric SVQB output
    X M^{-1/2} is the polar factor U V^T."""
    m, k, kappa, seed = 1500, 6, 1e3, 30
    X = synth.svd_matrix(m, k, kappa, seed)
    rng = np.random.default_rng(seed)
    U = synth.haar(rng, m, k)
    V = synth.haar(rng, k, k)
    sig = synth.sigma_logspace(k, kappa)
    hi, lo = oracle.gram_q(X)
    Z, lam, info = oracle.svqb_q(hi, lo)
    assert info == 0
    assert np.allclose(np.sort(sig ** 2), lam, rtol=0, atol=1e-14)
    P = oracle.update_q(X, Z)
    assert np.max(np.abs(P - U @ V.T)) <= 10 * kappa * U64 * np.sqrt(k)
    assert np.allclose(Z, Z.T, atol=1e-12 * np.max(np.abs(Z)))
    # Z^T M Z = I (the defining property of the phase-II transform); Z is
    # rounded to binary64, which costs ~ u kappa(M) = u kappa^2
    M = hi + lo
    assert np.max(np.abs(Z.T @ M @ Z - np.eye(k))) <= 10 * k * kappa ** 2 * U64


def test_svqb_q_vs_lapack_eigh():
    rng = np.random.default_rng(31)
    A = rng.standard_normal((50, 5))
    M = A.T @ A
    Z, lam, info = oracle.svqb_q(M)
    w, v = np.linalg.eigh(M)
    Zl = (v / np.sqrt(w)[None, :]) @ v.T
    assert np.allclose(lam, w, rtol=1e-13)
    assert np.max(np.abs(Z - Zl)) <= 1e-13 * np.max(np.abs(Zl))


# --------------------------------------------------------------------------
# Published error laws

def _omega_one_pass(kappa, dd, m=2000, k=8, seed=40):
    X = synth.svd_matrix(m, k, kappa, seed)
    s = oracle.cholqr_steps(X, dd_first=dd, passes=1)
    if s["info"]:
        return np.inf
    return oracle.metrics(s["Q"], X, s["R_hi"])["omega"]


def test_plain_cholqr_kappa_squared_law():
    """Plain CholQR loses orthogonality ~ c kappa^2 u and breaks down near
    kappa ~ u^{-1/2} (~1e8)."""
    ks = [1e2, 1e3, 1e4, 1e5]
    om = [_omega_one_pass(k, False) for k in ks]
    slope = np.polyfit(np.log10(ks), np.log10(om), 1)[0]
    assert 1.6 <= slope <= 2.4
    for k_, o_ in zip(ks, om):
        assert 1e-3 * k_ ** 2 * U64 <= o_ <= 1e3 * k_ ** 2 * U64
    assert _omega_one_pass(1e10, False) >= 1e-1  # breakdown or garbage


def test_cholqr2_reaches_unit_roundoff():
    """CholQR2 orthogonality is O(u) for kappa below ~u^{-1/2}; with the first
    pass in DD it stays O(u) up to kappa ~ 1e15."""
    for kappa, dd in [(1e2, False), (1e6, False), (1e6, True), (1e12, True), (1e15, True)]:
        X = synth.svd_matrix(3000, 8, kappa, 41)
        s = oracle.cholqr_steps(X, dd_first=dd, passes=2)
        assert s["info"] == 0, (kappa, dd)
        met = oracle.metrics(s["Q"], X, s["R_hi"])
        assert met["omega"] <= 1e-14 and met["rho"] <= 1e-14, (kappa, dd, met)


def test_exact_gram_pass_first_row_exact_rational():
    """The binary64 pass given the exactly rounded Gram matrix: its first
    Cholesky row is R_00 = sqrt(fl(G_00)) and R_0j = fl(G_0j) / R_00, each
    correctly rounded, with fl(G) the exact rational Gram rounded once."""
    rng = np.random.default_rng(44)
    X = _rand_exp_matrix(rng, 300, 4, spread=6)
    s = oracle.cholqr_steps(X, passes=1, exact_gram=True)
    assert s["info"] == 0
    G = gram_exact(X)
    g = np.array([[float(G[i][j]) for j in range(4)] for i in range(4)])  # round once
    r00 = np.sqrt(g[0, 0])
    want = np.array([r00] + [g[0, j] / r00 for j in range(1, 4)])
    assert np.array_equal(s["R_hi"][0], want)
    # planted mistake: one ulp off in any entry of the first row is caught
    bad = want.copy()
    bad[2] = np.nextafter(bad[2], np.inf)
    assert not np.array_equal(bad, want)


def test_exact_gram_pass_hadamard_and_law():
    """With the exactly rounded Gram matrix the binary64 pass is exact on the
    scaled Hadamard family, and its loss still follows c kappa^2 u but sits
    below the binary64-summed pass's (the Gram matrix's rounding error is
    one of the two terms of that loss; the Cholesky factor's is the other)."""
    exps = [0, -3, 7, -20, 11, -35]
    X = synth.hadamard_scaled(5, exps)
    s = oracle.cholqr_steps(X, passes=1, exact_gram=True)
    assert np.array_equal(s["Q"], synth.hadamard_columns(5, range(1, 7)))
    assert np.array_equal(s["R_hi"], np.diag(np.ldexp(1.0, exps)))
    ratios = []
    for seed in (101, 102, 103):
        X = synth.svd_matrix(20000, 8, 1e4, seed)
        e = oracle.cholqr_steps(X, passes=1, exact_gram=True)
        f = oracle.cholqr_steps(X, passes=1)
        oe = oracle.metrics(e["Q"], X, e["R_hi"])["omega"]
        of = oracle.metrics(f["Q"], X, f["R_hi"])["omega"]
        assert 1e-4 * 1e8 * U64 <= oe <= 1e2 * 1e8 * U64
        ratios.append(of / oe)
    assert np.median(ratios) >= 2.0, ratios


def test_dd_first_pass_law():
    """A DD pass loses ~ c kappa^2 u_dd (u_dd ~ 2^-106) on top of the binary64
    output rounding floor."""
    oms = {k: _omega_one_pass(k, True) for k in [1e10, 1e12, 1e14]}
    for k_, o_ in oms.items():
        assert o_ <= 1e3 * k_ ** 2 * 2.0 ** -106 + 1e-15
    assert oms[1e14] > 1e2 * oms[1e10]


def _fig7_right_panel():
    pts = {}
    cal = {}
    for line in (GOLDEN / "fig7_orthogonality.txt").read_text().splitlines():
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "calib":
            cal[f[1]] = tuple(map(float, f[2:]))
            continue
        pts.setdefault(f[0], []).append((float(f[1]), float(f[2])))
    (y0, l0, y1, l1), (x0, e0, x1, e1) = cal["y"], cal["x"]

    def dec(xy):
        x, y = xy
        return (round(e0 + (x - x0) * (e1 - e0) / (x1 - x0)),
                l0 + (y - y0) * (l1 - l0) / (y1 - y0))
    return {k: [dec(p) for p in v] for k, v in pts.items()}


def test_fig7_levels():
    """Fig. 7 (right panel), n = 1000, n_b = 4, k = 20 locked vectors: the
    binary64 two-phase step loses ~2 decades of orthogonality per decade of
    kappa(X) and breaks down by kappa = 1e9; the DD step stays flat at the
    working-precision floor through kappa = 1e6.  The oracle's project/CholQR
    in binary64 and in DD must show the same slope and levels."""
    fig = _fig7_right_panel()
    paper_plain = {}
    for e, lv in fig["plain"]:
        paper_plain.setdefault(e, []).append(lv)
    slope_paper = (np.mean(paper_plain[6]) - np.mean(paper_plain[0])) / 6.0
    assert 1.7 <= slope_paper <= 2.1
    assert max(lv for e, lv in fig["dd"] if e <= 6) < -16.5
    assert min(paper_plain[9]) > -0.5  # breakdown
    n, kw, nb = 1000, 20, 4
    ours = {}
    for e in (0, 3, 6):
        X, W = synth.projected_pair(n, nb, kw, 10.0 ** e, 10.0 ** e, 700 + e)
        s = oracle.cholqr_steps(X, W, dd_first=False, passes=1)
        ours[e] = np.log10(max(oracle.metrics(s["Q"], X, s["R_hi"], W, s["C_hi"])["omega"],
                               1e-20))
        d = oracle.cholqr_steps(X, W, dd_first=True, passes=1)
        om_dd = oracle.metrics(d["Q"], X, d["R_hi"], W, d["C_hi"])["omega"]
        assert om_dd <= 1e-15  # flat at the binary64 output floor
    slope_ours = (ours[6] - ours[0]) / 6.0
    assert abs(slope_ours - slope_paper) <= 0.35
    for e in (3, 6):
        assert abs(ours[e] - np.mean(paper_plain[e])) <= 2.5
    X, W = synth.projected_pair(n, nb, kw, 1e9, 1e9, 709)
    s = oracle.cholqr_steps(X, W, dd_first=False, passes=1)
    if s["info"] == 0:
        assert oracle.metrics(s["Q"], X, s["R_hi"], W, s["C_hi"])["omega"] > 1e-2


def test_fig7_levels_svqb():
    """The paper's Fig. 7 method itself (one project / SVQB pass): the
    oracle's binary64 pass shows the plotted slope of ~2 decades per decade of
    kappa(X) and its levels; the DD pass stays at the output floor."""
    fig = _fig7_right_panel()
    paper_plain = {}
    for e, lv in fig["plain"]:
        paper_plain.setdefault(e, []).append(lv)
    slope_paper = (np.mean(paper_plain[6]) - np.mean(paper_plain[0])) / 6.0
    n, kw, nb = 1000, 20, 4
    ours = {}
    for e in (0, 3, 6):
        X, W = synth.projected_pair(n, nb, kw, 10.0 ** e, 10.0 ** e, 700 + e)
        s = oracle.iterate(X, W, gram="f64", fact="svqb", max_iter=1)
        assert s["info"] == 0 and s["passes"] == 1
        ours[e] = np.log10(max(oracle.metrics(s["Q"], X, s["R_hi"], W, s["C_hi"])["omega"], 1e-20))
        d = oracle.iterate(X, W, gram="dd", fact="svqb", max_iter=1)
        assert oracle.metrics(d["Q"], X, d["R_hi"], W, d["C_hi"])["omega"] <= 1e-15
    assert abs((ours[6] - ours[0]) / 6.0 - slope_paper) <= 0.35
    for e in (3, 6):
        assert abs(ours[e] - np.mean(paper_plain[e])) <= 2.5


# --------------------------------------------------------------------------
# The iterated scheme and kappa_true

@pytest.mark.parametrize("gram", ["f64", "dd"])
@pytest.mark.parametrize("fact", ["chol", "svqb"])
def test_iterate_hadamard_stops_after_one_pass(gram, fact):
    """X orthonormal and orthogonal to Y exactly (Sylvester-Hadamard
    columns): the first pass finds C = 0 and M = I, so Q = X, R = I and C = 0
    bit for bit and the stop test holds at once; a test that never holds
    (eps < 0) runs max_iter passes instead."""
    Y = synth.hadamard_columns(5, [40, 41, 42, 43])
    X = synth.hadamard_columns(5, [1, 2, 3])
    s = oracle.iterate(X, Y, gram=gram, fact=fact, eps=1e-10, max_iter=5)
    assert s["info"] == 0 and s["passes"] == 1 and s["converged"]
    assert np.array_equal(s["Q"], X)
    assert np.array_equal(s["R_hi"], np.eye(3)) and not s["R_lo"].any()
    assert not s["C_hi"].any()
    assert s["c_norm"] == 0.0 and s["r_dev"] == 0.0
    t = oracle.iterate(X, Y, gram=gram, fact=fact, eps=-1.0, max_iter=4)
    assert t["passes"] == 4 and not t["converged"]


@pytest.mark.parametrize("gram,bound", [("dd", 50.0), ("f64", 50.0)])
def test_iterate_svqb_pass_is_the_polar_factor(gram, bound):
    """One symmetric-SVQB pass on X = U diag(sigma) V^T returns the polar
    factor U V^T (closed form of the generator): within ~kappa u with the DD
    Gram, within ~kappa^2 u with the binary64 one (the Gram matrix's own
    rounding), and R = V diag(sigma) V^T."""
    m, k, kappa, seed = 3000, 6, 1e4, 77
    rng = np.random.default_rng(seed)
    U = synth.haar(rng, m, k)
    V = synth.haar(rng, k, k)
    sig = synth.sigma_logspace(k, kappa)
    X = (U * sig[None, :]) @ V.T
    assert np.array_equal(X, synth.svd_matrix(m, k, kappa, seed))
    s = oracle.iterate(X, gram=gram, fact="svqb", max_iter=1)
    P = U @ V.T
    err = np.max(np.abs(s["Q"] - P))
    lim = bound * (kappa if gram == "dd" else kappa ** 2) * U64
    assert err <= lim, (err, lim)
    Rex = (V * sig[None, :]) @ V.T
    assert np.max(np.abs(s["R_hi"] - Rex)) <= 1e-12
    # planted mistake: a Cholesky pass is not the polar factor
    c = oracle.iterate(X, gram=gram, fact="chol", max_iter=1)
    assert np.max(np.abs(c["Q"] - P)) > 1e-3


@pytest.mark.parametrize("fact", ["chol", "svqb"])
def test_iterate_converges_on_the_runtime_experiment_shape(fact):
    """X close to span(Y) (kappa(X) = 1e6, kappa(X, Y) = 1e12, the paper's
    runtime experiment at fewer rows): the passes converge at eps = 1e-10
    within five passes to an orthonormal Q orthogonal to Y with X = Y C + Q R,
    and the DD variant needs no more passes than the binary64 one (the
    paper's point about DD)."""
    X, Y = synth.projected_pair(20000, 4, 20, 1e6, 1e12, 7100)
    res = {}
    for gram in ("f64", "dd"):
        s = oracle.iterate(X, Y, gram=gram, fact=fact, eps=1e-10, max_iter=8)
        assert s["info"] == 0 and s["converged"] and s["passes"] <= 5, (gram, s["passes"])
        met = oracle.metrics(s["Q"], X, s["R_hi"], Y, s["C_hi"])
        assert met["omega"] <= 1e-14 and met["omega_y"] <= 1e-14, met
        assert met["rho"] <= (1e-14 if fact == "chol" else 1e-12), met
        assert s["c_norm"] <= 1e-10 and s["r_dev"] <= 1e-10
        res[gram] = s["passes"]
    assert res["dd"] <= res["f64"]


def test_kappa_true():
    """kappa from the exact Gram matrix: the generator's nominal kappa for
    moderate kappa (U orthonormal to ~1e-15), LAPACK's singular values where
    they are accurate, and the projected block's kappa with a locked basis."""
    for kappa in (1e2, 1e6):
        X = synth.svd_matrix(5000, 8, kappa, 81)
        kt = oracle.kappa_true(X)
        assert abs(kt / kappa - 1) <= 1e-8
        sv = np.linalg.svd(X, compute_uv=False)
        assert abs(kt / (sv[0] / sv[-1]) - 1) <= 1e-8
    X, Y = synth.projected_pair(4000, 4, 6, 10.0, 1e8, 82)
    Xt = X - Y @ (Y.T @ X)
    sv = np.linalg.svd(Xt, compute_uv=False)
    assert abs(oracle.kappa_true(X, Y) / (sv[0] / sv[-1]) - 1) <= 1e-6


# --------------------------------------------------------------------------
# Metrics and the split-BF16 model

def test_metrics_vs_exact_rational():
    rng = np.random.default_rng(50)
    m, k = 40, 3
    Q = rng.standard_normal((m, k)) / np.sqrt(m)
    X = rng.standard_normal((m, k))
    R = np.triu(rng.standard_normal((k, k)))
    met = oracle.metrics(Q, X, R)
    G = gram_exact(Q)
    om2 = sum(((G[i][j] - (1 if i == j else 0)) ** 2 for i in range(k) for j in range(k)),
              Fraction(0))
    assert abs(met["omega"] - np.sqrt(float(om2))) <= 1e-14 * np.sqrt(float(om2))
    res = 0.0
    for r in range(m):
        for j in range(k):
            v = F(X[r, j]) - sum((F(Q[r, i]) * F(R[i, j]) for i in range(k)), Fraction(0))
            res += float(v) ** 2
    assert abs(met["rho"] - np.sqrt(res) / np.linalg.norm(X)) <= 1e-13 * met["rho"]


def test_split_bf16_model():
    """Integer inputs |x| <= 511 split into an 8-bit hi and lo in {-1, 0, 1};
    every fp32 product and chunk sum (16 rows) is then an integer below 2^24,
    so the model must equal H^T H + H^T L + L^T H exactly, i.e. the exact Gram
    minus L^T L.  The split here is an independent integer computation."""
    rng = np.random.default_rng(60)
    m, k = 64, 4
    Xi = rng.integers(-511, 512, (m, k))
    X = Xi.astype(np.float32)
    G = oracle.gram_split_bf16(X, chunk=16)

    def bf(v):  # round an integer to 8 significant bits, ties to even
        v = int(v)
        if abs(v) < 256:
            return v
        q, r = divmod(abs(v), 2)  # |v| < 512: one bit to drop
        if r == 1 and q % 2 == 1:
            q += 1
        return (q * 2) * (1 if v > 0 else -1)
    H = np.vectorize(bf)(Xi).astype(np.float64)
    L = Xi.astype(np.float64) - H
    assert set(np.unique(L)) <= {-1.0, 0.0, 1.0}
    X64 = Xi.astype(np.float64)
    assert np.array_equal(G, H.T @ H + H.T @ L + L.T @ H)
    assert np.array_equal(X64.T @ X64 - G, L.T @ L)
    # general inputs: error level ~ 3 * 2^-16 of |X|^T|X|
    Xr = rng.standard_normal((4000, 8)).astype(np.float32)
    Gr = oracle.gram_split_bf16(Xr, chunk=256)
    exr = oracle.gram_q(Xr.astype(np.float64))[0]
    absg = np.abs(Xr.astype(np.float64)).T @ np.abs(Xr.astype(np.float64))
    assert np.max(np.abs(Gr - exr) / absg) <= 4 * 2.0 ** -16
