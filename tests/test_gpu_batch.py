"""GPU tests of the batched path (many independent blocks per launch).

Every block of a batch must satisfy what the single-block method guarantees
(oracle metrics: rho, omega, omega_Y <= 1e-14 for DD CholQR2 with the
projection repeated, Sec. 4.2), results must not depend on the other blocks
(a breakdown stays in its block), graph replays and in-place runs are
bitwise identical to the eager run, and the autotune table round-trips.
Both drivers are covered: the launch per phase (the default) and the
persistent single launch (persistent=True where every block fits it;
BORTH_LOG reports which driver ran).
"""
import re

import numpy as np
import pytest

import oracle
import synth
from gpu_common import U64, dev, host, lib, note, rel_fro, torch_gpu

pytestmark = pytest.mark.gpu


def _blocks(specs):
    """specs: (m, k, ky, kappa, seed) -> host arrays and device blocks."""
    hostb, devb = [], []
    for (m, k, ky, kappa, seed) in specs:
        X = synth.svd_matrix(m, k, kappa, seed)
        Y = synth.locked_basis(m, ky, seed + 7777) if ky else None
        hostb.append((X, Y))
        d = {"X": dev(X)}
        if ky:
            d["Y"] = dev(Y)
        devb.append(d)
    return hostb, devb


MIXED = [(3001, 8, 16, 1e3, 11), (12007, 32, 16, 1e9, 12), (2500, 64, 16, 1e5, 13),
         (7003, 16, 0, 1e10, 14), (20011, 13, 5, 1e7, 15), (4099, 1, 0, 1.0, 16),
         (9001, 40, 16, 1e8, 17), (15013, 64, 0, 1e6, 18), (5000, 20, 3, 1e4, 19),
         (6007, 3, 16, 1e2, 20)]


# every block fits the persistent launch: 5 <= k <= 64, ky <= 16
PERSIST = [(3001, 8, 16, 1e3, 41), (12007, 32, 16, 1e9, 42), (2500, 64, 16, 1e5, 43),
           (7003, 16, 0, 1e10, 44), (20011, 13, 5, 1e7, 45), (4099, 5, 0, 1e2, 46),
           (9001, 40, 16, 1e8, 47), (15013, 64, 0, 1e6, 48), (5000, 20, 3, 1e4, 49),
           (60007, 24, 16, 1e6, 50)]


def _drivers(capfd):
    """persistent=0/1 of each batched call since the last read (BORTH_LOG)."""
    return [int(x) for x in re.findall(r"borth: batch .*persistent=(\d)", capfd.readouterr().err)]


def _check_vs_oracle(hostb, outs, infos, specs):
    for (X, Y), (Q, R, C), inf, spec in zip(hostb, outs, infos, specs):
        note("block", spec, inf)
        assert inf.status == 0 and inf.passes_run == 2
        met = oracle.metrics(host(Q), X, host(R), Y, host(C) if C is not None else None)
        note("  ", met)
        assert met["rho"] <= 1e-14 and met["omega"] <= 1e-14
        if Y is not None:
            assert met["omega_y"] <= 1e-14
            o1 = oracle.qr_q(X, Y)
            assert np.max(np.abs(host(C) - o1["C"])) <= 1e-13
        Rh = host(R)
        assert np.all(np.tril(Rh, -1) == 0) and np.all(np.diag(Rh) > 0)


def test_batch_persistent_vs_oracle(monkeypatch, capfd):
    """The persistent single launch: DD-Gram CholQR2 with the projection
    repeated on ten blocks of uneven height, width and conditioning."""
    monkeypatch.setenv("BORTH_LOG", "1")
    borth = lib()
    hostb, devb = _blocks(PERSIST)
    outs, infos = borth.batch_orthonormalize(devb, gram="dd", passes=2, persistent=True)
    assert _drivers(capfd) == [1]
    _check_vs_oracle(hostb, outs, infos, PERSIST)


@pytest.mark.parametrize("passes", [1, 2])
def test_batch_persistent_matches_phases(passes, monkeypatch, capfd):
    """Both drivers run the same task bodies on the same workgroup shares:
    one pass (Gram, reduction, factor, update) is bitwise identical; with a
    second pass the fused Gram of the first update is summed over a
    different number of waves per workgroup, so the second factor differs
    in rounding only."""
    monkeypatch.setenv("BORTH_LOG", "1")
    borth = lib()
    torch = torch_gpu()
    hostb, devb = _blocks(PERSIST)
    op, ip = borth.batch_orthonormalize(devb, gram="dd", passes=passes, persistent=True)
    of, inf_ = borth.batch_orthonormalize(devb, gram="dd", passes=passes)
    assert _drivers(capfd) == [1, 0]
    for (Qp, Rp, Cp), (Qf, Rf, Cf), a, b, spec in zip(op, of, ip, inf_, PERSIST):
        assert a.status == b.status == 0 and a.passes_run == b.passes_run == passes
        if passes == 1:
            assert torch.equal(Qp, Qf) and torch.equal(Rp, Rf), spec
            if Cp is not None:
                assert torch.equal(Cp, Cf)
        else:
            kappa = max(spec[3], 1.0)
            assert np.max(np.abs(host(Qp) - host(Qf))) <= 1e-13, spec
            assert rel_fro(host(Rp), host(Rf)) <= 1e3 * kappa * U64, spec


def test_batch_persistent_graph_replay_and_in_place(monkeypatch, capfd):
    """The persistent launch takes its tasks in a different order on every
    run, but each task's arithmetic is fixed: replays of the captured graph
    and in-place runs give the eager run's bits."""
    monkeypatch.setenv("BORTH_LOG", "1")
    borth = lib()
    torch = torch_gpu()
    hostb, devb = _blocks(PERSIST[:6])
    ref, _ = borth.batch_orthonormalize(devb, gram="dd", passes=2, persistent=True)
    ref = [(Q.clone(), R.clone()) for (Q, R, _) in ref]
    for d, (Q, R) in zip(devb, ref):
        d["Q"] = torch.empty_like(Q)
        d["R"] = torch.empty_like(R)
    for rep in range(3):
        for d in devb:
            d["Q"].fill_(0.0)
        outs, infos = borth.batch_orthonormalize(devb, gram="dd", passes=2, graph=True,
                                                 persistent=True)
        torch.cuda.synchronize()
        junk = torch.randn(512, 512, device="cuda", dtype=torch.float64).sum()  # eager work
        torch.cuda.synchronize()
        del junk
        for (Q, R, _), (Qr, Rr), inf in zip(outs, ref, infos):
            assert inf.status == 0
            assert torch.equal(Q, Qr) and torch.equal(R, Rr), rep
    for d in devb:
        d["X"] = d["X"].clone()
        d["Q"] = d["X"]
    outs, infos = borth.batch_orthonormalize(devb, gram="dd", passes=2, persistent=True)
    for (Q, R, _), (Qr, Rr), inf in zip(outs, ref, infos):
        assert inf.status == 0
        assert torch.equal(Q, Qr) and torch.equal(R, Rr)
    assert set(_drivers(capfd)) == {1}


def test_batch_persistent_breakdown_and_fallback(monkeypatch, capfd):
    """A breakdown stays in its block in the persistent launch too; a batch
    that some block does not fit (k = 3) runs per phase even when the
    persistent launch is asked for."""
    monkeypatch.setenv("BORTH_LOG", "1")
    borth = lib()
    Xbad = synth.hadamard_columns(6, [1, 2, 3, 4, 2, 5])
    good = [synth.svd_matrix(5000, 8, 1e6, 31), synth.svd_matrix(7000, 24, 1e4, 32)]
    devb = [{"X": dev(good[0])}, {"X": dev(Xbad)}, {"X": dev(good[1])}]
    outs, infos = borth.batch_orthonormalize(devb, gram="dd", passes=2, check=False, persistent=True)
    assert _drivers(capfd) == [1]
    assert infos[1].status == 4 and infos[1].failed_pass == 1 and infos[1].failed_pivot == 5
    for i in (0, 2):
        assert infos[i].status == 0
        X = good[0] if i == 0 else good[1]
        met = oracle.metrics(host(outs[i][0]), X, host(outs[i][1]))
        assert met["rho"] <= 1e-14 and met["omega"] <= 1e-14
    narrow = [{"X": dev(synth.svd_matrix(4000, 3, 1e2, 33))}, {"X": dev(good[1])}]
    _, infos = borth.batch_orthonormalize(narrow, gram="dd", passes=2, persistent=True)
    assert _drivers(capfd) == [0] and all(i.status == 0 for i in infos)


def test_batch_dd_cholqr2_vs_oracle():
    """DD-Gram CholQR2 with the projection repeated (P,C,P,C) on ten blocks
    of uneven height, width and conditioning (kappa up to 1e10)."""
    borth = lib()
    hostb, devb = _blocks(MIXED)
    outs, infos = borth.batch_orthonormalize(devb, gram="dd", passes=2)
    for (X, Y), (Q, R, C), inf, spec in zip(hostb, outs, infos, MIXED):
        note("block", spec, inf)
        assert inf.status == 0 and inf.passes_run == 2
        met = oracle.metrics(host(Q), X, host(R), Y, host(C) if C is not None else None)
        note("  ", met)
        assert met["rho"] <= 1e-14 and met["omega"] <= 1e-14
        if Y is not None:
            assert met["omega_y"] <= 1e-14
            o1 = oracle.qr_q(X, Y)
            assert np.max(np.abs(host(C) - o1["C"])) <= 1e-13
        Rh = host(R)
        assert np.all(np.tril(Rh, -1) == 0) and np.all(np.diag(Rh) > 0)


def test_batch_matches_single_block_path():
    """The batched sweeps split each block over a different number of
    workgroups than the single-block call, so results agree to rounding:
    both R factors within 1e3 kappa u of each other, both Q orthonormal."""
    borth = lib()
    specs = MIXED[:5]
    hostb, devb = _blocks(specs)
    outs, _ = borth.batch_orthonormalize(devb, gram="dd", passes=2)
    for (X, Y), d, (Qb, Rb, Cb), spec in zip(hostb, devb, outs, specs):
        Qs, Rs, Cs, info = borth.orthonormalize(d["X"], d.get("Y"), gram="dd", passes=2)
        assert info.status == 0
        kappa = max(spec[3], 1.0)
        assert rel_fro(host(Rb), host(Rs)) <= 1e3 * kappa * U64
        assert rel_fro(host(Qb), host(Qs)) <= 1e3 * kappa * U64


def test_batch_graph_replay_and_in_place():
    borth = lib()
    torch = torch_gpu()
    specs = MIXED[:6]
    hostb, devb = _blocks(specs)
    ref, _ = borth.batch_orthonormalize(devb, gram="dd", passes=2)
    ref = [(Q.clone(), R.clone()) for (Q, R, _) in ref]
    # graph: captured once, replayed; outputs preallocated
    for d, (Q, R) in zip(devb, ref):
        d["Q"] = torch.empty_like(Q)
        d["R"] = torch.empty_like(R)
    for rep in range(3):
        for d in devb:
            d["Q"].fill_(0.0)
        outs, infos = borth.batch_orthonormalize(devb, gram="dd", passes=2, graph=True)
        torch.cuda.synchronize()
        junk = torch.randn(512, 512, device="cuda", dtype=torch.float64).sum()  # eager work
        torch.cuda.synchronize()
        del junk
        for (Q, R, _), (Qr, Rr), inf in zip(outs, ref, infos):
            assert inf.status == 0
            assert torch.equal(Q, Qr) and torch.equal(R, Rr), rep
    # in place: Q = X
    for d in devb:
        d["X"] = d["X"].clone()
        d["Q"] = d["X"]
    outs, infos = borth.batch_orthonormalize(devb, gram="dd", passes=2)
    for (Q, R, _), (Qr, Rr), inf in zip(outs, ref, infos):
        assert inf.status == 0
        assert torch.equal(Q, Qr) and torch.equal(R, Rr)


def test_batch_breakdown_stays_in_its_block():
    """A rank-deficient block (exact Hadamard duplicate column: pivot 5 is 0
    in every precision) reports its own breakdown; its neighbours finish."""
    borth = lib()
    Xbad = synth.hadamard_columns(6, [1, 2, 3, 4, 2, 5])
    good = [synth.svd_matrix(5000, 8, 1e6, 31), synth.svd_matrix(7000, 24, 1e4, 32)]
    devb = [{"X": dev(good[0])}, {"X": dev(Xbad)}, {"X": dev(good[1])}]
    for gram in ("f64", "dd"):
        outs, infos = borth.batch_orthonormalize(devb, gram=gram, passes=2, check=False)
        assert infos[1].status == 4 and infos[1].failed_pass == 1 and infos[1].failed_pivot == 5
        for i in (0, 2):
            assert infos[i].status == 0
            X = good[0] if i == 0 else good[1]
            met = oracle.metrics(host(outs[i][0]), X, host(outs[i][1]))
            assert met["rho"] <= 1e-14 and met["omega"] <= 1e-14


@pytest.mark.parametrize("gram,fact,passes,project_once", [
    ("f64", "chol", 2, False), ("f64", "chol", 1, False), ("dd", "chol", 3, False),
    ("dd", "chol", 2, True), ("f64", "svqb", 2, False), ("dd", "svqb", 2, False)])
def test_batch_options(gram, fact, passes, project_once):
    borth = lib()
    specs = [(4001, 8, 16, 1e3, 41), (9001, 32, 0, 1e5, 42), (3003, 17, 16, 1e4, 43),
             (6001, 64, 16, 1e2, 44)]
    hostb, devb = _blocks(specs)
    outs, infos = borth.batch_orthonormalize(devb, gram=gram, fact=fact, passes=passes,
                                             project_once=project_once)
    for (X, Y), (Q, R, C), inf, spec in zip(hostb, outs, infos, specs):
        assert inf.status == 0 and inf.passes_run == passes
        met = oracle.metrics(host(Q), X, host(R), Y, host(C) if C is not None else None)
        note(gram, fact, passes, project_once, spec, met)
        kappa, k = spec[3], spec[1]
        if fact == "svqb" and gram == "f64":
            # binary64 SVQB: the dense symmetric Z is applied as a product, so
            # the residual carries k kappa u (CholQR's triangular structure
            # keeps its residual O(u)), and omega is the orthogonality level
            # of the Jacobi eigenvectors, O(k u).  The single-block path lands
            # at the same levels on the same input.
            Qs, Rs, Cs, _ = borth.orthonormalize(devb[specs.index(spec)]["X"],
                                                 devb[specs.index(spec)].get("Y"),
                                                 gram=gram, fact=fact, passes=passes)
            ms = oracle.metrics(host(Qs), X, host(Rs), Y, host(Cs) if Cs is not None else None)
            note("  single block:", ms)
            assert met["rho"] <= max(1e-14, k * kappa * U64)
            assert met["rho"] <= 4 * ms["rho"] + 1e-15
            assert met["omega"] <= 20 * k * U64
            assert met["omega"] <= 4 * ms["omega"] + 1e-15
            continue
        if fact == "svqb":
            # DD SVQB in the first pass, binary64 SVQB in the second: the
            # batched update applies the dense Z in binary64, so the residual
            # carries k kappa u, and the last pass's Jacobi gives O(k u)
            assert met["rho"] <= max(1e-14, k * kappa * U64)
            assert met["omega"] <= 20 * k * U64
            if Y is not None:
                assert met["omega_y"] <= 1e-14
            continue
        assert met["rho"] <= 1e-14
        if passes == 1:
            # one plain pass: omega ~ c kappa^2 u (binary64 Gram)
            assert met["omega"] <= 10 * spec[1] * kappa ** 2 * U64
        else:
            assert met["omega"] <= 1e-14
        if Y is not None and not project_once and passes >= 2:
            assert met["omega_y"] <= 1e-14


def test_batch_unaligned_rows_in_a_class():
    """A block whose rows are not 16-byte aligned (odd leading dimension)
    takes its whole width class off the direct-transfer update path; the
    aligned blocks of the other classes keep it.  Every block is checked
    against the oracle."""
    borth = lib()
    torch = torch_gpu()
    specs = [(6001, 32, 16, 1e6, 61), (4003, 30, 16, 1e8, 62), (5003, 64, 16, 1e5, 63),
             (3001, 50, 16, 1e7, 64), (7001, 64, 0, 1e6, 65), (2999, 32, 0, 1e4, 66)]
    hostb, devb = _blocks(specs)
    for i in (1, 3):  # X as a view with leading dimension k + 1 (odd)
        m, k = specs[i][0], specs[i][1]
        W = torch.full((m, k + 1), float("nan"), dtype=torch.float64, device="cuda")
        W[:, :k] = devb[i]["X"]
        devb[i]["X"] = W[:, :k]
    outs, infos = borth.batch_orthonormalize(devb, gram="dd", passes=2)
    _check_vs_oracle(hostb, outs, infos, specs)


def test_batch_c5_shape_reduced():
    """The batched workload's recipe (rows uniform, widths {8,16,32,64},
    kappa log-uniform in [1e3, 1e10], a 16-column locked basis per block) at
    reduced heights: 24 blocks, per-block omega / rho / omega_Y <= 1e-14."""
    borth = lib()
    table = synth.batch_table(24, seed=5000, m_lo=10_000, m_hi=60_000)
    specs = [(t["m"], t["k"], 16, t["kappa"], t["seed"]) for t in table]
    hostb, devb = _blocks(specs)
    outs, infos = borth.batch_orthonormalize(devb, gram="dd", passes=2, graph=True)
    for (X, Y), (Q, R, C), inf, spec in zip(hostb, outs, infos, specs):
        assert inf.status == 0
        met = oracle.metrics(host(Q), X, host(R), Y, host(C))
        assert met["rho"] <= 1e-14 and met["omega"] <= 1e-14 and met["omega_y"] <= 1e-14, (spec, met)


def test_batch_argument_errors():
    borth = lib()
    X = dev(np.zeros((100, 8)))
    with pytest.raises(borth.BorthError):
        borth.batch_orthonormalize([{"X": dev(np.zeros((5, 8)))}])  # m < k
    with pytest.raises(borth.BorthError):
        borth.batch_orthonormalize([{"X": X, "Y": dev(np.zeros((100, 20)))}])  # ky > 16
    with pytest.raises(borth.BorthError):
        borth.batch_orthonormalize([{"X": dev(np.zeros((100, 8), np.float32))}], gram="split")
    with pytest.raises(borth.BorthError):
        borth.batch_orthonormalize([{"X": X}], shift=float("nan"))


def test_autotune_roundtrip(tmp_path):
    borth = lib()
    ctx = borth.Context(0)
    try:
        path = tmp_path / "tune.json"
        ctx.autotune(path, budget_ms=1500)
        txt = path.read_text()
        assert '"op": "gram"' in txt
        # the library's own grid (nwg 0) is a candidate; a tuned grid also
        # gives the batched sweeps their rows per workgroup share
        entries = re.findall(r'"nwg": (\d+), "ms": [\d.]+, "rows": (\d+)', txt)
        m_tune = int(re.search(r'"rows": (\d+), "entries"', txt).group(1))
        assert entries
        for nwg, rows in entries:
            nwg, rows = int(nwg), int(rows)
            assert rows == (-(-m_tune // nwg) if nwg > 0 else 0)
        ctx.autotune_load(path)
        bad = tmp_path / "bad.json"
        bad.write_text("{}\n")
        with pytest.raises(borth.BorthError):
            ctx.autotune_load(bad)
        # the cache names the device it was tuned on; another device's is refused
        assert '"device": "gfx950' in txt
        other = tmp_path / "other.json"
        other.write_text(re.sub(r'"device": "[^"]*"', '"device": "gfx942:sramecc+:xnack-/304cu/hip1"', txt))
        with pytest.raises(borth.BorthError, match="autotune cache made on"):
            ctx.autotune_load(other)
        # the tuned shapes still give correct results (single and batched)
        X = synth.svd_matrix(30000, 32, 1e10, 77)
        Q, R, _, info = borth.orthonormalize(dev(X), gram="dd", ctx=ctx)
        assert info.status == 0
        met = oracle.metrics(host(Q), X, host(R))
        assert met["rho"] <= 1e-14 and met["omega"] <= 1e-14
        # tuned grids may exceed the default workgroup count: the partial
        # buffers must still fit (widest DD Gram: [Y | X] with 16 + 64 columns)
        Xw = synth.svd_matrix(50000, 64, 1e3, 78)
        Yw = synth.locked_basis(50000, 16, 79)
        ghi, glo = borth.gram(dev(Xw), A=dev(Yw), prec="dd", ctx=ctx)
        ehi, elo = oracle.gram_q(np.hstack([Yw, Xw]))
        assert rel_fro(host(ghi) + host(glo), ehi + elo) <= 1e-28
        hostb, devb = _blocks(MIXED[:3])
        outs, infos = borth.batch_orthonormalize(devb, gram="dd", ctx=ctx)
        for (Xh, Yh), (Qb, Rb, Cb), inf in zip(hostb, outs, infos):
            assert inf.status == 0
            met = oracle.metrics(host(Qb), Xh, host(Rb), Yh, host(Cb) if Cb is not None else None)
            assert met["rho"] <= 1e-14 and met["omega"] <= 1e-14
    finally:
        ctx.close()
