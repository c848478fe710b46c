"""Benchmark of the block-orthonormalization hot path on one MI355X.

Default workload: double-double CholQR2 of X (4,000,000 x 32, binary64,
kappa(X) = 1e12, X = U diag(sigma) V^T from seed 302) -- the configuration
the headline metric "block-orth GB/s (% HBM peak) at ||Q^T Q - I|| <= 1e-14:
DD/split vs plain FP64 CholQR" is quoted on.  One step = one full pass of the
path on device-resident input: DD Gram sweep, DD k x k Cholesky, update sweep
with the fused binary64 Gram of Q_1, binary64 Cholesky, final update sweep.

value = algorithmic bytes / time (CholQR2: 32 m k bytes per step), counted
only if ||Q^T Q - I||_F <= 1e-14 and the residual <= 1e-14, both measured
after the timed region by the CPU oracle (binary128-accurate measures of the
binary64 Q and R; with --no-cpu the library's DD Gram of Q stands in, and
the line says so).  The plain binary64 CholQR on the same input is timed
beside it (its GB/s and time ratio are reported; it does not reach the
orthogonality gate at this kappa).

Other workloads (--workload): c2 (binary64 CholQR2, 1e7 x k), c4 (fp32
16,777,216 x 64, split-BF16 Gram + binary64 passes), c5 (256-block batch with
a locked basis), c1 (plain CholQR 20000 x 8).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0
FP64_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # FP64 lane-ops per second (39.3 T)
# The DD Gram's algorithmic work per (i <= j) pair and row: the biased
# accumulation's fma, exact difference, fma for the remainder and add (its
# once-per-panel fold and the padding of diagonal tiles are overhead).
DD_GRAM_OPS = 4.0
# The same work counted as a Dot2 step (TwoProduct + TwoSum and the error
# accumulation, about 10 binary64 instructions per product): the count the
# measurement plan prices a DD Gram at.  A fraction against it can exceed 1,
# as the biased sums need fewer instructions for the same accuracy.
DD_GRAM_OPS_DOT2 = 10.0

# HBM bytes per dispatch of the dominant kernel of the default workload, from
# two rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE; calibrated on a plain
# device copy of known size, see profiles/dd_cholqr2_4Mx32_hbm_counters.md).
# Valid only for the kernel sources they were taken on: reported as null once
# those sources change.
DD_GRAM_TRAFFIC = {"bytes": 1033706710, "lane_ops": 10228965376,
                   "sources": ["gram.hip", "gram_impl.hpp", "dd.hpp", "internal.hpp"],
                   "sha256": "2ceb2a0649039a8c2d06e7938f41266fb11b968b1b8fca7126d2550b8afcf7a2"}


def measured_traffic(rec, key="bytes"):
    import hashlib
    if rec.get("sha256") is None:
        return None
    h = hashlib.sha256()
    for f in rec["sources"]:
        h.update((ROOT / "paper_1806_01036_amd" / "csrc" / f).read_bytes())
    return rec[key] if h.hexdigest() == rec["sha256"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def omega_dd(borth, Q):
    ghi, glo = borth.gram(Q, prec="dd")
    g = ghi.cpu().numpy()
    lo = glo.cpu().numpy()
    k = g.shape[0]
    e = (g - np.eye(k)) + lo
    return float(np.linalg.norm(e))


def rho_gpu(torch, X, Q, R):
    res = X.to(torch.float64) - Q @ R
    return float(torch.linalg.norm(res) / torch.linalg.norm(X.to(torch.float64)))


def timed(torch, fn, steps, warmup):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def step_stats(torch, fn, n=20):
    """Per-step times (ms) of n more steps, each bracketed by its own pair of
    events on the library's stream: median, min and 90th percentile."""
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(n)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    return {"median": round(ms[n // 2], 4), "min": round(ms[0], 4),
            "p90": round(ms[int(0.9 * (n - 1))], 4)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_metrics(X, Q, R):
    """omega and rho of the GPU's result by the CPU oracle (binary128-
    accurate measures), and the seconds they took."""
    import oracle
    t0 = time.perf_counter()
    met = oracle.metrics(Q.cpu().numpy(), X, R.cpu().numpy())
    return float(met["omega"]), float(met["rho"]), time.perf_counter() - t0


def cpu_baseline_extra(X, dd, rows1=500_000, rows_q=250_000):
    """The oracle's DD CholQR2 at one thread, and its binary128 thin QR (O1),
    each on the first rows of X, in GB/s of the same algorithmic bytes."""
    import oracle
    k = X.shape[1]
    nthr = oracle.num_threads()
    out = {}
    try:
        oracle.set_num_threads(1)
        r = min(rows1, X.shape[0])
        t0 = time.perf_counter()
        oracle.cholqr_steps(X[:r], dd_first=dd, passes=2)
        dt = time.perf_counter() - t0
        out["one_thread"] = dict(value=32.0 * r * k / dt / 1e9, unit="GB/s", cores=1,
                                 sample=f"oracle step-by-step {'DD' if dd else 'binary64'} CholQR2, "
                                        f"first {r} rows, 1 thread ({dt:.1f} s)")
    finally:
        oracle.set_num_threads(nthr)
    r = min(rows_q, X.shape[0])
    t0 = time.perf_counter()
    oracle.qr_q(X[:r])
    dt = time.perf_counter() - t0
    out["o1_binary128_qr"] = dict(value=24.0 * r * k / dt / 1e9, unit="GB/s", cores=nthr,
                                  sample=f"oracle exact thin QR in binary128 (Gram, Cholesky, "
                                         f"update; 24 m k bytes), first {r} rows ({dt:.1f} s)")
    # the oracle's DD Gram sweep alone (Dot2), at all threads and at one
    for nt, rows in ((nthr, 4 * rows1), (1, rows1 // 2)):
        try:
            oracle.set_num_threads(nt)
            r = min(rows, X.shape[0])
            t0 = time.perf_counter()
            oracle.gram_dot2(X[:r])
            dt = time.perf_counter() - t0
        finally:
            oracle.set_num_threads(nthr)
        out["o2_dd_gram" + ("" if nt == nthr else "_one_thread")] = dict(
            value=8.0 * r * k / dt / 1e9, unit="GB/s", cores=nt,
            sample=f"oracle DD Gram (Dot2, 8 m k bytes), first {r} rows, {nt} thread(s) ({dt:.1f} s)")
    return out


def cpu_baseline_cholqr2(X, dd, target_s=10.0):
    import oracle
    m = X.shape[0]
    rows = min(m, 250_000)
    t0 = time.perf_counter()
    oracle.cholqr_steps(X[:rows], dd_first=dd, passes=2)
    dt = time.perf_counter() - t0
    if dt < target_s and rows < m:
        rows = int(min(m, rows * max(1.0, target_s / max(dt, 1e-3))))
        t0 = time.perf_counter()
        oracle.cholqr_steps(X[:rows], dd_first=dd, passes=2)
        dt = time.perf_counter() - t0
    # the whole block takes less than the target: repeat it (at most 10 runs)
    reps = 1
    if dt < target_s and rows == m:
        reps = int(min(10, np.ceil(target_s / max(dt, 1e-3))))
        if reps > 1:
            t0 = time.perf_counter()
            for _ in range(reps):
                oracle.cholqr_steps(X, dd_first=dd, passes=2)
            dt = time.perf_counter() - t0
    k = X.shape[1]
    return dict(value=32.0 * rows * k * reps / dt / 1e9, unit="GB/s", cores=oracle.num_threads(),
                kind="oracle", cpu_model=cpu_model(),
                sample=f"oracle step-by-step {'DD' if dd else 'binary64'} CholQR2 on the first "
                       f"{rows} rows of the same X, {reps} run(s) ({dt:.1f} s)")


def run_c3(args, torch, borth, synth):
    m, k, kappa, seed = 4_000_000, 32, 1e12, 302
    log(f"generating X {m}x{k} kappa={kappa:g}")
    X = synth.svd_matrix(m, k, kappa, seed)
    import hashlib
    x_sha = hashlib.sha256(X.tobytes()).hexdigest()  # the input, for reproduction
    Xd = torch.from_numpy(X).cuda()
    Q = torch.empty_like(Xd)
    R = torch.empty((k, k), dtype=torch.float64, device="cuda")
    ctx = borth.default_context()
    if args.copy_probe:
        # plain device copy of known size (8 m k bytes read and written):
        # calibrates the HBM byte counters of a profiling run
        for _ in range(3):
            Q.copy_(Xd)
        torch.cuda.synchronize()
        log(f"copy probe: 3 x {8 * m * k} bytes")

    def step():
        borth.orthonormalize(Xd, gram="dd", passes=2, out=Q, R=R, sync=False, ctx=ctx)

    # correctness of the timed configuration (status + orthogonality gate)
    _, _, _, info = borth.orthonormalize(Xd, gram="dd", passes=2, out=Q, R=R, ctx=ctx)
    assert info.status == 0, info
    # the dominant kernel (DD Gram sweep) is timed with HIP events inside the
    # timed region; the update sweeps in a few steps after it
    ctx.set_profiling(True, kinds=(0,))
    t = timed(torch, step, args.steps, args.warmup)
    gram_ms, gram_n = ctx.kernel_time(0)
    ctx.set_profiling(False)
    ctx.set_profiling(True, kinds=(1,))
    timed(torch, step, 5, 0)
    upd_ms, upd_n = ctx.kernel_time(1)
    ctx.set_profiling(False)
    per_step = step_stats(torch, step)
    om_dd = omega_dd(borth, Q)
    rho_dd = rho_gpu(torch, Xd, Q, R)
    if args.no_cpu:
        om, rho, gate = om_dd, rho_dd, "library DD Gram of Q (--no-cpu)"
    else:
        om, rho, t_met = oracle_metrics(X, Q, R)
        gate = f"CPU oracle, binary128-accurate measures ({t_met:.1f} s)"
    log(f"DD CholQR2: {t*1e3:.3f} ms/step omega={om:.2e} rho={rho:.2e} ({gate}) "
        f"gram {gram_ms:.3f} ms x{gram_n}, update {upd_ms:.3f} ms x{upd_n}")

    # plain binary64 CholQR on the same input
    Qp = torch.empty_like(Xd)

    def step_plain():
        borth.orthonormalize(Xd, gram="f64", passes=1, out=Qp, R=R, sync=False, check=False,
                             ctx=ctx)
    tp = timed(torch, step_plain, args.steps, args.warmup)
    _, _, _, infp = borth.orthonormalize(Xd, gram="f64", passes=1, out=Qp, R=R, check=False,
                                         ctx=ctx)

    def step_f2():
        borth.orthonormalize(Xd, gram="f64", passes=2, out=Qp, R=R, sync=False, check=False,
                             ctx=ctx)
    tf2 = timed(torch, step_f2, args.steps, args.warmup)

    # streaming probes on the same X (the library's plain HIP kernels): a
    # read of 8 m k bytes, a copy (8 m k read + 8 m k written) with ordinary
    # and with non-temporal stores
    _, read_gbs, _ = borth.stream_probe("read", Xd, Qp, reps=10, ctx=ctx)
    _, copy_gbs, _ = borth.stream_probe("copy", Xd, Qp, reps=10, ctx=ctx)
    _, copynt_gbs, _ = borth.stream_probe("copy_nt", Xd, Qp, reps=10, ctx=ctx)
    # FP64 vector-ALU probe (register-only chains): the issue ceiling the DD
    # Gram sweep is bound by, plain FMAs and the DD step's fma/add/fma/add
    fma_rate, fma_waves = borth.valu_probe("fma", Qp, ctx=ctx)
    dd_rate, dd_waves = borth.valu_probe("dd_step", Qp, ctx=ctx)

    bytes_step = 32.0 * m * k
    gbs = bytes_step / t / 1e9 if (om <= 1e-14 and rho <= 1e-14) else 0.0
    # dominant kernel: the DD Gram sweep, bound by the FP64 vector ALUs.
    # Algorithmic work: DD_GRAM_OPS FP64 VALU lane-ops per (i <= j) pair per row.
    pairs = k * (k + 1) / 2 * m
    ops = DD_GRAM_OPS * pairs
    achieved = ops / (gram_ms * 1e-3) / 1e12
    executed = measured_traffic(DD_GRAM_TRAFFIC, "lane_ops")
    out = {
        "metric": "block-orth GB/s (% HBM peak) at ||Q^T Q - I|| <= 1e-14: DD/split vs plain FP64 CholQR",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+dd",
        "data": "synthetic",
        "config": {"workload": "DD-Gram CholQR2, X 4,000,000 x 32 binary64, kappa=1e12 "
                               "(U diag(sigma) V^T, seed 302)",
                   "m": m, "k": k, "kappa": kappa, "passes": 2, "gram": "dd"},
        "input_sha256": x_sha,
        "pct_hbm_peak": round(100.0 * gbs / HBM_PEAK_GBS, 2),
        "step_ms": per_step,
        "stream_probe": {"kernel": "borth_stream_probe (hand-written HIP, 16-byte vectors)",
                         "read_GBs": round(read_gbs, 1), "copy_GBs": round(copy_gbs, 1),
                         "copy_nt_GBs": round(copynt_gbs, 1),
                         "value_over_read_probe": round(gbs / read_gbs, 4)},
        "valu_probe": {"kernel": "borth_valu_probe (hand-written HIP, register-only FP64 chains)",
                       "fma_Tops": round(fma_rate / 1e12, 2), "fma_waves_per_simd": fma_waves,
                       "dd_step_Tops": round(dd_rate / 1e12, 2), "dd_step_waves_per_simd": dd_waves,
                       "unit": "T FP64 VALU lane-ops/s"},
        "omega": om,
        "rho": rho,
        "gate": gate,
        "omega_dd_gram": om_dd,
        "plain_fp64_cholqr": {"ms_per_step": round(tp * 1e3, 4),
                              "GB/s": round(24.0 * m * k / tp / 1e9, 2),
                              "status": infp.status,
                              "dd_cholqr2_time_ratio": round(t / tp, 3)},
        "fp64_cholqr2_ms_per_step": round(tf2 * 1e3, 4),
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VALU_TOPS,
                     "unit": "Tops/s (FP64 VALU lane-ops)", "frac": round(achieved / FP64_VALU_TOPS, 4),
                     "work": "4 lane-ops per (i <= j) pair and row (the biased DD sums)",
                     "frac_dot2_count": round(DD_GRAM_OPS_DOT2 * pairs / (gram_ms * 1e-3) / 1e12
                                              / FP64_VALU_TOPS, 4),
                     "frac_executed": (round(executed / (gram_ms * 1e-3) / 1e12 / FP64_VALU_TOPS, 4)
                                       if executed else None),
                     "frac_of_fma_probe": round(achieved * 1e12 / fma_rate, 4),
                     "traffic": measured_traffic(DD_GRAM_TRAFFIC),
                     "traffic_unit": "bytes per launch (algorithmic 8 m k = %d)" % (8 * m * k),
                     "kernel": "gram_dd_dma_kernel",
                     "kernel_ms": round(gram_ms, 4)},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_cholqr2(X, dd=True)
        out["cpu_baseline"].update(cpu_baseline_extra(X, dd=True))
    return out


def run_c1(args, torch, borth, synth):
    """Plain binary64 CholQR of a small block (20,000 x 8, kappa 1e4): bound
    by launch latency, not by HBM; timed eagerly and as a replayed hipGraph."""
    m, k = 20_000, 8
    X = synth.svd_matrix(m, k, 1e4, 101)
    Xd = torch.from_numpy(X).cuda()
    Q = torch.empty_like(Xd)
    R = torch.empty((k, k), dtype=torch.float64, device="cuda")
    ctx = borth.default_context()
    res = {}
    # one pass of plain CholQR loses c kappa^2 u of orthogonality: the
    # per-stage gate is omega <= 100 kappa^2 u and rho <= 1e-14
    kappa = 1e4
    om_gate = 100.0 * kappa ** 2 * 2.0 ** -53
    for graph in (False, True):
        def step():
            borth.orthonormalize(Xd, gram="f64", passes=1, graph=graph, out=Q, R=R, sync=False,
                                 ctx=ctx)
        steps = max(args.steps, 200)
        t = timed(torch, step, steps, max(args.warmup, 20))
        if args.no_cpu:
            om, rho = omega_dd(borth, Q), rho_gpu(torch, Xd, Q, R)
        else:
            om, rho, _ = oracle_metrics(X, Q, R)
        res["graph" if graph else "eager"] = dict(us=t * 1e6, GBs=24.0 * m * k / t / 1e9, omega=om,
                                                  rho=rho)
        log("graph" if graph else "eager", res["graph" if graph else "eager"])
    r = res["graph"]
    ok = r["omega"] <= om_gate and r["rho"] <= 1e-14
    return {
        "metric": "block-orth GB/s (% HBM peak) at ||Q^T Q - I|| <= 1e-14: DD/split vs plain FP64 CholQR",
        "value": round(r["GBs"] if ok else 0.0, 3), "unit": "GB/s", "n_gpus": 1,
        "gate": f"one plain CholQR pass: omega <= 100 kappa^2 u = {om_gate:.2e}, rho <= 1e-14"
                + (" (library DD Gram, --no-cpu)" if args.no_cpu else " (CPU oracle)"),
        "steps": max(args.steps, 200), "warmup": max(args.warmup, 20),
        "ms_per_step": round(r["us"] * 1e-3, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "plain binary64 CholQR, X 20,000 x 8, kappa=1e4", "m": m, "k": k},
        "all": res,
    }


def run_c2(args, torch, borth, synth):
    m, k = 10_000_000, args.k
    X = synth.svd_matrix(m, k, 1e6, 200 + k)
    Xd = torch.from_numpy(X).cuda()
    Q = torch.empty_like(Xd)
    R = torch.empty((k, k), dtype=torch.float64, device="cuda")
    ctx = borth.default_context()
    res = {}
    for sched in ("recompute", "materialize"):
        def step():
            borth.orthonormalize(Xd, gram="f64", passes=2, sched=sched, out=Q, R=R, sync=False,
                                 ctx=ctx)
        ctx.set_profiling(True)
        t = timed(torch, step, args.steps, args.warmup)
        g_ms, _ = ctx.kernel_time(0)
        u_ms, _ = ctx.kernel_time(1)
        ctx.set_profiling(False)
        om = omega_dd(borth, Q)
        res[sched] = dict(ms=t * 1e3, GBs=32.0 * m * k / t / 1e9, omega=om, gram_ms=g_ms,
                          gram_GBs=8.0 * m * k / (g_ms * 1e-3) / 1e9, update_ms=u_ms)
        log(sched, res[sched])
    best = min(res, key=lambda s: res[s]["ms"])
    r = res[best]
    return {
        "metric": "block-orth GB/s (% HBM peak) at ||Q^T Q - I|| <= 1e-14: DD/split vs plain FP64 CholQR",
        "value": round(r["GBs"] if r["omega"] <= 1e-14 else 0.0, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(r["ms"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"binary64 CholQR2, X 10,000,000 x {k}, kappa=1e6", "m": m, "k": k,
                   "sched": best},
        "all": res,
        "roofline": {"bound": "hbm", "achieved": round(r["gram_GBs"], 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(r["gram_GBs"] / HBM_PEAK_GBS, 4),
                     "traffic": None, "kernel": "gram_mfma_kernel"},
    }


def run_c4(args, torch, borth, synth):
    m, k = 16_777_216, 64
    log("generating fp32 X", m, k)
    X = synth.svd_matrix(m, k, 1e6, 401).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    del X
    Q = torch.empty((m, k), dtype=torch.float64, device="cuda")
    R = torch.empty((k, k), dtype=torch.float64, device="cuda")
    ctx = borth.default_context()
    res = {}
    for passes in (2, 3):
        def step():
            borth.orthonormalize(Xd, gram="split", passes=passes, out=Q, R=R, sync=False, ctx=ctx)
        ctx.set_profiling(True)
        t = timed(torch, step, args.steps, args.warmup)
        g_ms, _ = ctx.kernel_time(0)
        ctx.set_profiling(False)
        om = omega_dd(borth, Q)
        nbytes = (4.0 + 12.0 + 16.0 * (passes - 1)) * m * k
        res[passes] = dict(ms=t * 1e3, GBs=nbytes / t / 1e9, omega=om, gram_ms=g_ms,
                           gram_GBs=4.0 * m * k / (g_ms * 1e-3) / 1e9)
        log(passes, res[passes])
    r = res[3]
    return {"metric": "block-orth GB/s (% HBM peak) at ||Q^T Q - I|| <= 1e-14: DD/split vs plain FP64 CholQR",
            "value": round(r["GBs"] if r["omega"] <= 1e-14 else 0.0, 2), "unit": "GB/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(r["ms"], 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32+bf16-split+f64", "data": "synthetic",
            "config": {"workload": "split-BF16 Gram + 2 binary64 passes, X 16,777,216 x 64 fp32, kappa=1e6"},
            "all": res}


def run_c5(args, torch, borth, synth):
    """256 independent blocks (rows uniform in [1e4, 1e6], widths {8, 16, 32,
    64}, kappa log-uniform in [1e3, 1e10], a 16-column locked basis each):
    projection + DD-Gram CholQR2 (P,C,P,C) of all blocks per step, one graph
    launch."""
    nb = args.blocks
    table = synth.batch_table(nb, seed=5000)
    ky = 16
    log(f"generating {nb} blocks on the device")
    blocks = []
    tot_rows = 0
    for t in table:
        X = synth.svd_matrix_device(t["m"], t["k"], t["kappa"], t["seed"])
        Y = synth.locked_basis_device(t["m"], ky, t["seed"] + 100_000)
        blocks.append({"X": X, "Y": Y, "Q": torch.empty_like(X),
                       "R": torch.empty((t["k"], t["k"]), dtype=torch.float64, device="cuda"),
                       "C": torch.empty((ky, t["k"]), dtype=torch.float64, device="cuda")})
        tot_rows += t["m"]
    torch.cuda.synchronize()
    ctx = borth.default_context()
    t0 = time.perf_counter()
    ctx.autotune(None, budget_ms=args.tune_ms)
    log(f"autotune {time.perf_counter() - t0:.1f} s")
    # per-kernel durations from an eager (profiled) run, then the graph
    ctx.set_profiling(True)
    _, infos = borth.batch_orthonormalize(blocks, gram="dd", passes=2, ctx=ctx)
    g_ms, g_n = ctx.kernel_time(0)
    u_ms, u_n = ctx.kernel_time(1)
    ctx.set_profiling(False)
    bad = [i for i, inf in enumerate(infos) if inf.status != 0]
    assert not bad, f"blocks with nonzero status: {bad[:10]}"

    persistent = False  # the default driver: one launch per phase

    def step():
        borth.batch_orthonormalize(blocks, gram="dd", passes=2, graph=True, sync=False, ctx=ctx)
    t = timed(torch, step, args.steps, args.warmup)

    # the persistent single launch, timed beside it (the whole step in one
    # kernel: its duration from the library's event timing)
    def step_persistent():
        borth.batch_orthonormalize(blocks, gram="dd", passes=2, graph=True, persistent=True,
                                   sync=False, ctx=ctx)
    t_ps = timed(torch, step_persistent, args.steps, args.warmup)
    ctx.set_profiling(True)
    borth.batch_orthonormalize(blocks, gram="dd", passes=2, persistent=True, ctx=ctx)
    ps_ms, ps_n = ctx.kernel_time(0)
    ctx.set_profiling(False)
    log(f"batch: one persistent launch {t_ps*1e3:.3f} ms/step (kernel {ps_ms:.3f} ms x {ps_n})")
    # per-block orthogonality (DD Gram of [Y | Q]): omega and omega_Y
    om_max = omy_max = 0.0
    for b in blocks:
        ghi, glo = borth.gram(b["Q"], A=b["Y"], prec="dd")
        g = ghi.cpu().numpy() + 0.0
        lo = glo.cpu().numpy()
        k = b["X"].shape[1]
        gq = (g[ky:, ky:] - np.eye(k)) + lo[ky:, ky:]
        gy = g[:ky, ky:] + lo[:ky, ky:]
        om_max = max(om_max, float(np.linalg.norm(gq)))
        omy_max = max(omy_max, float(np.linalg.norm(gy)))
    ok = om_max <= 1e-14 and omy_max <= 1e-14
    nbytes = sum(8.0 * tt["m"] * (4 * tt["k"] + 3 * ky) for tt in table)
    gbs = nbytes / t / 1e9 if ok else 0.0
    # dominant kernel: the persistent launch (the whole step: every sweep,
    # reduction and k x k step), or the batched DD Gram launches (one per
    # shape class) of the launch-per-phase driver
    ops = sum(DD_GRAM_OPS * tt["m"] * (ky + tt["k"]) * (ky + tt["k"] + 1) / 2 for tt in table)
    gram_total_ms = g_ms * g_n
    achieved = ops / (gram_total_ms * 1e-3) / 1e12
    log(f"batch: {t*1e3:.3f} ms/step, {gbs:.1f} GB/s, omega_max={om_max:.2e} "
        f"omega_y_max={omy_max:.2e}; persistent={persistent}; timed launches: {g_n} x {g_ms:.3f} ms"
        f" (Gram or whole step), updates {u_n} x {u_ms:.3f} ms")
    if persistent:
        roof = {"bound": "hbm", "achieved": round(nbytes / (gram_total_ms * 1e-3) / 1e9, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(nbytes / (gram_total_ms * 1e-3) / 1e9
                                                                  / HBM_PEAK_GBS, 4),
                "work": "algorithmic bytes of the step (sum 8 m (4 k + 3 ky)) over the persistent "
                        "launch, which runs the whole step",
                "dd_gram_alu_frac": round(achieved / FP64_VALU_TOPS, 4),
                "traffic": None, "kernel": "batch_persistent_kernel", "kernel_ms": round(gram_total_ms, 4)}
    else:
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VALU_TOPS,
                "unit": "Tops/s (FP64 VALU lane-ops)", "frac": round(achieved / FP64_VALU_TOPS, 4),
                "traffic": None, "kernel": "gram DD sweeps (batched, all classes)",
                "kernel_ms": round(gram_total_ms, 4)}
    out = {
        "metric": "block-orth GB/s (% HBM peak) at ||Q^T Q - I|| <= 1e-14: DD/split vs plain FP64 CholQR",
        "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t * 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64+dd", "data": "synthetic",
        "config": {"workload": f"{nb} blocks, rows U[1e4,1e6] (total {tot_rows}), k in "
                               "{8,16,32,64}, kappa log-U[1e3,1e10], locked Y 16 columns; "
                               "projection + DD-Gram CholQR2 (P,C,P,C), one hipGraph launch",
                   "blocks": nb, "rows_total": tot_rows, "ky": ky, "passes": 2, "gram": "dd"},
        "pct_hbm_peak": round(100.0 * gbs / HBM_PEAK_GBS, 2),
        "driver": "one launch per phase",
        "persistent_launch": {"ms_per_step": round(t_ps * 1e3, 4), "kernel_ms": round(ps_ms, 4),
                              "GB/s": round(nbytes / t_ps / 1e9, 1) if ok else 0.0},
        "omega_max": om_max, "omega_y_max": omy_max,
        "roofline": roof,
    }
    if not args.no_cpu:
        import oracle
        t0_ = table[0]
        rows = min(t0_["m"], 100_000)
        X0 = blocks[0]["X"][:rows].cpu().numpy()
        Y0 = blocks[0]["Y"][:rows].cpu().numpy()
        tc = time.perf_counter()
        oracle.cholqr_steps(X0, Y0, dd_first=True, passes=2, project_each_pass=True)
        dt = time.perf_counter() - tc
        out["cpu_baseline"] = dict(
            value=8.0 * rows * (4 * t0_["k"] + 3 * ky) / dt / 1e9, unit="GB/s",
            cores=oracle.num_threads(), kind="oracle",
            sample=f"oracle DD CholQR2 with projection on {rows} rows of block 0 "
                   f"(k={t0_['k']}, {dt:.1f} s)")
    return out


# Runtime per block vector of the paper's iterated project / SVQB experiment
# (Fig. 8, an Intel Haswell workstation; n = 8e6 rows, kappa(X) = 1e6,
# kappa(X, W) = 1e12), read off the figure: (k_y, n_b) -> seconds, for the
# plain binary64 variant, the variant with fused operations and the one with
# fused DD operations.  Context only (other hardware).
FIG8_PAPER = {
    "plain": {(10, 1): 0.0164, (10, 2): 0.0216, (10, 4): 0.0195, (20, 1): 0.0324, (20, 2): 0.0425,
              (20, 4): 0.0382, (40, 1): 0.0805, (40, 2): 0.0901, (40, 4): 0.0644},
    "fused": {(10, 1): 0.0151, (10, 2): 0.0180, (10, 4): 0.0138, (20, 1): 0.0307, (20, 2): 0.0357,
              (20, 4): 0.0246, (40, 1): 0.0784, (40, 2): 0.0814, (40, 4): 0.0466},
    "fused_dd": {(10, 1): 0.0152, (10, 2): 0.0127, (10, 4): 0.0117, (20, 1): 0.0309, (20, 2): 0.0256,
                 (20, 4): 0.0205, (40, 1): 0.0783, (40, 2): 0.0611, (40, 4): 0.0410}}
# variant -> (Gram precision, phase II, fused Gram columns); "fused_dd" is the
# paper's DD project / SVQB, "fused_dd_chol" the same with DD Cholesky
FIG8_VARIANTS = {"plain": ("f64", "svqb", False), "fused": ("f64", "svqb", True),
                 "fused_dd": ("dd", "svqb", True), "fused_dd_chol": ("dd", "chol", True)}


def run_fig8(args, torch, borth, synth):
    """Iterated two-phase scheme to convergence (eps 1e-10) on the shapes of
    the paper's runtime experiment: n = 8e6 rows, k_y in {10, 20, 40} locked
    vectors, n_b in {1, 2, 4} new ones, kappa(X) = 1e6, kappa(X, Y) = 1e12.
    Variants: binary64 Gram with SVQB, a full Gram sweep in every pass
    ("plain"); the same with each update accumulating the next pass's Gram
    columns ("fused"); DD Gram with DD SVQB, fused ("fused_dd"), and with DD
    Cholesky ("fused_dd_chol")."""
    n = 8_000_000
    rows = []
    for ky in (10, 20, 40):
        for k in (1, 2, 4):
            X, Y = synth.projected_pair_device(n, k, ky, 1e6, 1e12, 7000 + 10 * ky + k)
            Q = torch.empty_like(X)
            for var, (gram, fact, fuse) in FIG8_VARIANTS.items():
                kw = dict(gram=gram, fact=fact, eps=1e-10, max_iter=10, out=Q, fuse=fuse)
                res = borth.orthonormalize_iter(X, Y, **kw)
                torch.cuda.synchronize()
                ts = []
                for _ in range(max(1, args.steps)):
                    t0 = time.perf_counter()
                    res = borth.orthonormalize_iter(X, Y, **kw)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                t = sorted(ts)[len(ts) // 2]
                it = res[3]
                ghi, glo = borth.gram(Q, A=Y, prec="dd")
                g = ghi.cpu().numpy()
                lo = glo.cpu().numpy()
                om = float(np.linalg.norm((g[ky:, ky:] - np.eye(k)) + lo[ky:, ky:]))
                omy = float(np.linalg.norm(g[:ky, ky:] + lo[:ky, ky:]))
                r = dict(ky=ky, nb=k, variant=var, passes=it.passes_run, converged=it.converged,
                         s_per_vector=t / k, omega=om, omega_y=omy,
                         paper_haswell_s_per_vector=FIG8_PAPER[var.replace("_chol", "")][(ky, k)])
                log(r)
                rows.append(r)
            del X, Y, Q
    return {"workload": "iterated project / orthonormalize to convergence, n = 8e6, "
                        "kappa(X) = 1e6, kappa(X, Y) = 1e12 (the paper's runtime experiment)",
            "data": "synthetic", "n_gpus": 1, "results": rows}


def _orth_levels(borth, Q, Y, k, ky):
    """||Q^T Q - I||_F and ||Y^T Q||_F from the library's DD Gram of [Y | Q]."""
    ghi, glo = borth.gram(Q, A=Y, prec="dd") if ky else borth.gram(Q, prec="dd")
    g = ghi.cpu().numpy() + glo.cpu().numpy()
    om = float(np.linalg.norm(g[ky:, ky:] - np.eye(k)))
    omy = float(np.linalg.norm(g[:ky, ky:])) if ky else 0.0
    return om, omy


def _orth_levels_dd(torch, borth, Qh, Ql, Y, k, ky):
    """The same levels for a DD result Qh + Ql, from the library's Dot2 DD Gram
    of [Y | Qh | Ql], its blocks combined so that the low words count."""
    ghi, glo = borth.gram(torch.cat([Qh, Ql], dim=1), A=Y, prec="dd_dot2")
    hi, lo = ghi.cpu().numpy(), glo.cpu().numpy()
    H, L = slice(ky, ky + k), slice(ky + k, ky + 2 * k)
    D = (((hi[H, H] - np.eye(k)) + lo[H, H]) + ((hi[H, L] + hi[L, H]) + (lo[H, L] + lo[L, H]))
         + hi[L, L])
    om = float(np.linalg.norm(D))
    omy = float(np.linalg.norm((hi[:ky, H] + hi[:ky, L]) + (lo[:ky, H] + lo[:ky, L]))) if ky else 0.0
    return om, omy


def run_fig7(args, torch, borth, synth):
    """One two-phase pass (projection against Y, then orthonormalization) on
    the shape of the paper's accuracy experiment (Fig. 7): n = 1000 rows,
    k_y = 20 locked vectors, n_b = 4 new ones.  Left: ||Y^T Q|| against
    kappa(X, Y) at kappa(X) in {1, 1e3}; right: ||Q^T Q - I|| against kappa(X)
    at kappa(X, Y) = kappa(X).  Variants: binary64 Gram with SVQB; DD Gram
    (biased accumulation) with DD SVQB or DD Cholesky and DD update; the
    latter with the Dot2 accumulation, rounded to binary64 or returned in DD
    (Q + Q_lo, measured as such)."""
    n, ky, k = 1000, 20, 4
    variants = {"f64_svqb": ("f64", "svqb"), "dd_svqb": ("dd", "svqb"), "dd_chol": ("dd", "chol"),
                "dd_chol_dot2": ("dd_dot2", "chol")}
    rows = []

    def one(kx, kxy, seed):
        X, Y = synth.projected_pair_device(n, k, ky, kx, kxy, seed)
        for var, (gram, fact) in variants.items():
            Q, R, C, info = borth.orthonormalize(X, Y, gram=gram, fact=fact, passes=1, check=False)
            torch.cuda.synchronize()
            om, omy = _orth_levels(borth, Q, Y, k, ky)
            r = dict(kappa_x=kx, kappa_xy=kxy, variant=var, status=info.status, omega=om,
                     omega_y=omy)
            log(r)
            rows.append(r)
        # the DD result itself (Q + Q_lo), Dot2 accumulation
        Q, Ql, R, C, info = borth.orthonormalize_dd(X, Y, dot2=True, check=False)
        torch.cuda.synchronize()
        om, omy = _orth_levels_dd(torch, borth, Q, Ql, Y, k, ky)
        r = dict(kappa_x=kx, kappa_xy=kxy, variant="dd_chol_dot2_ddq", status=info.status,
                 omega=om, omega_y=omy)
        log(r)
        rows.append(r)

    for kx in (1.0, 1e3):
        for e in range(0, 19, 3):
            kxy = 10.0 ** e
            if kxy >= kx:
                one(kx, kxy, 4000 + e + (0 if kx == 1.0 else 100))
    for e in range(0, 13, 3):
        kx = 10.0 ** e
        one(kx, kx, 4500 + e)
    return {"workload": "one project / orthonormalize pass, n = 1000, k_y = 20, n_b = 4 "
                        "(the paper's accuracy experiment)",
            "data": "synthetic", "n_gpus": 1, "results": rows}


def run_binner(args, torch, borth, synth):
    """Iterated scheme in a B-inner product, B = diag(w), w log-uniform with
    kappa(B) = 1e4, on the runtime experiment's shapes (n = 8e6, kappa(X) =
    1e6, kappa(X, Y) = 1e12), against the same call with B = I."""
    n = 8_000_000
    rows = []
    for ky, k in ((20, 4), (40, 1), (10, 2)):
        X0, Y0 = synth.projected_pair_device(n, k, ky, 1e6, 1e12, 7000 + 10 * ky + k)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(8000 + ky + k)
        w = torch.exp((torch.rand(n, generator=gen, dtype=torch.float64, device="cuda") - 0.5)
                      * np.log(1e4))
        s = torch.rsqrt(w)[:, None]
        X = (X0 * s).contiguous()  # B-orthonormal Y, same conditions as (X0, Y0) in B
        Y = (Y0 * s).contiguous()
        Q = torch.empty_like(X)
        for var, gram, fact in (("f64_svqb", "f64", "svqb"), ("dd_svqb", "dd", "svqb")):
            for weighted in (True, False):
                # B = I: the Euclidean problem (X0, Y0) of the same shape
                kw = dict(gram=gram, fact=fact, eps=1e-10, max_iter=10, out=Q,
                          B=w if weighted else None)
                Xi, Yi = (X, Y) if weighted else (X0, Y0)
                res = borth.orthonormalize_iter(Xi, Yi, **kw)
                torch.cuda.synchronize()
                ts = []
                for _ in range(max(1, args.steps)):
                    t0 = time.perf_counter()
                    res = borth.orthonormalize_iter(Xi, Yi, **kw)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t0)
                t = sorted(ts)[len(ts) // 2]
                r = dict(ky=ky, nb=k, variant=var, B="diag(w)" if weighted else "I",
                         passes=res[3].passes_run, converged=res[3].converged,
                         s_per_vector=t / k)
                if weighted:
                    # B-orthogonality from the DD Gram of [W^1/2 Y | W^1/2 Q]
                    sw = torch.sqrt(w)[:, None]
                    om, omy = _orth_levels(borth, (Q * sw).contiguous(), (Y * sw).contiguous(),
                                           k, ky)
                    r.update(omega_b=om, omega_y_b=omy)
                log(r)
                rows.append(r)
        del X, Y, Q, w, X0, Y0
    return {"workload": "iterated project / orthonormalize in a B-inner product, n = 8e6, "
                        "kappa(B) = 1e4", "data": "synthetic", "n_gpus": 1, "results": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "c4", "c5", "fig7", "fig8", "binner"])
    ap.add_argument("--k", type=int, default=32)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--blocks", type=int, default=256)
    ap.add_argument("--tune-ms", type=int, default=3000)
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a plain copy of X before timing (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("this benchmark runs on exactly one GPU: the block orthonormalization path is "
              "built and measured on a single MI355X (multi-GPU sharding is design only)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1806_01036_amd as borth
    import synth
    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    fn = {"c1": run_c1, "c3": run_c3, "c2": run_c2, "c4": run_c4, "c5": run_c5, "fig7": run_fig7, "fig8": run_fig8, "binner": run_binner}.get(args.workload)
    if fn is None:
        raise SystemExit(f"workload {args.workload} not available")
    out = fn(args, torch, borth, synth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
