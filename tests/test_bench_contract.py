"""CPU checks of bench.py's contract that need no GPU: one GPU only, and the
HBM-traffic figure it reports is tied to the kernel sources it was measured
on (a change to them turns the figure into null until it is measured again)."""
import re
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_figure_matches_the_profiled_sources():
    sys.path.insert(0, str(ROOT))
    import bench
    rec = bench.DD_GRAM_TRAFFIC
    if rec["sha256"] is None:
        # not measured on the current kernel sources: no figure is reported
        assert bench.measured_traffic(rec) is None
        assert bench.measured_traffic(rec, "lane_ops") is None
        return
    assert bench.measured_traffic(rec) == rec["bytes"]
    assert bench.measured_traffic(rec, "lane_ops") == rec["lane_ops"]
    # the committed counter summary holds the same figures
    prof = (ROOT / "profiles" / "dd_cholqr2_4Mx32_hbm_counters.md").read_text()
    m = re.search(r"`gram_dd_dma_kernel<false, false, 32, false>` \| \d+ \| [\d.]+ \| [\d.]+ \| ([\d.e+]+) \|", prof)
    assert m and abs(float(m.group(1)) - rec["bytes"]) <= 1e-4 * rec["bytes"]
    prof = (ROOT / "profiles" / "dd_cholqr2_4Mx32_valu_mfma_counters.md").read_text()
    m = re.search(r"`gram_dd_dma_kernel<false, false, 32, false>` \| [\d.]+ \| [\d.e+]+ \| ([\d.e+]+) \|", prof)
    assert m and abs(float(m.group(1)) * 64 - rec["lane_ops"]) <= 1e-3 * rec["lane_ops"]
    # any other source text gives no figure
    fake = dict(rec, sha256="0" * 64)
    assert bench.measured_traffic(fake) is None
