"""The measurement probes the bench compares its sweeps against: the HBM
streaming kernels (read, copy) and the FP64 vector-ALU kernel.  Their rates
must lie below the device's published peaks (8 TB/s HBM; 39.3 T FP64 lane
operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz) and the copy
must move the bytes unchanged."""
import pytest

from gpu_common import lib, note, torch_gpu

HBM_PEAK = 8.0e12
FP64_LANE_PEAK = 256 * 4 * 16 * 2.4e9


@pytest.mark.gpu
def test_stream_probe_rates_and_copy():
    borth = lib()
    torch = torch_gpu()
    n = 64 << 20  # 64 MiB
    src = torch.randn(n // 8, dtype=torch.float64, device="cuda")
    dst = torch.zeros_like(src)
    for kind in ("read", "copy", "copy_nt"):
        note("stream probe", kind, n)
        ms, gbs, grid = borth.stream_probe(kind, src, dst, reps=3)
        note("  ", ms, "ms", gbs, "GB/s grid", grid)
        assert ms > 0 and 1e2 < gbs < HBM_PEAK / 1e9 * 1.05
        assert grid % 2 == 0 and grid > 0
        if kind != "read":
            assert torch.equal(src, dst)
            dst.zero_()


@pytest.mark.gpu
def test_valu_probe_rates():
    borth = lib()
    torch = torch_gpu()
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    sink = torch.empty(8 * 256 * cus, dtype=torch.float64, device="cuda")
    for kind in ("fma", "dd_step"):
        note("valu probe", kind)
        rate, waves = borth.valu_probe(kind, sink)
        note("  ", rate / 1e12, "T lane-ops/s at", waves, "waves per SIMD")
        assert 1e12 < rate < FP64_LANE_PEAK * 1.01
        assert waves in (1, 2, 4, 8)
    assert torch.isfinite(sink).all()
    with pytest.raises(borth.BorthError):
        borth.valu_probe("fma", sink[: 256 * cus])
