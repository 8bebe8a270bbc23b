"""The adjoint wave-trace analysis (paper_1002_0916_amd/probe/wave_trace.py)
on a synthetic trace: two SIMDs of one CU, known start and end times and
shader-clock cycles.  No GPU."""
import importlib.util
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _module():
    spec = importlib.util.spec_from_file_location(
        "wave_trace_under_test", os.path.join(ROOT, "paper_1002_0916_amd", "probe",
                                              "wave_trace.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_trace_analysis_on_a_synthetic_trace():
    wt = _module()
    buf = np.zeros((wt.MAX_WAVES, 4), dtype=np.uint64)
    base = 10 ** 9  # 100 MHz ticks: 1 tick = 10 ns
    # SIMD 0 (HW_ID bits 4-5 = 0): two waves 0-100 us and 0-50 us;
    # SIMD 1 (= 1): one wave 10-60 us.  XCC 3 for all.  Cycles at 2.0 GHz.
    waves = [(0, 100, 0), (0, 50, 0), (10, 60, 1)]
    for i, (s_us, e_us, simd) in enumerate(waves):
        buf[i, 0] = base + s_us * 100
        buf[i, 1] = base + e_us * 100
        buf[i, 2] = (np.uint64(3) << np.uint64(32)) | np.uint64(simd << 4)
        buf[i, 3] = (e_us - s_us) * 2000  # 2.0 GHz
    r = wt._analyse(buf, kernel_ms=0.1)
    assert r["waves"] == 3 and r["simds"] == 2
    assert r["span_us"] == 100.0
    assert r["waves_per_simd"] == [1, 2]
    assert r["simd_last_end_pct_0_10_50_90_100"][0] == 60.0
    assert r["simd_last_end_pct_0_10_50_90_100"][-1] == 100.0
    assert abs(r["xcd_median_clock_ghz"][3] - 2.0) < 1e-9
    # live waves per SIMD averaged over the span: SIMD 0 holds 2 waves for
    # 50 us and 1 for 50 us, SIMD 1 holds 1 for 50 us: (150 + 50) / (2 * 100)
    assert abs(r["live_mean"] - 1.0) < 0.01
    # at 90% of the span only SIMD 0's long wave is live
    assert r["simds_by_live_at_90pct"][:2] == [1, 1]
