"""The profiles/ summaries that bench.py writes from rocprofv3 CSV output
(`bench.py --summarize`), on small synthetic CSV files: the copy calibration
of FETCH_SIZE / WRITE_SIZE, the per-interaction counter arithmetic, the
trace-versus-event table, and the rule that a kernel's recorded traffic is
withheld once its sources change; that the committed record matches the
headline kernels' current sources; and the one-GPU guard.  No GPU."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HEADER = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name",
          "Counter_Value"]
ADJ1 = ("void cgh::(anonymous namespace)::adj_partial_kernel<1>(HIP_vector_type<float, 4u> "
        "const*, float const*, long, int)")


@pytest.fixture()
def bench(tmp_path, monkeypatch):
    spec = importlib.util.spec_from_file_location("bench_under_test",
                                                  os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    out = tmp_path / "profiles"
    out.mkdir()
    monkeypatch.setattr(mod, "PROFILES", str(out))
    return mod


def _counters(path, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(HEADER)
        for i, (kernel, counter, value) in enumerate(rows):
            w.writerow([i + 1, i + 1, kernel, 1024, counter, float(value)])


def test_traffic_is_copy_calibrated_and_withheld_when_sources_change(bench, tmp_path):
    run = tmp_path / "run"
    # the kernel: FETCH_SIZE 1000 and 3000 KiB (mean 2000), WRITE_SIZE 500 KiB
    _counters(run / "fetch" / "f_counter_collection.csv",
              [(ADJ1, "FETCH_SIZE", 1000), (ADJ1, "FETCH_SIZE", 3000)])
    _counters(run / "write" / "w_counter_collection.csv", [(ADJ1, "WRITE_SIZE", 500)])
    # a 256 MiB copy reads FETCH_SIZE = half its bytes and WRITE_SIZE = all of them
    _counters(run / "copy_fetch" / "c_counter_collection.csv",
              [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 131072)] * 2)
    _counters(run / "copy_write" / "c_counter_collection.csv",
              [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 262144)])
    bench.summarize("traffic", str(run))
    path = os.path.join(bench.PROFILES, "traffic_paper_1920x1024_n1024.json")
    with open(path) as f:
        rec = json.load(f)
    assert rec["fetch_factor"] == pytest.approx(0.5)
    assert rec["write_factor"] == pytest.approx(1.0)
    k = rec["kernels"]["adj_partial_kernel<1>"]
    assert k["fetch_bytes"] == pytest.approx(2000 * 1024 / 0.5)
    assert k["write_bytes"] == pytest.approx(500 * 1024)
    assert bench.measured_traffic("adj_partial_kernel<1>", path) == pytest.approx(
        2000 * 1024 / 0.5 + 500 * 1024)
    assert os.path.exists(os.path.join(bench.PROFILES, "traffic_paper_1920x1024_n1024.md"))
    # a kernel without counters is left out; a changed source withholds the figure
    assert bench.measured_traffic("adj_partial_kernel<0>", path) is None
    k["source_sha256_16"] = "0" * 16
    with open(path, "w") as f:
        json.dump(rec, f)
    assert bench.measured_traffic("adj_partial_kernel<1>", path) is None


def test_traffic_counts_read_requests_at_their_size(bench, tmp_path):
    run = tmp_path / "run"
    _counters(run / "fetch" / "f_counter_collection.csv", [(ADJ1, "FETCH_SIZE", 1000)])
    _counters(run / "write" / "w_counter_collection.csv", [(ADJ1, "WRITE_SIZE", 500)])
    _counters(run / "copy_fetch" / "c_counter_collection.csv",
              [("__amd_rocclr_copyBuffer", "FETCH_SIZE", 131072)])
    _counters(run / "copy_write" / "c_counter_collection.csv",
              [("__amd_rocclr_copyBuffer", "WRITE_SIZE", 262144)])
    # the kernel: 10 32-byte, 1000 64-byte and 3 128-byte read requests
    _counters(run / "rdreq" / "r_counter_collection.csv",
              [(ADJ1, "TCC_EA0_RDREQ_32B_sum", 10), (ADJ1, "TCC_EA0_RDREQ_64B_sum", 1000),
               (ADJ1, "TCC_EA0_RDREQ_128B_sum", 3), (ADJ1, "TCC_EA0_RDREQ_sum", 1013)])
    _counters(run / "copy_rdreq" / "c_counter_collection.csv",
              [("__amd_rocclr_copyBuffer", "TCC_EA0_RDREQ_32B_sum", 0),
               ("__amd_rocclr_copyBuffer", "TCC_EA0_RDREQ_64B_sum", 0),
               ("__amd_rocclr_copyBuffer", "TCC_EA0_RDREQ_128B_sum", 2097152),
               ("__amd_rocclr_copyBuffer", "TCC_EA0_RDREQ_sum", 2097152)])
    bench.summarize("traffic", str(run))
    path = os.path.join(bench.PROFILES, "traffic_paper_1920x1024_n1024.json")
    with open(path) as f:
        rec = json.load(f)
    assert rec["copy_read_bytes_sized"] == 268435456
    k = rec["kernels"]["adj_partial_kernel<1>"]
    assert k["read_bytes_sized"] == 10 * 32 + 1000 * 64 + 3 * 128
    sized = 10 * 32 + 1000 * 64 + 3 * 128 + 500 * 1024
    assert bench.measured_traffic("adj_partial_kernel<1>", path,
                                  key="traffic_bytes_sized") == pytest.approx(sized)
    # the copy-calibrated figure is unchanged
    assert bench.measured_traffic("adj_partial_kernel<1>", path) == pytest.approx(
        1000 * 1024 / 0.5 + 500 * 1024)
    with open(os.path.join(bench.PROFILES, "traffic_paper_1920x1024_n1024.md")) as f:
        text = f.read()
    assert "| adj_partial_kernel<1> | 10 | 1000 | 3 |" in text


def test_counter_summary_per_interaction(bench, tmp_path):
    run = tmp_path / "ctr"
    n = bench.HEADLINE_INTERACTIONS
    gui = 8 * 2.4e3 * 100  # 100 us of 8 XCDs' GRBM_GUI_ACTIVE at 2.4 GHz
    for v, kernels in bench.COUNTER_KERNELS.items():
        for i, k in enumerate(kernels):
            name = "void cgh::(anonymous namespace)::%s(float const*)" % k
            _counters(run / ("%s.1" % v) / ("k%d_counter_collection.csv" % i),
                      [(name, "SQ_INSTS_VALU", 4 * n / 64), (name, "SQ_INSTS_VALU_TRANS_F32", n / 64),
                       (name, "SQ_INSTS_SALU", n / 64), (name, "SQ_INSTS_SMEM", n / 640),
                       (name, "SQ_INSTS_LDS", 0), (name, "SQ_WAVES", 1), (name, "GRBM_GUI_ACTIVE", gui)])
            _counters(run / ("%s.2" % v) / ("k%d_counter_collection.csv" % i),
                      [(name, "SQ_ACTIVE_INST_VALU", 0.5 * 1024 * gui / 8 / 4),
                       (name, "GRBM_GUI_ACTIVE", gui)])
    g = "void cgh::(anonymous namespace)::gemm_half_kernel<2, 0>(float const*)"
    _counters(run / "separable_f16x3.1" / "x_counter_collection.csv",
              [(g, "SQ_INSTS_VALU", 300), (g, "SQ_INSTS_LDS", 100), (g, "GRBM_GUI_ACTIVE", gui)])
    _counters(run / "separable_f16x3.2" / "x_counter_collection.csv",
              [(g, "SQ_INSTS_MFMA", 100), (g, "SQ_VALU_MFMA_BUSY_CYCLES", 3200),
               (g, "GRBM_GUI_ACTIVE", gui)])
    bench.summarize("counters", str(run))
    with open(os.path.join(bench.PROFILES, "counters_paper_1920x1024_n1024.md")) as f:
        text = f.read()
    # 4 VALU (1 transcendental) per interaction against the algorithmic 3 (1):
    # 2 FP32 ops + 4 slots for the cosine = 6 slots; VALU busy 50%
    assert "| `fwd_comp_residual_kernel` | 4.00 | 1.00 | 3 (1) | 6 | 50% | 0.250 | 0.0250 | 0.0000 |" in text
    assert "| `adj_partial_kernel<2>` | 4.00 | 1.00 | 6 (2) | 12 | 50% |" in text
    assert "| 100 | 32.0 |" in text  # MFMA per dispatch, busy cycles per MFMA


def test_stats_summary_compares_trace_with_events(bench, tmp_path):
    run = tmp_path / "stats"
    run.mkdir()
    with open(run / "bench_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                    "MaxNs", "StdDev"])
        w.writerow([ADJ1, 10, 4.6e6, 460000.0, 60.0, 450000, 470000, 1.0])
    line = {"ms_per_step": 0.7, "variants": {"compensated": {"adj_kernel_ms": 0.46,
                                                             "fwd_kernel_ms": 0.25}}}
    with open(run / "bench_stdout.log", "w") as f:
        f.write("noise\n" + json.dumps(line) + "\n")
    bench.summarize("stats", str(run))
    with open(os.path.join(bench.PROFILES, "bench_paper_1920x1024_n1024_kernel_stats.md")) as f:
        text = f.read()
    assert "| adj_partial_kernel<1> | 10 | 460.0 | 450.0 | 470.0 | 60.0% |" in text
    assert "| adj_partial_kernel<1> | 460.0 | 460.0 | 1.000 |" in text
    # with an unprofiled run of the same command beside it, a second ratio
    unprof = {"ms_per_step": 0.69, "variants": {"compensated": {"adj_kernel_ms": 0.4,
                                                                "fwd_kernel_ms": 0.25}}}
    with open(run / "unprofiled.log", "w") as f:
        f.write(json.dumps(unprof) + "\n")
    bench.summarize("stats", str(run))
    with open(os.path.join(bench.PROFILES, "bench_paper_1920x1024_n1024_kernel_stats.md")) as f:
        text = f.read()
    assert "| adj_partial_kernel<1> | 460.0 | 460.0 | 1.000 | 400.0 | 1.150 |" in text
    assert "Profiled step of the headline (compensated) variant: 0.700 ms." in text
    assert "Unprofiled step of the same command: 0.690 ms." in text


def test_summarize_rejects_unknown_kind(bench):
    with pytest.raises(SystemExit):
        bench.summarize("nonsense", "/nonexistent")


def test_source_hash_ignores_comments_not_code(bench, tmp_path):
    src = "__global__ void k(float* p) {\n  p[0] = 1.0f;  // one\n}\n"
    (tmp_path / "k.hip").write_text(src)
    h = bench._sources_hash(["k.hip"], str(tmp_path))
    (tmp_path / "k.hip").write_text("/* a new\n   comment */\n" + src.replace("// one", "// uno"))
    assert bench._sources_hash(["k.hip"], str(tmp_path)) == h
    (tmp_path / "k.hip").write_text(src.replace("1.0f", "2.0f"))
    assert bench._sources_hash(["k.hip"], str(tmp_path)) != h


def test_sweep_summary_fits_a_line(bench, tmp_path):
    """Times exactly linear in N give R^2 = 1, zero residuals, and the
    intercept and slope they were made from."""
    run = tmp_path / "sweep"
    run.mkdir()
    rows = []
    for n in (512, 1024, 2048, 4096):
        rec = {"n": n, "paper_hd5850_ms": {512: 19, 1024: 31}.get(n)}
        for v, (a, b) in {"plain": (0.01, 3.8e-4), "recurrence": (0.02, 2.6e-4),
                          "compensated": (0.005, 2.3e-4)}.items():
            rec[v + "_ms"] = a + b * n
            rec[v + "_gpps"] = n * 1920 * 1024 / (rec[v + "_ms"] * 1e-3) / 1e9
        rows.append(rec)
    (run / "sweep.log").write_text("noise line\n" + json.dumps(
        {"mode": "sweep", "hologram": "1920x1024", "rows": rows}) + "\n")
    a, b, r2, worst = bench._linear_fit([r["n"] for r in rows], [r["plain_ms"] for r in rows])
    assert a == pytest.approx(0.01) and b == pytest.approx(3.8e-4)
    assert r2 == pytest.approx(1.0) and worst < 1e-12
    bench.summarize("sweep", str(run))
    text = open(os.path.join(bench.PROFILES, "sweep_1920x1024.md")).read()
    assert "| compensated | 5.0 | 230.00 | 1.000000 | 0.00% |" in text
    assert "| 512 | 19 |" in text and "| 4096 | - |" in text


def test_workload_summary_tables_and_loss_curve(bench, tmp_path):
    run = tmp_path / "wl"
    run.mkdir()
    r = {"fwd_kernel_ms": 2.0, "fwd_gpps": 8000.0, "fwd_roofline_frac": 0.61,
         "fwd_frac_of_mix": 0.83, "adj_kernel_ms": 4.0, "adj_gpps": 4000.0,
         "adj_roofline_frac": 0.6, "adj_frac_of_mix": None,
         "max_err_vs_fp64_over_sum_abs_a": 1.5e-7}
    line = {"mode": "workload", "workload": "fit4k", "description": "desc", "nx": 3840,
            "ny": 2160, "n_points": 16384, "interactions": 1, "reps": 3, "fwd_f64_ms": 90.0,
            "fwd_f64_gpps": 600.0, "compensated": r,
            "fit": {"iterations": 3, "seconds": 0.1, "iterations_per_s": 30.0, "lr": 0.01,
                    "params": "A and z/pitch", "loss_first": 4.0, "loss_last": 3.0,
                    "loss_curve": [4.0, 3.5, 3.0], "fwd_kernel_ms": 14.0, "adj_kernel_ms": 28.0,
                    "fwd_gpps": 9000.0, "adj_gpps": 4500.0,
                    "fitted_fwd_max_err_vs_fp64_over_sum_abs_a": 2e-7}}
    (run / "workload_fit4k.log").write_text(json.dumps(line) + "\n")
    bench.summarize("workloads", str(run))
    text = open(os.path.join(bench.PROFILES, "workload_fit4k_3840x2160.md")).read()
    # a missing mix fraction is derived from the rate: 4000 G/s against the
    # compensated adjoint's probe mix, 256 CUs x 2.4 GHz x 64 / 4.033 clocks
    assert 4000e9 / bench.mix_interactions("adj_compensated") == pytest.approx(0.4103, abs=1e-4)
    assert "| compensated | 2 | 8000 | 0.61 | 0.83 | 4 | 4000 | 0.60 | 0.41 | 1.50e-07 |" in text
    assert "loss 4 -> 3 (-25.0%)" in text
    assert "| 2 | 3 |" in text


def test_library_gemm_summary_matches_kernels_by_format_and_fold(bench, tmp_path):
    run = tmp_path / "lib"
    (run / "stats").mkdir(parents=True)
    with open(run / "stats" / "bench_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs",
                    "MaxNs"])
        w.writerow(["void cgh::(anonymous namespace)::gemm_half_kernel<2, 0>(unsigned short "
                    "const*)", 10, 330000, 33000.0, 1.0, 32000, 34000])
        w.writerow(["void cgh::(anonymous namespace)::gemm_f32_kernel<false, true, 2>(float "
                    "const*)", 10, 800000, 80000.0, 1.0, 79000, 81000])
    res = [{"gemm": "forward I = Y X^T", "format": "f16x3", "M": 1024, "N": 1920, "K": 2048,
            "depth": 6144, "us": 48.0, "flops": 2.0 * 1024 * 1920 * 6144, "fold": 0},
           {"gemm": "adjoint P, K = columns", "format": "f32", "M": 2048, "N": 1024,
            "K": 1920, "depth": 1920, "us": 60.0, "flops": 2.0 * 2048 * 1024 * 1920, "fold": 2},
           {"gemm": "adjoint P, K = columns", "format": "bf16", "M": 2048, "N": 1024,
            "K": 1920, "depth": 1920, "us": 20.0, "flops": 2.0 * 2048 * 1024 * 1920, "fold": 2}]
    (run / "library.log").write_text(json.dumps({"mode": "library_gemm", "torch": "x",
                                                 "results": res}) + "\n")
    bench.summarize("library", str(run))
    text = open(os.path.join(bench.PROFILES, "gemm_library_comparison_1920x1024.md")).read()
    # f16x3: 24.2 GFLOP in 48 us = 503 TFLOP/s (20.1% of 2.5 PF); ours 33 us: 732, 1.45x
    assert "| forward I = Y X^T (1024 x 1920 x 2048) | f16x3 | 48.0 | 503 | 20.1% | 33.0 | 732 " \
           "| 29.3% | 1.45x |" in text
    # FP32 against the FP32 peak; P's FP32 kernel is <false, true, 2>
    assert "| f32 | 60.0 | 134 | 85.3% | 80.0 | 101 | 64.0% | 0.75x |" in text
    # a format with no kernel in the stats run gets dashes
    assert "| bf16 | 20.0 | 403 | 16.1% | - | - | - | - |" in text


def test_committed_traffic_matches_the_headline_kernels(bench):
    """The committed counter record still describes the current sources of
    the headline step's two kernels, so the bench line carries their traffic
    (a code edit to either kernel withholds it until the counters are taken
    again)."""
    for kernel in ("adj_partial_kernel<1>", "fwd_comp_residual_kernel"):
        assert bench.measured_traffic(kernel) is not None, kernel
        assert bench.measured_traffic(kernel, key="traffic_bytes_sized") is not None, kernel


def test_more_than_one_gpu_is_refused():
    """One GPU only: --gpus above 1 exits with a message and a non-zero
    status before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU only" in r.stderr


def test_ramp_summary_against_the_steady_state(bench, tmp_path):
    run = tmp_path / "run"
    run.mkdir()
    blocks = [{"first_step": 20 * i, "fwd_ms": 0.2 if i >= 3 else 0.25,
               "adj_ms": 0.3 if i >= 3 else 0.36} for i in range(20)]
    line = {"mode": "ramp", "variant": "compensated", "steps": 400, "block": 20,
            "blocks": blocks}
    (run / "ramp.log").write_text(json.dumps(line) + "\n")
    bench.summarize("ramp", str(run))
    text = open(os.path.join(bench.PROFILES, "clock_ramp_paper_1920x1024.md")).read()
    # the steady state is the mean of the second half of the blocks
    assert "| 0-19 | 0.2500 | 1.250 | 0.3600 | 1.200 |" in text
    assert "| 380-399 | 0.2000 | 1.000 | 0.3000 | 1.000 |" in text
