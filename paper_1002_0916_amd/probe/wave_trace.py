"""Wave trace of the compensated adjoint kernel (a diagnostic, not part of the
library): when each wave starts and ends, on which XCD, CU and SIMD it runs,
and at what shader clock.

The library is built a second time with -DCGH_WAVE_TRACE (paper_1002_0916_amd
/probe/libcgh_trace.so): the kernel then records, per wave of its last launch,
the 100 MHz constant clock (s_memrealtime) at its start and end, its hardware
ids and the shader-clock cycles (s_memtime) in between.  The traced build
holds one more VGPR than the library's (the same 3 waves per SIMD).  Each
workload's adjoint first runs for WARM_S seconds, so the traced launch sees
the settled clock: from a cold start the clock takes tens of milliseconds of
load to ramp up, and a launch traced right after start-up runs about 15%
slower.

  python paper_1002_0916_amd/probe/wave_trace.py build          (before the run)
  python paper_1002_0916_amd/probe/wave_trace.py run <out>      (on the MI355X)
  python paper_1002_0916_amd/probe/wave_trace.py summarize <out>
"""
import ctypes
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
LIB = os.path.join(HERE, "libcgh_trace.so")
SUMMARY = os.path.join(ROOT, "profiles", "adjoint_wave_trace.md")
# (workload, cloud): the headline shape and two larger ones; G is a seeded
# standard normal grid.
CASES = (("paper", "paper"), ("mesh8k", "mesh8k"), ("fit4k", "fit4k"))
MAX_WAVES = 65536
WARM_S = 0.15


def build():
    from paper_1002_0916_amd import build as B
    B.build_variant(LIB, ["CGH_WAVE_TRACE"], verbose=True)


def _cloud(W, name):
    if name == "paper":
        return W.paper_cloud()
    if name == "mesh8k":
        return W.mesh_clouds()[0]
    return W.fit_clouds()[1]


def run(out):
    import numpy as np
    import torch
    from paper_1002_0916_amd import binding as B
    from paper_1002_0916_amd import workloads as W

    if not os.path.exists(LIB):
        raise SystemExit("missing %s: run `wave_trace.py build` first" % LIB)
    B.LIB_PATH = LIB
    lib = B.load_library()
    lib.cgh_wave_trace_read.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    lib.cgh_wave_trace_read.restype = ctypes.c_int
    os.makedirs(out, exist_ok=True)
    dev = torch.device("cuda:0")
    meta = []
    for wl_name, cloud_name in CASES:
        wl = W.WORKLOADS[wl_name]
        print("trace", wl_name, wl.nx, wl.ny, wl.n, flush=True)
        c = _cloud(W, cloud_name)
        x, y, z, a = (torch.from_numpy(v).to(dev) for v in c.astuple())
        G = torch.from_numpy(np.random.default_rng(3).standard_normal((wl.ny, wl.nx))
                             .astype(np.float32)).to(dev)
        import time
        t0, k = time.perf_counter(), 0
        while k < 5 or time.perf_counter() - t0 < WARM_S:
            for _ in range(5):  # enqueued back to back, then one wait
                B.backward(x, y, z, a, G, wl.nx, wl.ny, wl.pitch, wl.wavelength, "compensated")
            torch.cuda.synchronize()
            k += 5
        B.profile_read(B.KERNEL_ADJ_COMPENSATED)
        B.profile_enable(True)
        B.backward(x, y, z, a, G, wl.nx, wl.ny, wl.pitch, wl.wavelength, "compensated")
        torch.cuda.synchronize()
        B.profile_enable(False)
        kernel_ms = float(B.profile_read_each(B.KERNEL_ADJ_COMPENSATED)[-1])
        buf = np.zeros((MAX_WAVES, 4), dtype=np.uint64)
        if lib.cgh_wave_trace_read(buf.ctypes.data, buf.nbytes) != 0:
            raise SystemExit("cgh_wave_trace_read failed")
        np.save(os.path.join(out, "trace_%s.npy" % wl_name), buf)
        meta.append({"workload": wl_name, "nx": wl.nx, "ny": wl.ny, "n": wl.n,
                     "kernel_ms": kernel_ms})
    with open(os.path.join(out, "meta.json"), "w") as f:
        json.dump(meta, f)
    print("done", flush=True)


def _analyse(buf, kernel_ms):
    import numpy as np

    st, en = buf[:, 0].astype(np.int64), buf[:, 1].astype(np.int64)
    used = st > 0
    # the last launch only: waves that start within twice the kernel time of
    # the latest end (earlier launches left entries that the last one did not
    # overwrite only where it had fewer waves)
    last = en[used].max()
    used &= st > last - int(2 * kernel_ms * 1e5)
    st, en, hw, cyc = st[used], en[used], buf[used, 2], buf[used, 3].astype(np.int64)
    t0 = st.min()
    s_us, e_us = (st - t0) / 100.0, (en - t0) / 100.0
    hwid = (hw & 0xFFFFFFFF).astype(np.int64)
    xcc = (hw >> np.uint64(32)).astype(np.int64) & 0xF
    simd = (hwid >> 4) & 3
    cu = (hwid >> 8) & 15
    sh = (hwid >> 12) & 1
    se = (hwid >> 13) & 7
    key = (((xcc * 8 + se) * 2 + sh) * 16 + cu) * 4 + simd
    simds, inv = np.unique(key, return_inverse=True)
    span = float(e_us.max())
    per = np.bincount(inv)
    last_end = np.zeros(simds.size)
    np.maximum.at(last_end, inv, e_us)
    grid = np.linspace(0.0, span, 401)[:-1] + span / 800
    live = np.array([np.bincount(inv[(s_us <= t) & (e_us > t)], minlength=simds.size)
                     for t in grid])
    clk = cyc / ((en - st) / 100e6) / 1e9
    x_med_clk = {int(x): float(np.median(clk[xcc == x])) for x in np.unique(xcc)}
    x_last = {}
    for x in np.unique(xcc):
        m = np.isin(simds, np.unique(key[xcc == x]))
        x_last[int(x)] = float(np.median(last_end[m]))
    pct = lambda v, q: [round(float(u), 1) for u in np.percentile(v, q)]
    return {
        "waves": int(used.sum()), "simds": int(simds.size), "span_us": round(span, 1),
        "waves_per_simd": [int(per.min()), int(per.max())],
        "wave_us_pct_0_10_50_90_100": pct(e_us - s_us, [0, 10, 50, 90, 100]),
        "live_mean": round(float(live.mean()), 2),
        "live_by_tenth": [round(float(live[i * 40:(i + 1) * 40].mean()), 2) for i in range(10)],
        "simds_by_live_at_90pct": np.bincount(live[360], minlength=4).tolist(),
        "simd_last_end_pct_0_10_50_90_100": pct(last_end, [0, 10, 50, 90, 100]),
        "clock_ghz_pct_0_10_50_90_100": [round(float(u), 3) for u in
                                         np.percentile(clk, [0, 10, 50, 90, 100])],
        "xcd_median_clock_ghz": x_med_clk,
        "xcd_median_simd_last_end_us": {k: round(v, 1) for k, v in x_last.items()},
    }


def summarize(out):
    import numpy as np

    with open(os.path.join(out, "meta.json")) as f:
        meta = json.load(f)
    lines = [
        "# Wave trace of the compensated adjoint kernel",
        "",
        "Commands (from the repository root; the build here, the run on an MI355X machine):",
        "",
        "```",
        "python paper_1002_0916_amd/probe/wave_trace.py build",
        "timeout -k 10 300 python paper_1002_0916_amd/probe/wave_trace.py run <out>",
        "python paper_1002_0916_amd/probe/wave_trace.py summarize <out>",
        "```",
        "",
        ("The library built with -DCGH_WAVE_TRACE records, per wave of the last adjoint launch, "
         "the 100 MHz constant clock at its start and end, its XCD, CU and SIMD, and the "
         "shader-clock cycles in between (clock = cycles / elapsed time).  Each workload's cloud, "
         "G a seeded standard normal grid; %.2f s of back-to-back launches (the clock settles), "
         "then the traced one.  Live waves: waves resident on a SIMD, sampled at 400 instants of "
         "the span (the kernel holds at most 3 per SIMD)." % WARM_S),
        "",
    ]
    for m in meta:
        buf = np.load(os.path.join(out, "trace_%s.npy" % m["workload"]))
        r = _analyse(buf, m["kernel_ms"])
        lines += [
            "## %s: %dx%d, N = %d" % (m["workload"], m["nx"], m["ny"], m["n"]), "",
            "| quantity | value |", "|---|---|",
            "| kernel (HIP events) | %.1f us |" % (1e3 * m["kernel_ms"]),
            "| waves, SIMDs | %d, %d |" % (r["waves"], r["simds"]),
            "| waves per SIMD (min, max) | %d, %d |" % tuple(r["waves_per_simd"]),
            "| span of the trace | %.1f us |" % r["span_us"],
            "| wave duration, us (0/10/50/90/100 %%) | %s |" % r["wave_us_pct_0_10_50_90_100"],
            "| live waves per SIMD, time mean | %.2f |" % r["live_mean"],
            "| live waves per SIMD, mean by tenth of the span | %s |" % r["live_by_tenth"],
            "| SIMDs holding 0/1/2/3 waves at 90%% of the span | %s |"
            % r["simds_by_live_at_90pct"],
            "| a SIMD's last wave ends, us (0/10/50/90/100 %%) | %s |"
            % r["simd_last_end_pct_0_10_50_90_100"],
            "| shader clock per wave, GHz (0/10/50/90/100 %%) | %s |"
            % r["clock_ghz_pct_0_10_50_90_100"],
            "| median clock by XCD, GHz | %s |" % ", ".join(
                "%d: %.3f" % (k, v) for k, v in sorted(r["xcd_median_clock_ghz"].items())),
            "| median SIMD end by XCD, us | %s |" % ", ".join(
                "%d: %.1f" % (k, v) for k, v in sorted(r["xcd_median_simd_last_end_us"].items())),
            "",
        ]
    with open(SUMMARY, "w") as f:
        f.write("\n".join(lines))
    print("wrote", SUMMARY)


if __name__ == "__main__":
    if len(sys.argv) < 2 or sys.argv[1] not in ("build", "run", "summarize"):
        raise SystemExit(__doc__)
    if sys.argv[1] == "build":
        build()
    elif len(sys.argv) < 3:
        raise SystemExit(__doc__)
    elif sys.argv[1] == "run":
        run(sys.argv[2])
    else:
        summarize(sys.argv[2])
