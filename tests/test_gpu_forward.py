"""GPU parity of the forward kernels (cgh_forward, cgh_forward_f64) against the
FP64 CPU oracle of Eq. (1), through the C ABI.

Full grids at sizes the oracle finishes in seconds (several tiles plus ragged
tails), and sampled pixels at the full workload sizes in the launch
configuration the benchmark times.  Plus the exact invariants that hold for
the GPU arithmetic: 8-fold symmetry, power-of-two scaling in A, integer
translation (compensated) and run-to-run determinism; and every lane shape of
the recurrence forward of Eq. (2).
"""
import numpy as np
import pytest
import torch

from gpu_helpers import TOL_FWD, device, max_err_frac, say, to_dev
from paper_1002_0916_amd import binding as B
from paper_1002_0916_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["plain", "compensated", "recurrence", "separable", "separable_f16x3",
            "separable_f16", "separable_bf16"]


def run(cloud, nx, ny, variant, dev, pitch=W.PITCH, wl=W.WAVELENGTH):
    x, y, z, a = to_dev(cloud, dev)
    I = B.forward(x, y, z, a, nx, ny, pitch, wl, variant)
    torch.cuda.synchronize()
    return I.cpu().numpy()


@pytest.mark.parametrize("variant", VARIANTS)
def test_small_workload_full_grid(oracle_mod, variant):
    dev = device()
    c = W.small_cloud()
    say("small 256x256 N=64", variant)
    I = run(c, 256, 256, variant, dev)
    ref = oracle_mod.forward(*c.astuple(), 256, 256, threads=0)
    err = max_err_frac(I, ref, c)
    say("  max|dI|/sum|A| =", err)
    assert err <= TOL_FWD[variant]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", [(197, 77, 37), (64, 32, 256), (65, 33, 257), (1, 1, 1),
                                   (1, 300, 5), (300, 1, 5), (130, 70, 1)])
def test_ragged_full_grid(oracle_mod, variant, shape):
    nx, ny, n = shape
    dev = device()
    c = W.random_cloud(100 + n, n, nx, ny, zlo=0.2, zhi=1.5, alo=-1.0, ahi=1.0, margin=40)
    say("ragged", shape, variant)
    I = run(c, nx, ny, variant, dev)
    ref = oracle_mod.forward(*c.astuple(), nx, ny, threads=0)
    err = max_err_frac(I, ref, c)
    say("  max|dI|/sum|A| =", err)
    assert err <= TOL_FWD[variant]


def _rec_shape(nx, ny):
    """The recurrence forward's (pixels per lane K, rows per lane R) for an
    nx x ny hologram: the library's cost model, restated (the workgroups per
    CU times K R times the slots per interaction 4 + 1/R + (4R + 7)/(KR))."""
    best = None
    for k, r in ((8, 4), (8, 2), (8, 1), (6, 4), (6, 2), (6, 1), (4, 4), (4, 2), (4, 1)):
        wgs = -(-nx // (64 * k)) * -(-ny // (4 * r))
        t = -(-wgs // 256) * k * r * (4 + 1 / r + (4 * r + 7) / (k * r))
        if best is None or t < best[0]:
            best = (t, k, r)
    return best[1:]


# One hologram shape per recurrence lane shape (all ragged against the lane
# and workgroup tiles, except where a side is one tile or less).
REC_SHAPES = [(777, 2048), (2368, 333), (2368, 150), (3520, 333), (3392, 150), (1600, 150),
              (64, 2160), (64, 2048), (64, 1)]


def test_recurrence_shapes_cover_every_instantiation():
    assert sorted(_rec_shape(nx, ny) for nx, ny in REC_SHAPES) == sorted(
        (k, r) for k in (4, 6, 8) for r in (1, 2, 4))


@pytest.mark.parametrize("shape", REC_SHAPES, ids=lambda s: "%dx%d" % s)
def test_recurrence_every_lane_shape(oracle_mod, shape):
    """Full-grid parity of the recurrence forward for each (K, R)
    instantiation of its kernel."""
    nx, ny = shape
    n = 24
    dev = device()
    c = W.random_cloud(150 + nx % 97, n, nx, ny, zlo=0.2, zhi=1.5, alo=-1.0, ahi=1.0, margin=40)
    say("recurrence", shape, "lane shape", _rec_shape(nx, ny))
    I = run(c, nx, ny, "recurrence", dev)
    ref = oracle_mod.forward(*c.astuple(), nx, ny, threads=0)
    err = max_err_frac(I, ref, c)
    say("  max|dI|/sum|A| =", err)
    assert err <= TOL_FWD["recurrence"]


@pytest.mark.parametrize("variant", VARIANTS)
def test_empty_point_set_gives_zeros(variant):
    dev = device()
    e = torch.zeros(0, dtype=torch.float32, device=dev)
    out = torch.full((20, 30), 7.0, device=dev)
    B.forward(e, e, e, e, 30, 20, variant=variant, out=out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0


def test_empty_point_set_f64_gives_zeros():
    dev = device()
    e = torch.zeros(0, dtype=torch.float32, device=dev)
    I = B.forward_f64(e, e, e, e, 30, 20)
    torch.cuda.synchronize()
    assert torch.count_nonzero(I).item() == 0


def _sampled(oracle_mod, cloud, nx, ny, variant, dev, m, seed):
    px, py = W.sample_pixels(seed, nx, ny, m)
    say("  oracle on", px.shape[0], "sampled pixels")
    ref = oracle_mod.forward_at(*cloud.astuple(), nx, ny, px, py, threads=0)
    I = run(cloud, nx, ny, variant, dev)
    return max_err_frac(I[py, px], ref, cloud)


@pytest.mark.parametrize("variant", VARIANTS)
def test_paper_workload_sampled(oracle_mod, variant):
    dev = device()
    c = W.paper_cloud()
    say("paper 1920x1024 N=1024", variant)
    err = _sampled(oracle_mod, c, 1920, 1024, variant, dev, 4096, 31)
    say("  max|dI|/sum|A| =", err)
    assert err <= TOL_FWD[variant]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("which", [0, 1])
def test_mesh_workloads_sampled(oracle_mod, variant, which):
    dev = device()
    c = W.mesh_clouds()[which]
    say("mesh 1920x1080 N=%d" % c.n, variant)
    err = _sampled(oracle_mod, c, 1920, 1080, variant, dev, 2048 if which else 4096, 32)
    say("  max|dI|/sum|A| =", err)
    assert err <= TOL_FWD[variant]


@pytest.mark.parametrize("variant", VARIANTS)
def test_fit_workload_sampled(oracle_mod, variant):
    """3840x2160: r^2 reaches 1.94e7 > 2^24, beyond FP32-exact integers."""
    dev = device()
    _, c = W.fit_clouds()
    say("fit 3840x2160 N=16384", variant)
    err = _sampled(oracle_mod, c, 3840, 2160, variant, dev, 2048, 33)
    say("  max|dI|/sum|A| =", err)
    assert err <= TOL_FWD[variant]


def test_f64_kernel_small(oracle_mod):
    dev = device()
    c = W.random_cloud(41, 50, 97, 61, zlo=0.2, zhi=1.5, alo=-1.0, ahi=1.0, margin=1500)
    x, y, z, a = to_dev(c, dev)
    I = B.forward_f64(x, y, z, a, 97, 61).cpu().numpy()
    ref = oracle_mod.forward(*c.astuple(), 97, 61)
    err = max_err_frac(I, ref, c)
    say("f64 max|dI|/sum|A| =", err)
    assert err <= 1e-11


def test_f64_kernel_mesh_sampled(oracle_mod):
    dev = device()
    c = W.mesh_clouds()[0]
    x, y, z, a = to_dev(c, dev)
    I = B.forward_f64(x, y, z, a, 1920, 1080).cpu().numpy()
    px, py = W.sample_pixels(34, 1920, 1080, 1024)
    ref = oracle_mod.forward_at(*c.astuple(), 1920, 1080, px, py, threads=0)
    err = max_err_frac(I[py, px], ref, c)
    say("f64 mesh8k max|dI|/sum|A| =", err)
    assert err <= 1e-11


def test_f64_kernel_mesh64k_sampled(oracle_mod):
    """The FP64 GPU forward on the 65,536-point mesh cloud (the error
    reference of the FP32 variants at that workload)."""
    dev = device()
    c = W.mesh_clouds()[1]
    x, y, z, a = to_dev(c, dev)
    I = B.forward_f64(x, y, z, a, 1920, 1080).cpu().numpy()
    px, py = W.sample_pixels(35, 1920, 1080, 512)
    ref = oracle_mod.forward_at(*c.astuple(), 1920, 1080, px, py, threads=0)
    err = max_err_frac(I[py, px], ref, c)
    say("f64 mesh64k max|dI|/sum|A| =", err)
    assert err <= 1e-11


@pytest.mark.parametrize("variant", ["plain", "compensated"])
def test_eightfold_symmetry_bitwise(variant):
    """(The separable variant multiplies A into the row table, so swapping x
    and y reorders a product: equal in exact arithmetic, not bitwise.)"""
    dev = device()
    c = W.Cloud(*[np.array([v], dtype=np.float32) for v in (50.0, 60.0, 0.41, 0.9)])
    I = run(c, 101, 121, variant, dev)
    x0, y0 = 50, 60
    for u in range(0, 51):
        for v in range(0, 51):
            vals = {I[y0 + v, x0 + u], I[y0 + v, x0 - u], I[y0 - v, x0 + u], I[y0 - v, x0 - u],
                    I[y0 + u, x0 + v], I[y0 + u, x0 - v], I[y0 - u, x0 + v], I[y0 - u, x0 - v]}
            assert len(vals) == 1, (u, v, vals)


@pytest.mark.parametrize("variant", VARIANTS)
def test_power_of_two_amplitude_scaling_bitwise(variant):
    dev = device()
    c = W.random_cloud(42, 300, 200, 150, alo=-1.0, ahi=1.0, margin=20)
    c4 = W.Cloud(c.x, c.y, c.z, (c.a * 4).astype(np.float32))
    assert np.array_equal(run(c4, 200, 150, variant, dev), 4 * run(c, 200, 150, variant, dev))


@pytest.mark.parametrize("variant", [v for v in VARIANTS if v != "recurrence"])
def test_integer_translation_bitwise(variant):
    """Shifting points and grid by whole tiles reproduces the hologram bitwise.
    (Not the recurrence: a pixel's rounding depends on its offset from the
    first pixel of its lane's run, which the shift and the per-shape run
    length can change; its translated results are covered to its bar by the
    parity tests.)"""
    dev = device()
    c = W.random_cloud(43, 100, 160, 96, margin=10)
    # coordinates on a 1/1024 grid so that the integer shift is exact in FP32
    c = W.Cloud((np.round(c.x * 1024) / 1024).astype(np.float32),
                (np.round(c.y * 1024) / 1024).astype(np.float32), c.z, c.a)
    s, t = 64, 32  # whole forward tiles, so the rows/columns map to the same lanes
    cs = W.Cloud((c.x + s).astype(np.float32), (c.y + t).astype(np.float32), c.z, c.a)
    assert np.array_equal(cs.x - s, c.x) and np.array_equal(cs.y - t, c.y)
    I = run(c, 160, 96, variant, dev)
    J = run(cs, 160 + s, 96 + t, variant, dev)
    assert np.array_equal(J[t:, s:], I)


@pytest.mark.parametrize("variant", VARIANTS)
def test_run_to_run_deterministic(variant):
    dev = device()
    c = W.paper_cloud(n=300)
    assert np.array_equal(run(c, 777, 333, variant, dev), run(c, 777, 333, variant, dev))


def test_kernel_profiling_counts_launches():
    dev = device()
    c = W.small_cloud()
    x, y, z, a = to_dev(c, dev)
    B.profile_enable(True)
    try:
        for _ in range(3):
            B.forward(x, y, z, a, 256, 256, variant="compensated")
    finally:
        B.profile_enable(False)
    n, ms = B.profile_read(B.KERNEL_FWD_COMPENSATED)
    assert n == 3 and ms > 0
    assert B.profile_read(B.KERNEL_FWD_COMPENSATED) == (0, 0.0)
    # per-launch durations: one per launch, summing to the total
    B.profile_enable(True)
    try:
        for _ in range(4):
            B.forward(x, y, z, a, 256, 256, variant="separable_f16x3")
    finally:
        B.profile_enable(False)
    each = B.profile_read_each(B.KERNEL_FWD_SEPARABLE)
    assert len(each) == 4 and all(v > 0 for v in each)
    assert B.profile_read(B.KERNEL_FWD_SEPARABLE) == (0, 0.0)


def test_separable_symmetry_to_rounding():
    dev = device()
    c = W.Cloud(*[np.array([v], dtype=np.float32) for v in (50.0, 60.0, 0.41, 0.9)])
    I = run(c, 101, 121, "separable", dev)
    x0, y0 = 50, 60
    for u in range(0, 51):
        for v in range(0, 51):
            vals = np.array([I[y0 + v, x0 + u], I[y0 + v, x0 - u], I[y0 - v, x0 + u],
                             I[y0 - v, x0 - u], I[y0 + u, x0 + v], I[y0 + u, x0 - v],
                             I[y0 - u, x0 + v], I[y0 - u, x0 - v]])
            assert np.ptp(vals) <= 4e-7, (u, v, vals)


HALF = ["separable_f16x3", "separable_f16", "separable_bf16"]


@pytest.mark.parametrize("variant", HALF)
@pytest.mark.parametrize("scale", [1e6, 1e-6])
def test_half_variants_amplitude_range(oracle_mod, variant, scale):
    """Amplitudes far outside the fp16 range (1e6) or deep in its subnormals
    (1e-6): the power-of-two operand scaling keeps the error at the bar."""
    dev = device()
    c = W.random_cloud(44, 200, 150, 110, alo=-1.0, ahi=1.0, margin=15)
    c = W.Cloud(c.x, c.y, c.z, (c.a * scale).astype(np.float32))
    I = run(c, 150, 110, variant, dev)
    ref = oracle_mod.forward(*c.astuple(), 150, 110, threads=0)
    err = max_err_frac(I, ref, c)
    say(variant, "scale", scale, "max|dI|/sum|A| =", err)
    assert np.all(np.isfinite(I))
    assert err <= TOL_FWD[variant]
