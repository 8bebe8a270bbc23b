"""GPU parity at the limits of the C ABI, for every variant, forward and
adjoint: the largest point count (n = 4,000,000), a side of 1,048,576 pixels
(wide and tall), and a hologram of more than 2^31 pixels, where every pixel
offset needs 64-bit arithmetic.

On the 2^20-pixel sides and the > 2^31-pixel grid, pitch and wavelength are
chosen so that the phase spans a few revolutions over the whole hologram: the
FP32 variants need |phase| well inside FP32 range to meet their bars, which
the paper's optics (1e5 revolutions at 65536 pixels) would exceed.  The
workloads still run every index path at its full size.

For the > 2^31-pixel adjoint the oracle cannot sweep 2.15e9 pixels.  G is
zero except on a 64 x 64 window in the far corner, and the expected gradients
are the oracle's on that window with the points moved by the same whole
pixels: the phase depends only on pixel-minus-point differences, which the
move leaves exact (points on a 1/64-pixel grid, < 2^17 pixels from the
origin, so the shifted FP32 coordinates are exact).
"""
import gc

import numpy as np
import pytest
import torch

from gpu_helpers import TOL_ADJ, TOL_FWD, device, max_err_frac, rel_l2, say, to_dev
from paper_1002_0916_amd import binding as B
from paper_1002_0916_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["plain", "compensated", "recurrence", "separable", "separable_f16x3",
            "separable_f16", "separable_bf16"]
GROUPS = ("x", "y", "z", "a")


@pytest.fixture(autouse=True)
def _release():
    yield
    B.release_workspaces()
    gc.collect()
    torch.cuda.empty_cache()


def _gather(I, px, py, nx, dev):
    idx = torch.from_numpy(py.astype(np.int64) * nx + px.astype(np.int64)).to(dev)
    return I.reshape(-1)[idx].double().cpu().numpy()


def _check_forward(oracle_mod, cloud, nx, ny, variant, pitch, wl, px, py, dev, f64=False):
    x, y, z, a = to_dev(cloud, dev)
    ref = oracle_mod.forward_at(*cloud.astuple(), nx, ny, px, py, pitch, wl, threads=0)
    I = B.forward(x, y, z, a, nx, ny, pitch, wl, variant)
    torch.cuda.synchronize()
    err = max_err_frac(_gather(I, px, py, nx, dev), ref, cloud)
    del I
    say("  forward %s max|dI|/sum|A| = %.3e" % (variant, err))
    assert err <= TOL_FWD[variant]
    if f64:
        I64 = B.forward_f64(x, y, z, a, nx, ny, pitch, wl)
        e64 = max_err_frac(_gather(I64, px, py, nx, dev), ref, cloud)
        del I64
        say("  forward f64 max|dI|/sum|A| = %.3e" % e64)
        assert e64 <= 1e-11


def _compare_grads(gg, ref, variant):
    for name, g, r in zip(GROUPS, gg, ref):
        e = rel_l2(g, r)
        say("  adjoint %s d%s rel-L2 = %.3e" % (variant, name, e))
        assert np.all(np.isfinite(g))
        assert e <= TOL_ADJ[variant], (name, e)


@pytest.mark.parametrize("variant", VARIANTS)
def test_four_million_points(oracle_mod, variant):
    """n = 4,000,000 (the largest accepted): 62,500 point groups in the adjoint
    grid, 8e6-long contractions in the separable form."""
    nx, ny, n = 64, 16, 4_000_000
    dev = device()
    say("limits: n = %d on %dx%d, %s" % (n, nx, ny, variant))
    c = W.random_cloud(401, n, nx, ny, zlo=0.2, zhi=1.0, alo=-1.0, ahi=1.0, margin=30)
    px, py = W.sample_pixels(402, nx, ny, 60)
    _check_forward(oracle_mod, c, nx, ny, variant, W.PITCH, W.WAVELENGTH, px, py, dev,
                   f64=variant == "compensated")
    rng = np.random.default_rng(403)
    G = rng.standard_normal((ny, nx)).astype(np.float32)
    idx = np.sort(rng.choice(n, size=48, replace=False))
    x, y, z, a = to_dev(c, dev)
    g = torch.from_numpy(G).to(dev)
    gg = [t[torch.from_numpy(idx).to(dev)].cpu().numpy()
          for t in B.backward(x, y, z, a, g, nx, ny, variant=variant)]
    ref = oracle_mod.adjoint(*c.astuple(), nx, ny, G, idx=idx, threads=0)
    _compare_grads(gg, ref, variant)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", [(1 << 20, 2), (2, 1 << 20)], ids=["wide", "tall"])
def test_longest_side(oracle_mod, variant, shape):
    """A side of 2^20 pixels (the largest accepted), wide and tall."""
    nx, ny = shape
    pitch, wl = 1e-7, 1e-3  # Prev = p^2 / (2 lambda z) ~ 5e-12 rev/px^2
    dev = device()
    say("limits: %dx%d, %s" % (nx, ny, variant))
    c = W.random_cloud(410 + nx % 7, 64, nx, ny, zlo=0.5, zhi=1.0, alo=-1.0, ahi=1.0)
    px, py = W.sample_pixels(411, nx, ny, 2048)
    _check_forward(oracle_mod, c, nx, ny, variant, pitch, wl, px, py, dev,
                   f64=variant == "compensated")
    rng = np.random.default_rng(412)
    G = rng.standard_normal((ny, nx)).astype(np.float32)
    x, y, z, a = to_dev(c, dev)
    g = torch.from_numpy(G).to(dev)
    gg = [t.cpu().numpy() for t in B.backward(x, y, z, a, g, nx, ny, pitch, wl, variant)]
    idx = np.arange(0, 64, 4)
    ref = oracle_mod.adjoint(*c.astuple(), nx, ny, G, idx=idx, pitch=pitch, wavelength=wl,
                             threads=0)
    _compare_grads([v[idx] for v in gg], ref, variant)


def test_compensated_adjoint_without_row_table(oracle_mod):
    """4096 rows x 16448 points: the compensated adjoint's row table would take
    more than its 512 MiB bound, so the kernel forms the row phases itself
    (the inline form of the same arithmetic).  The points stay inside the
    grid, within the 4096 pixels of exact-grid arithmetic of every pixel."""
    nx, ny, n = 32, 4096, 16448
    assert ny * n * 8 > 512 << 20
    assert (B.workspace_bytes(n, nx, ny, "compensated", B.OP_BACKWARD)
            == B.workspace_bytes(n, nx, ny, "plain", B.OP_BACKWARD))
    dev = device()
    say("limits: compensated adjoint without the row table, %dx%d, n = %d" % (nx, ny, n))
    c = W.random_cloud(430, n, nx, ny, zlo=0.5, zhi=1.0, alo=-1.0, ahi=1.0)
    rng = np.random.default_rng(431)
    G = rng.standard_normal((ny, nx)).astype(np.float32)
    idx = np.sort(rng.choice(n, size=24, replace=False))
    x, y, z, a = to_dev(c, dev)
    g = torch.from_numpy(G).to(dev)
    gg = [t[torch.from_numpy(idx).to(dev)].cpu().numpy()
          for t in B.backward(x, y, z, a, g, nx, ny, variant="compensated")]
    ref = oracle_mod.adjoint(*c.astuple(), nx, ny, G, idx=idx, threads=0)
    _compare_grads(gg, ref, "compensated")


@pytest.mark.parametrize("variant", VARIANTS)
def test_more_than_2_31_pixels(oracle_mod, variant):
    """65536 x 32769 = 2,147,549,184 pixels (> 2^31): forward on sampled
    pixels including the last ones, adjoint with G supported on the far-corner
    window."""
    nx, ny, n = 65536, 32769, 64
    assert nx * ny > 2 ** 31
    pitch, wl = 1e-6, 1e-3  # Prev ~ 1e-9 rev/px^2: a few revolutions across the grid
    dev = device()
    say("limits: %dx%d (%d pixels), %s" % (nx, ny, nx * ny, variant))
    c = W.random_cloud(420, n, nx, ny, zlo=0.4, zhi=0.6, alo=-1.0, ahi=1.0)
    c = W.Cloud((np.round(c.x * 64) / 64).astype(np.float32),
                (np.round(c.y * 64) / 64).astype(np.float32), c.z, c.a)
    px, py = W.sample_pixels(421, nx, ny, 4096)
    _check_forward(oracle_mod, c, nx, ny, variant, pitch, wl, px, py, dev)

    X0, Y0, w = nx - 64, ny - 64, 64
    rng = np.random.default_rng(422)
    Gw = rng.standard_normal((w, w)).astype(np.float32)
    x, y, z, a = to_dev(c, dev)
    g = torch.zeros((ny, nx), dtype=torch.float32, device=dev)
    g[Y0:, X0:] = torch.from_numpy(Gw).to(dev)
    gg = [t.cpu().numpy() for t in B.backward(x, y, z, a, g, nx, ny, pitch, wl, variant)]
    del g
    shifted = W.Cloud((c.x - X0).astype(np.float32), (c.y - Y0).astype(np.float32), c.z, c.a)
    assert np.array_equal(shifted.x.astype(np.float64), c.x.astype(np.float64) - X0)
    assert np.array_equal(shifted.y.astype(np.float64), c.y.astype(np.float64) - Y0)
    ref = oracle_mod.adjoint(*shifted.astuple(), w, w, Gw, pitch=pitch, wavelength=wl,
                             threads=0)
    _compare_grads(gg, ref, variant)
