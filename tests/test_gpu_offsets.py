"""GPU parity at large pixel offsets with the paper's optics (pitch 8 um,
633 nm, z in [0.2, 0.4] m), through the C ABI.

The compensated axis phase forms the square of the grid offset
m = x_h - rint(x_j) as an exact FP32 pair, so its accuracy does not end at
|m| = 4096 (where m^2 leaves FP32's exact integers).  Long thin holograms
(8192 and 16384 pixels along one axis) with points up to 3000 px outside the
aperture put |m| past 11,000 and 19,000, where the phase reaches 3e4 to 1e5
revolutions; every variant built on the compensated axis phase (compensated,
and the separable forms whose per-axis tables use it) must still meet its
bar against the FP64 oracle, forward (full grid, element by element) and
adjoint (all points).  A 2^20-pixel side checks the stated error bound of
the axis phase where it is no longer small.
"""
import math

import numpy as np
import pytest
import torch

from gpu_helpers import TOL_ADJ, TOL_FWD, device, max_err_frac, rel_l2, say, to_dev
from paper_1002_0916_amd import binding as B
from paper_1002_0916_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["compensated", "separable", "separable_f16x3", "separable_f16", "separable_bf16"]
# (nx, ny, n): long sides of 8192 and 16384 pixels in x and in y.
SHAPES = [(8192, 64, 96), (64, 8192, 96), (16384, 16, 64), (16, 16384, 64)]
MARGIN = 3000.0


def cloud_for(nx, ny, n, seed):
    return W.random_cloud(seed, n, nx, ny, zlo=0.2, zhi=0.4, alo=-1.0, ahi=1.0, margin=MARGIN)


def _max_offset(c, nx, ny):
    mx = np.maximum(np.abs(np.rint(c.x)), np.abs(nx - 1 - np.rint(c.x)))
    my = np.maximum(np.abs(np.rint(c.y)), np.abs(ny - 1 - np.rint(c.y)))
    return int(max(mx.max(), my.max()))


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "%dx%d" % s[:2])
def test_forward_large_offsets_full_grid(oracle_mod, variant, shape):
    nx, ny, n = shape
    dev = device()
    c = cloud_for(nx, ny, n, 600 + nx % 1000)
    say("offsets forward", shape, variant, "max |m| =", _max_offset(c, nx, ny))
    x, y, z, a = to_dev(c, dev)
    I = B.forward(x, y, z, a, nx, ny, variant=variant)
    torch.cuda.synchronize()
    ref = oracle_mod.forward(*c.astuple(), nx, ny, threads=0)
    err = max_err_frac(I.cpu().numpy(), ref, c)
    say("  max|dI|/sum|A| =", err)
    assert err <= TOL_FWD[variant]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", SHAPES[:2], ids=lambda s: "%dx%d" % s[:2])
def test_adjoint_large_offsets_all_points(oracle_mod, variant, shape):
    nx, ny, n = shape
    dev = device()
    c = cloud_for(nx, ny, n, 700 + nx % 1000)
    # Upstream gradient: a hologram of points inside the aperture plus noise.
    h = W.random_cloud(701, 6, nx, ny, zlo=0.3, zhi=0.8, alo=0.5, ahi=1.0)
    G = (oracle_mod.forward(*h.astuple(), nx, ny, threads=0)
         + 0.5 * np.random.default_rng(702).standard_normal((ny, nx))).astype(np.float32)
    say("offsets adjoint", shape, variant, "max |m| =", _max_offset(c, nx, ny))
    x, y, z, a = to_dev(c, dev)
    gg = B.backward(x, y, z, a, torch.from_numpy(G).to(dev), nx, ny, variant=variant)
    torch.cuda.synchronize()
    ref = oracle_mod.adjoint(*c.astuple(), nx, ny, G, threads=0)
    for name, g, r in zip("xyza", gg, ref):
        e = rel_l2(g.cpu().numpy(), r)
        say("  d%s rel-L2 = %.3e" % (name, e))
        assert e <= TOL_ADJ[variant], (name, e)


def axis_phase_bound(m, prev):
    """The stated per-axis error bound of the compensated axis phase, in
    revolutions: 2^-24 (1 + 1.5 Prev |m|) + 2^-46 Prev m^2."""
    return 2.0 ** -24 * (1 + 1.5 * prev * m) + 2.0 ** -46 * prev * m * m


@pytest.mark.parametrize("variant", ["compensated", "separable"])
def test_side_2_20_paper_optics_within_stated_bound(oracle_mod, variant):
    """A 1,048,576 x 2 hologram at the paper's optics: |m| reaches 2^20 and
    the phase 3e8 revolutions.  The forward must stay within the error the
    axis-phase bound allows, summed over the points (each term's cosine moves
    by at most 2 pi times its phase error), plus the compensated bar for the
    cosine and the accumulation; and the cosine's argument must stay in range
    (finite, bounded results everywhere)."""
    nx, ny, n = 1 << 20, 2, 12
    dev = device()
    c = W.random_cloud(710, n, nx, ny, zlo=0.2, zhi=0.4, alo=-1.0, ahi=1.0)
    prev = W.PITCH ** 2 / (2 * W.WAVELENGTH * c.z.astype(np.float64))
    mx = np.maximum(np.abs(np.rint(c.x)), np.abs(nx - 1 - np.rint(c.x)))
    my = np.maximum(np.abs(np.rint(c.y)), np.abs(ny - 1 - np.rint(c.y)))
    per_term = 2 * math.pi * (axis_phase_bound(mx, prev) + axis_phase_bound(my, prev))
    suma = float(np.sum(np.abs(c.a.astype(np.float64))))
    bar = float(np.sum(np.abs(c.a) * per_term)) / suma + TOL_FWD["compensated"]
    x, y, z, a = to_dev(c, dev)
    I = B.forward(x, y, z, a, nx, ny, variant=variant).cpu().numpy()
    assert np.all(np.isfinite(I)) and np.max(np.abs(I)) <= suma * (1 + 1e-6)
    px, py = W.sample_pixels(711, nx, ny, 4096)
    ref = oracle_mod.forward_at(*c.astuple(), nx, ny, px, py, threads=0)
    err = max_err_frac(I[py, px], ref, c)
    say("2^20 side", variant, "max|dI|/sum|A| =", err, "bar", bar)
    assert err <= bar
