"""cgh_forward_residual on the GPU: the hologram it writes is cgh_forward's,
bit for bit, and the residual is I - T with one FP32 subtraction per pixel
(the compensated forward computes it in its own store pass, the others in a
second kernel).  The hologram itself is parity-tested against the oracle in
test_gpu_forward.py."""
import numpy as np
import pytest
import torch

from gpu_helpers import device, say, to_dev
from paper_1002_0916_amd import binding as B
from paper_1002_0916_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["plain", "compensated", "recurrence", "separable", "separable_f16x3",
            "separable_f16", "separable_bf16"]


def _target(nx, ny, seed, dev):
    t = np.random.default_rng(seed).standard_normal((ny, nx)).astype(np.float32)
    return torch.from_numpy(t).to(dev)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", [(100, 75, 130), (64, 33, 7)])
def test_residual_matches_forward_minus_target(variant, shape):
    nx, ny, n = shape
    dev = device()
    say("residual", shape, variant)
    c = W.random_cloud(900 + n, n, nx, ny, zlo=0.2, zhi=1.0, alo=-1.0, ahi=1.0, margin=30)
    x, y, z, a = to_dev(c, dev)
    T = _target(nx, ny, 901 + n, dev)
    I, G = B.forward_residual(x, y, z, a, T, nx, ny, variant=variant)
    ref = B.forward(x, y, z, a, nx, ny, variant=variant)
    torch.cuda.synchronize()
    assert torch.equal(I, ref)
    assert torch.equal(G, ref - T)


def test_residual_at_the_headline_shape():
    wl = W.WORKLOADS["paper"]
    dev = device()
    say("residual at the headline shape")
    x, y, z, a = to_dev(W.paper_cloud(), dev)
    T = _target(wl.nx, wl.ny, 905, dev)
    I = torch.empty((wl.ny, wl.nx), dtype=torch.float32, device=dev)
    G = torch.empty_like(I)
    B.forward_residual(x, y, z, a, T, wl.nx, wl.ny, wl.pitch, wl.wavelength, "compensated",
                       out=I, residual=G)
    ref = B.forward(x, y, z, a, wl.nx, wl.ny, wl.pitch, wl.wavelength, "compensated")
    torch.cuda.synchronize()
    assert torch.equal(I, ref)
    assert torch.equal(G, ref - T)


def test_residual_of_no_points():
    dev = device()
    e = torch.empty(0, dtype=torch.float32, device=dev)
    T = _target(40, 30, 906, dev)
    I, G = B.forward_residual(e, e, e, e, T, 40, 30, variant="compensated")
    torch.cuda.synchronize()
    assert torch.count_nonzero(I).item() == 0
    assert torch.equal(G, -T)


def test_residual_without_the_column_table():
    """4096 columns and 16448 points: the forward's column table would take
    4096 x 16448 x 4 B = 269.5 MB, above its 256 MiB bound, so the forward
    forms the x-phases itself (the inline kernels).  The residual instance of
    that kernel writes the same I as the one without a target."""
    nx, ny, n = 4096, 4, 16448
    assert nx * n * 4 > 256 << 20
    dev = device()
    say("residual, inline x-phases", (nx, ny, n))
    c = W.random_cloud(907, n, nx, ny, zlo=0.2, zhi=1.0, alo=-1.0, ahi=1.0, margin=30)
    x, y, z, a = to_dev(c, dev)
    T = _target(nx, ny, 908, dev)
    I, G = B.forward_residual(x, y, z, a, T, nx, ny, variant="compensated")
    ref = B.forward(x, y, z, a, nx, ny, variant="compensated")
    torch.cuda.synchronize()
    assert torch.equal(I, ref)
    assert torch.equal(G, ref - T)
