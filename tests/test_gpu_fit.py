"""GPU tests of the fitting driver (Adam on A and z/p through CGHFunction)."""
import numpy as np
import pytest
import torch

from gpu_helpers import device, say, to_dev
from paper_1002_0916_amd import binding as B
from paper_1002_0916_amd import fit as F
from paper_1002_0916_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("variant", ["compensated", "plain", "separable_f16x3"])
def test_fit_reduces_loss(variant):
    dev = device()
    nx, ny = 160, 120
    hidden = W.random_cloud(61, 80, nx, ny, zlo=0.3, zhi=0.6, alo=0.5, ahi=1.0)
    rng = np.random.default_rng(62)
    start = W.Cloud(hidden.x, hidden.y,
                    (hidden.z + rng.normal(0, 2e-6, hidden.n)).astype(np.float32),
                    (hidden.a + rng.normal(0, 0.1, hidden.n)).astype(np.float32))
    hx, hy, hz, ha = to_dev(hidden, dev)
    T = B.forward_f64(hx, hy, hz, ha, nx, ny).float()
    x, y, z, a = to_dev(start, dev)
    res = F.fit(x, y, z, a, T, nx, ny, iters=60, lr=1e-2, variant=variant)
    say(variant, "loss", res.losses[0], "->", res.losses[-1], "it/s", res.iterations_per_s)
    assert len(res.losses) == 60
    assert all(np.isfinite(res.losses))
    assert res.losses[-1] < 0.2 * res.losses[0]
    # A moved towards the hidden amplitudes
    da0 = np.abs(start.a - hidden.a).mean()
    da1 = np.abs(res.a.cpu().numpy() - hidden.a).mean()
    assert da1 < 0.5 * da0


def test_fit_is_deterministic():
    dev = device()
    nx, ny = 96, 64
    hidden = W.random_cloud(63, 40, nx, ny)
    start = W.perturb(hidden, 64, sxy=0.0, sz=1e-6, sa=0.1)
    hx, hy, hz, ha = to_dev(hidden, dev)
    T = B.forward_f64(hx, hy, hz, ha, nx, ny).float()
    x, y, z, a = to_dev(start, dev)
    r1 = F.fit(x, y, z, a, T, nx, ny, iters=10, time_kernels=False)
    r2 = F.fit(x, y, z, a, T, nx, ny, iters=10, time_kernels=False)
    assert r1.losses == r2.losses
    assert torch.equal(r1.a, r2.a) and torch.equal(r1.z, r2.z)
