"""GPU parity of the adjoint (cgh_backward) against the FP64 CPU oracle's
chain-rule adjoint, with the same upstream gradient G on both sides.

Full point sets at small sizes (several pixel blocks plus ragged tails), and
sampled points at the full workload sizes in the launch configuration the
benchmark times.  Also: autograd wiring, determinism, n = 0.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import TOL_ADJ, device, rel_l2, say, to_dev, upstream_gradient
from paper_1002_0916_amd import binding as B
from paper_1002_0916_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["plain", "compensated"]
GROUPS = ("x", "y", "z", "a")


def gpu_grads(cloud, G, nx, ny, variant, dev):
    x, y, z, a = to_dev(cloud, dev)
    g = torch.from_numpy(np.ascontiguousarray(G)).to(dev)
    out = B.backward(x, y, z, a, g, nx, ny, variant=variant)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in out]


def compare(gg, ref, variant, tag):
    for name, g, r in zip(GROUPS, gg, ref):
        e = rel_l2(g, r)
        say("  %s d%s rel-L2 = %.3e" % (tag, name, e))
        assert e <= TOL_ADJ[variant], (name, e)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", [(64, 48, 37), (100, 75, 130), (16, 16, 64), (33, 1, 5),
                                   (1, 40, 3)])
def test_small_full(oracle_mod, variant, shape):
    nx, ny, n = shape
    dev = device()
    c = W.random_cloud(200 + n, n, nx, ny, zlo=0.2, zhi=1.0, alo=-1.0, ahi=1.0, margin=30)
    G = upstream_gradient(oracle_mod, nx, ny, 300 + n)
    say("adjoint", shape, variant)
    gg = gpu_grads(c, G, nx, ny, variant, dev)
    ref = oracle_mod.adjoint(*c.astuple(), nx, ny, G, threads=0)
    compare(gg, ref, variant, "full")


def _sampled(oracle_mod, cloud, nx, ny, variant, dev, m, seed):
    G = upstream_gradient(oracle_mod, nx, ny, seed)
    idx = np.sort(np.random.default_rng(seed).choice(cloud.n, size=min(m, cloud.n),
                                                     replace=False))
    say("  oracle adjoint on", idx.shape[0], "sampled points")
    ref = oracle_mod.adjoint(*cloud.astuple(), nx, ny, G, idx=idx, threads=0)
    gg = gpu_grads(cloud, G, nx, ny, variant, dev)
    compare([g[idx] for g in gg], ref, variant, "sampled")


@pytest.mark.parametrize("variant", VARIANTS)
def test_paper_workload_sampled(oracle_mod, variant):
    dev = device()
    say("adjoint paper 1920x1024 N=1024", variant)
    _sampled(oracle_mod, W.paper_cloud(), 1920, 1024, variant, dev, 48, 51)


@pytest.mark.parametrize("variant", VARIANTS)
def test_adjoint_workload_sampled(oracle_mod, variant):
    dev = device()
    _, c = W.adjoint_clouds()
    say("adjoint 1024x1024 N=4096", variant)
    _sampled(oracle_mod, c, 1024, 1024, variant, dev, 48, 52)


@pytest.mark.parametrize("variant", VARIANTS)
def test_fit_workload_sampled(oracle_mod, variant):
    dev = device()
    _, c = W.fit_clouds()
    say("adjoint 3840x2160 N=16384", variant)
    _sampled(oracle_mod, c, 3840, 2160, variant, dev, 24, 53)


@pytest.mark.parametrize("variant", VARIANTS)
def test_deterministic(oracle_mod, variant):
    dev = device()
    c = W.paper_cloud(n=700)
    G = np.random.default_rng(54).standard_normal((333, 555)).astype(np.float32)
    a = gpu_grads(c, G, 555, 333, variant, dev)
    b = gpu_grads(c, G, 555, 333, variant, dev)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_empty_point_set():
    dev = device()
    e = torch.zeros(0, dtype=torch.float32, device=dev)
    g = torch.ones((8, 8), device=dev)
    out = B.backward(e, e, e, e, g, 8, 8)
    torch.cuda.synchronize()
    assert all(t.numel() == 0 for t in out)


@pytest.mark.parametrize("variant", VARIANTS)
def test_autograd_function_matches_backward(variant):
    """A linear loss L = sum(W * I) has dL/dI = W, so autograd through
    CGHFunction must return exactly cgh_backward(W)."""
    dev = device()
    c = W.random_cloud(55, 90, 120, 80, margin=10)
    x, y, z, a = (t.clone().requires_grad_(True) for t in to_dev(c, dev))
    Wt = torch.from_numpy(
        np.random.default_rng(56).standard_normal((80, 120)).astype(np.float32)).to(dev)
    I = B.CGHFunction.apply(x, y, z, a, 120, 80, W.PITCH, W.WAVELENGTH, variant)
    (I * Wt).sum().backward()
    ref = B.backward(*(t.detach() for t in (x, y, z, a)), Wt, 120, 80, variant=variant)
    for t, r in zip((x, y, z, a), ref):
        assert torch.equal(t.grad, r)
