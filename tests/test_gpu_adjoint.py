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

VARIANTS = ["plain", "compensated", "recurrence", "separable", "separable_f16x3",
            "separable_f16", "separable_bf16"]
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
                                   (1, 40, 3), (96, 5, 64), (160, 3, 200)])
def test_small_full(oracle_mod, variant, shape):
    """Full-grid gradients against the oracle.  (96, 5, 64) and (160, 3, 200)
    give runs of 7-8 strip-rows over strips of 5 or 3 rows, so the priority
    quarters of a run fall at odd row offsets inside and across strip
    segments."""
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


def test_backward_rejects_misshaped_grad():
    """G is [ny][nx]: a transposed or flat tensor of the same size is refused
    rather than read in the wrong layout."""
    dev = device()
    x, y, z, a = to_dev(W.random_cloud(7, 10, 40, 30), dev)
    for shape in [(40, 30), (1200,), (1, 30, 40)]:
        with pytest.raises(ValueError):
            B.backward(x, y, z, a, torch.zeros(shape, device=dev), 40, 30)
    out = B.backward(x, y, z, a, torch.zeros((30, 40), device=dev), 40, 30)
    torch.cuda.synchronize()
    assert all(t.numel() == 10 for t in out)


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


@pytest.mark.parametrize("variant", ["separable_f16x3", "separable_f16", "separable_bf16"])
@pytest.mark.parametrize("scale", [1e6, 1e-6])
def test_half_variants_gradient_range(oracle_mod, variant, scale):
    """G far outside the fp16 range or deep in its subnormals: the power-of-two
    scaling of G keeps the gradients at the bar."""
    nx, ny, n = 120, 90, 70
    dev = device()
    c = W.random_cloud(210, n, nx, ny, zlo=0.2, zhi=1.0, alo=-1.0, ahi=1.0, margin=20)
    G = (upstream_gradient(oracle_mod, nx, ny, 310) * scale).astype(np.float32)
    say("adjoint", variant, "G scale", scale)
    gg = gpu_grads(c, G, nx, ny, variant, dev)
    ref = oracle_mod.adjoint(*c.astuple(), nx, ny, G, threads=0)
    assert all(np.all(np.isfinite(g)) for g in gg)
    compare(gg, ref, variant, "scaled")


def test_adjoint_workload_against_central_differences(oracle_mod):
    """The 1024x1024, 4096-point adjoint workload: G = I - T with T the FP64
    hologram of the hidden cloud and I that of the perturbed cloud (oracle).
    GPU gradients (compensated) of 32 seeded points are checked against central
    differences of the FP64 loss 0.5 ||I - T||^2.  Steps: 1e-3 px in x, y,
    1e-3 in A, 1e-3 of the 1 mm depth perturbation (1 um) in z.  Only point j's
    term changes under a perturbation of point j, so each difference costs two
    single-point holograms."""
    dev = device()
    nx = ny = 1024
    hidden, c = W.adjoint_clouds()
    say("oracle holograms of the hidden and perturbed clouds (4096 points, 1024^2)")
    T = oracle_mod.forward(*hidden.astuple(), nx, ny, threads=0)
    I = oracle_mod.forward(*c.astuple(), nx, ny, threads=0)
    R = I - T
    gg = gpu_grads(c, R.astype(np.float32), nx, ny, "compensated", dev)
    idx = np.sort(np.random.default_rng(55).choice(c.n, size=32, replace=False))
    x, y, z, a = (v.astype(np.float64) for v in c.astuple())
    steps = {"x": 1e-3, "y": 1e-3, "z": 1e-6, "a": 1e-3}
    for gi, name in enumerate(GROUPS):
        fd = np.empty(idx.shape[0])
        for t, j in enumerate(idx):
            base = [x[j:j + 1], y[j:j + 1], z[j:j + 1], a[j:j + 1]]
            old = oracle_mod.forward(*base, nx, ny)
            k = "xyza".index(name)
            vals = []
            for sgn in (1.0, -1.0):
                pert = [v.copy() for v in base]
                pert[k] = pert[k] + sgn * steps[name]
                new = oracle_mod.forward(*pert, nx, ny)
                vals.append(0.5 * np.sum((R - old + new) ** 2))
            fd[t] = (vals[0] - vals[1]) / (2 * steps[name])
        e = rel_l2(gg[gi][idx], fd)
        say("  d%s vs central differences rel-L2 = %.3e" % (name, e))
        assert e <= TOL_ADJ["compensated"], (name, e)
