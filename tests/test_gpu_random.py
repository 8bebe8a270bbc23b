"""Randomised GPU parity (hypothesis, derandomised so every run draws the same
cases): hologram shapes, point counts, depth ranges and amplitude scales
drawn per case, for every variant, forward and adjoint against the oracle at
that variant's bar."""
import numpy as np
import pytest
import torch
from hypothesis import given, settings
from hypothesis import strategies as st

from gpu_helpers import TOL_ADJ, TOL_FWD, device, max_err_frac, rel_l2, say, to_dev
from paper_1002_0916_amd import binding as B
from paper_1002_0916_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["plain", "compensated", "recurrence", "separable", "separable_f16x3",
            "separable_f16", "separable_bf16"]

CASES = dict(seed=st.integers(0, 2 ** 31 - 1), nx=st.integers(1, 260), ny=st.integers(1, 200),
             n=st.integers(1, 300), zlo=st.sampled_from([0.05, 0.2, 0.5, 2.0]),
             amp=st.sampled_from([1e-3, 1.0, 1e3]), margin=st.sampled_from([0.0, 25.0]))


@pytest.mark.parametrize("variant", VARIANTS)
@settings(max_examples=8, deadline=None, derandomize=True)
@given(**CASES)
def test_random_forward(oracle_mod, variant, seed, nx, ny, n, zlo, amp, margin):
    dev = device()
    c = W.random_cloud(seed, n, nx, ny, zlo=zlo, zhi=2 * zlo, alo=-amp, ahi=amp, margin=margin)
    say("random forward", variant, (nx, ny, n, zlo, amp, margin, seed))
    x, y, z, a = to_dev(c, dev)
    I = B.forward(x, y, z, a, nx, ny, variant=variant)
    torch.cuda.synchronize()
    ref = oracle_mod.forward(*c.astuple(), nx, ny, threads=0)
    err = max_err_frac(I.cpu().numpy(), ref, c)
    assert err <= TOL_FWD[variant], err


@pytest.mark.parametrize("variant", VARIANTS)
@settings(max_examples=6, deadline=None, derandomize=True)
@given(**CASES)
def test_random_adjoint(oracle_mod, variant, seed, nx, ny, n, zlo, amp, margin):
    dev = device()
    c = W.random_cloud(seed, n, nx, ny, zlo=zlo, zhi=2 * zlo, alo=-amp, ahi=amp, margin=margin)
    G = np.random.default_rng(seed ^ 0x5EED).standard_normal((ny, nx)).astype(np.float32)
    say("random adjoint", variant, (nx, ny, n, zlo, amp, margin, seed))
    x, y, z, a = to_dev(c, dev)
    g = torch.from_numpy(G).to(dev)
    gg = [t.cpu().numpy() for t in B.backward(x, y, z, a, g, nx, ny, variant=variant)]
    ref = oracle_mod.adjoint(*c.astuple(), nx, ny, G, threads=0)
    for name, gv, r in zip("xyza", gg, ref):
        assert np.all(np.isfinite(gv)), name
        e = rel_l2(gv, r)
        assert e <= TOL_ADJ[variant], (name, e)
