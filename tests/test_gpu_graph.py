"""A whole forward + (I - T) + adjoint step captured into one HIP graph
(torch.cuda.graph) and replayed.

The library only enqueues kernels on the caller's stream: no allocation, no
memset nodes (buffers are cleared by fill kernels), no host synchronisation.
Every replay is checked bitwise against an eager step on the same inputs (the
kernels are deterministic), with the inputs changed by eager work between
replays, so a replay that reused stale results or raced with the eager work
would show.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import device, say, to_dev
from paper_1002_0916_amd import binding as B
from paper_1002_0916_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["compensated", "plain", "recurrence", "separable", "separable_f16x3",
            "separable_f16", "separable_bf16"]


@pytest.mark.parametrize("variant", VARIANTS)
def test_graph_replay_matches_eager(variant):
    dev = device()
    nx, ny = 333, 190  # ragged against every tile size
    c = W.random_cloud(501, 300, nx, ny, zlo=0.3, zhi=0.8, alo=-1.0, ahi=1.0, margin=10)
    h = W.random_cloud(502, 300, nx, ny, zlo=0.3, zhi=0.8, alo=-1.0, ahi=1.0, margin=10)
    x, y, z, a = to_dev(c, dev)
    hx, hy, hz, ha = to_dev(h, dev)
    T = B.forward_f64(hx, hy, hz, ha, nx, ny).float()
    a0 = a.clone()

    def step():
        I = B.forward(x, y, z, a, nx, ny, variant=variant)
        G = I - T
        return (I,) + tuple(B.backward(x, y, z, a, G, nx, ny, variant=variant))

    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        for _ in range(2):
            step()
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        outs = step()
    torch.cuda.synchronize()

    for rep in range(4):
        # eager work between replays: new amplitudes, then an eager reference
        a.copy_(a0 * (1.0 + 0.25 * rep))
        ref = [t.clone() for t in step()]
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for name, got, want in zip(("I", "dx", "dy", "dz", "dA"), outs, ref):
            same = torch.equal(got, want)
            if not same:
                d = (got.double() - want.double()).abs().max().item()
                say("  replay %d %s differs by %.3e" % (rep, name, d))
            assert same, (rep, name)
        say("graph", variant, "replay", rep, "matches eager")
    del graph
    B.release_workspaces()
    assert np.isfinite(outs[0].cpu().numpy()).all()
