"""The allocation-free forward, cgh_forward_noalloc, through the C ABI.

It runs the same kernels as cgh_forward with its scratch in a static device
buffer instead of a caller's workspace, so for every variant its hologram
must equal cgh_forward's bitwise, and meet the variant's bar against the
FP64 oracle.  Two calls in a row, the second on a smaller problem, check that
a call does not depend on what the previous one left in the shared buffer.
The compensated forward that has to drop its column table to fit must still
give cgh_forward's bits.  Problems beyond the buffer are refused, and a
captured graph of the call replays bitwise like eager calls.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import TOL_FWD, device, max_err_frac, say, to_dev
from paper_1002_0916_amd import binding as B
from paper_1002_0916_amd import workloads as W

pytestmark = pytest.mark.gpu

VARIANTS = ["compensated", "plain", "recurrence", "separable", "separable_f16x3",
            "separable_f16", "separable_bf16"]


def _both(cloud, nx, ny, variant, dev):
    x, y, z, a = to_dev(cloud, dev)
    ref = B.forward(x, y, z, a, nx, ny, variant=variant)
    out = torch.full((ny, nx), float("nan"), device=dev)
    B.forward_noalloc(x, y, z, a, nx, ny, variant=variant, out=out)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("variant", VARIANTS)
def test_noalloc_matches_forward_two_calls(oracle_mod, variant):
    dev = device()
    big = W.paper_cloud()
    small = W.random_cloud(801, 77, 300, 200, zlo=0.2, zhi=1.0, alo=-1.0, ahi=1.0, margin=30)
    say("noalloc", variant, "call 1: 1920x1024 N=1024")
    got, ref = _both(big, 1920, 1024, variant, dev)
    assert np.array_equal(got, ref)
    px, py = W.sample_pixels(802, 1920, 1024, 1024)
    o = oracle_mod.forward_at(*big.astuple(), 1920, 1024, px, py, threads=0)
    err = max_err_frac(got[py, px], o, big)
    say("  bitwise equal to cgh_forward; max|dI|/sum|A| =", err)
    assert err <= TOL_FWD[variant]
    say("noalloc", variant, "call 2: 300x200 N=77")
    got, ref = _both(small, 300, 200, variant, dev)
    assert np.array_equal(got, ref)
    err = max_err_frac(got, oracle_mod.forward(*small.astuple(), 300, 200, threads=0), small)
    say("  bitwise equal to cgh_forward; max|dI|/sum|A| =", err)
    assert err <= TOL_FWD[variant]


def test_noalloc_compensated_without_column_table_same_bits():
    """4096 x 256 with 8192 points: the column table (134 MB) does not fit
    the 64 MiB buffer, so the allocation-free call forms the x-phases in the
    kernel; cgh_forward keeps the table.  Same bits."""
    dev = device()
    nx, ny, n = 4096, 256, 8192
    assert B.workspace_bytes(n, nx, ny, "compensated") > B.NOALLOC_SCRATCH_BYTES
    c = W.random_cloud(803, n, nx, ny, zlo=0.3, zhi=1.0, alo=-1.0, ahi=1.0, margin=20)
    got, ref = _both(c, nx, ny, "compensated", dev)
    assert np.array_equal(got, ref)


def test_noalloc_refuses_beyond_buffer():
    dev = device()
    _, c = W.fit_clouds()
    x, y, z, a = to_dev(c, dev)
    out = torch.zeros((2160, 3840), device=dev)
    with pytest.raises(B.CGHError, match="static buffer"):
        B.forward_noalloc(x, y, z, a, 3840, 2160, variant="compensated", out=out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0


@pytest.mark.parametrize("variant", ["compensated", "separable_f16x3"])
def test_noalloc_graph_replay(variant):
    dev = device()
    nx, ny = 333, 190
    c = W.random_cloud(804, 300, nx, ny, zlo=0.3, zhi=0.8, alo=-1.0, ahi=1.0, margin=10)
    x, y, z, a = to_dev(c, dev)
    a0 = a.clone()
    out = torch.empty((ny, nx), device=dev)
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        B.forward_noalloc(x, y, z, a, nx, ny, variant=variant, out=out)
    torch.cuda.current_stream(dev).wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        B.forward_noalloc(x, y, z, a, nx, ny, variant=variant, out=out)
    torch.cuda.synchronize()
    for rep in range(3):
        a.copy_(a0 * (1.0 + 0.5 * rep))
        want = B.forward(x, y, z, a, nx, ny, variant=variant).clone()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, want), rep
        say("noalloc graph", variant, "replay", rep, "matches cgh_forward")
    del graph
