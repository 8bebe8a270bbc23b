"""Shared helpers of the GPU parity tests (inputs, tolerances, comparisons)."""
import sys

import numpy as np
import torch

from paper_1002_0916_amd import workloads as W

# Unit roundoff of the 16-bit GEMM operand formats (11 and 8 significant bits).
U_F16, U_BF16 = 2.0 ** -11, 2.0 ** -8


def _half_fwd_bar(u):
    """Forward bar of a once-rounded 16-bit format: every table entry carries a
    relative error <= u, so a term A_j (cY cX - sY sX) is off by at most
    (2u + u^2) |A_j| (|cY cX| + |sY sX| <= 1), i.e. |dI| <= (2u + u^2) sum |A|,
    plus the FP32 bar for the phase and accumulation arithmetic."""
    return 2 * u + u * u + 1e-4


# Acceptance bars for the forward, as fractions of sum_j |A_j|: max |dI| over
# the compared pixels.
TOL_FWD = {"plain": 2e-3, "compensated": 1e-4, "recurrence": 2e-3, "separable": 1e-4,
           "separable_f16x3": 1e-4,
           "separable_f16": _half_fwd_bar(U_F16), "separable_bf16": _half_fwd_bar(U_BF16)}
# Relative L2 error bars per gradient group (A, x, y, z), same G on both sides.
TOL_ADJ = {"plain": 1e-3, "compensated": 1e-4, "recurrence": 1e-3, "separable": 1e-4,
           "separable_f16x3": 1e-4,
           "separable_f16": 2 * U_F16, "separable_bf16": 2 * U_BF16}


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()


def device():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    return torch.device("cuda:0")


def to_dev(cloud: W.Cloud, dev):
    return tuple(torch.from_numpy(np.ascontiguousarray(v)).to(dev) for v in cloud.astuple())


def sum_abs_a(cloud: W.Cloud) -> float:
    return float(np.sum(np.abs(cloud.a.astype(np.float64))))


def max_err_frac(gpu_vals, ref_vals, cloud) -> float:
    g = np.asarray(gpu_vals, dtype=np.float64)
    r = np.asarray(ref_vals, dtype=np.float64)
    return float(np.max(np.abs(g - r)) / sum_abs_a(cloud)) if g.size else 0.0


def rel_l2(g, r) -> float:
    g = np.asarray(g, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    den = np.linalg.norm(r)
    return float(np.linalg.norm(g - r) / den) if den > 0 else float(np.linalg.norm(g))


def upstream_gradient(oracle_mod, nx, ny, seed):
    """A hologram-like upstream gradient G (float32): the FP64 oracle hologram of
    a small seeded cloud plus seeded Gaussian noise."""
    c = W.random_cloud(seed, 8, nx, ny, zlo=0.3, zhi=0.8, alo=0.5, ahi=1.0)
    I = oracle_mod.forward(*c.astuple(), nx, ny, threads=0)
    rng = np.random.default_rng(seed + 1)
    return (I + 0.5 * rng.standard_normal((ny, nx))).astype(np.float32)
