"""Fitting point amplitudes and depths to a target hologram through the
differentiable hologram map (``binding.CGHFunction``).

Loss L = 0.5 ||I(x, y, z, A) - T||^2 with I from Eq. (1) (Section 1).  The
trainable parameters are A and z measured in units of the pixel pitch (z / p,
the same normalisation the paper applies to x and y), updated with Adam; x, y
stay fixed.  Every forward and adjoint runs in the HIP kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import torch

from . import binding as B


@dataclass
class FitResult:
    a: torch.Tensor
    z: torch.Tensor
    losses: list = field(default_factory=list)
    seconds: float = 0.0
    iterations: int = 0
    fwd_ms: float = 0.0
    adj_ms: float = 0.0

    @property
    def iterations_per_s(self) -> float:
        return self.iterations / self.seconds if self.seconds > 0 else 0.0


def fit(x, y, z, a, target, nx: int, ny: int, iters: int = 100, lr: float = 1e-2,
        pitch: float = 8e-6, wavelength: float = 633e-9, variant="compensated",
        time_kernels: bool = True) -> FitResult:
    """Adam on (A, z / pitch) for ``iters`` iterations; returns the fitted A, z
    (metres) and the per-iteration losses (read back once, at the end)."""
    a_p = a.detach().clone().requires_grad_(True)
    zp = (z.detach() / pitch).clone().requires_grad_(True)
    opt = torch.optim.Adam([a_p, zp], lr=lr)
    losses = []
    if time_kernels:
        for k in range(B.KERNEL_COUNT):
            B.profile_read(k)
        B.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        for _ in range(iters):
            opt.zero_grad(set_to_none=True)
            I = B.CGHFunction.apply(x, y, zp * pitch, a_p, nx, ny, pitch, wavelength, variant)
            loss = 0.5 * torch.sum((I - target) ** 2)
            loss.backward()
            opt.step()
            losses.append(loss.detach())
        torch.cuda.synchronize()
    finally:
        if time_kernels:
            B.profile_enable(False)
    seconds = time.perf_counter() - t0
    res = FitResult(a=a_p.detach(), z=(zp * pitch).detach(),
                    losses=[float(v) for v in torch.stack(losses).cpu()] if losses else [],
                    seconds=seconds, iterations=iters)
    if time_kernels:
        v = B.variant_id(variant)
        sep = v in B.SEPARABLE_IDS
        fk = B.KERNEL_FWD_SEPARABLE if sep else {B.PLAIN: B.KERNEL_FWD_PLAIN,
                                                 B.COMPENSATED: B.KERNEL_FWD_COMPENSATED,
                                                 B.RECURRENCE: B.KERNEL_FWD_RECURRENCE}[v]
        ak = B.KERNEL_ADJ_SEPARABLE if sep else {B.PLAIN: B.KERNEL_ADJ_PLAIN,
                                                 B.COMPENSATED: B.KERNEL_ADJ_COMPENSATED,
                                                 B.RECURRENCE: B.KERNEL_ADJ_RECURRENCE}[v]
        nf, tf = B.profile_read(fk)
        na, ta = B.profile_read(ak)
        res.fwd_ms = tf / max(nf, 1)
        res.adj_ms = ta / max(na, 1)
    return res
