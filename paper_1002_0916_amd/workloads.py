"""Seeded synthetic point clouds for the hologram workloads.

This module only draws inputs: it holds none of the hologram arithmetic, and
both the GPU library's callers and the CPU oracle's tests take their inputs
from it.  The paper measures on an unnamed 3-D object of N points at a
1,920 x 1,024 hologram (Section 2.2, Table 1); seeded uniform clouds and a
seeded random height-field triangle mesh stand in for it.

Units follow Section 1: x, y in pixel units (normalised by the pitch p), z,
pitch and wavelength in metres.  Every draw is float64 from
``numpy.random.default_rng(seed)`` in the order x, y, z, A, then rounded to
float32.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_BASE = 10020916
PITCH = 8e-6
WAVELENGTH = 633e-9


@dataclass
class Cloud:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    a: np.ndarray

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def take(self, k: int) -> "Cloud":
        return Cloud(self.x[:k].copy(), self.y[:k].copy(), self.z[:k].copy(), self.a[:k].copy())

    def astuple(self):
        return self.x, self.y, self.z, self.a


def _f32(v) -> np.ndarray:
    return np.ascontiguousarray(v, dtype=np.float32)


def uniform_cloud(seed: int, n: int, xmax: float, ymax: float, zlo: float, zhi: float,
                  alo: float, ahi: float) -> Cloud:
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, xmax, n)
    y = rng.uniform(0.0, ymax, n)
    z = rng.uniform(zlo, zhi, n)
    a = rng.uniform(alo, ahi, n)
    return Cloud(_f32(x), _f32(y), _f32(z), _f32(a))


def mesh_cloud(seed: int, n: int, nx: int, ny: int, zlo: float = 0.2, zhi: float = 1.5,
               gx: int = 17, gy: int = 10) -> Cloud:
    """Points on a seeded random triangle-mesh surface spanning the aperture.

    The surface is a height field: a gx x gy grid of vertices over
    [0, nx) x [0, ny) with iid uniform depths in [zlo, zhi], each cell split
    into two triangles along its main diagonal.  x, y are uniform over the
    aperture (area-uniform on the projected surface); z is the barycentric
    interpolation of the containing triangle's vertex depths, so it stays in
    [zlo, zhi].  A is uniform in [0, 1].
    """
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, nx, n)
    y = rng.uniform(0.0, ny, n)
    vz = rng.uniform(zlo, zhi, (gy, gx))
    a = rng.uniform(0.0, 1.0, n)
    cw = nx / (gx - 1)
    ch = ny / (gy - 1)
    u = x / cw
    v = y / ch
    ci = np.minimum(np.floor(u).astype(np.int64), gx - 2)
    cj = np.minimum(np.floor(v).astype(np.int64), gy - 2)
    fu = u - ci
    fv = v - cj
    z00 = vz[cj, ci]
    z10 = vz[cj, ci + 1]
    z01 = vz[cj + 1, ci]
    z11 = vz[cj + 1, ci + 1]
    lower = fu >= fv  # triangle (00, 10, 11)
    z_lo = z00 + fu * (z10 - z00) + fv * (z11 - z10)
    z_up = z00 + fv * (z01 - z00) + fu * (z11 - z01)
    z = np.where(lower, z_lo, z_up)
    return Cloud(_f32(x), _f32(y), _f32(z), _f32(a))


def perturb(cloud: Cloud, seed: int, sxy: float = 0.5, sz: float = 1e-3,
            sa: float = 0.1) -> Cloud:
    """Trainable cloud = hidden cloud + Gaussian noise (x, y in pixels, z in metres)."""
    rng = np.random.default_rng(seed)
    n = cloud.n
    dx = rng.normal(0.0, sxy, n)
    dy = rng.normal(0.0, sxy, n)
    dz = rng.normal(0.0, sz, n)
    da = rng.normal(0.0, sa, n)
    return Cloud(_f32(cloud.x.astype(np.float64) + dx), _f32(cloud.y.astype(np.float64) + dy),
                 _f32(cloud.z.astype(np.float64) + dz), _f32(cloud.a.astype(np.float64) + da))


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    n: int
    description: str
    pitch: float = PITCH
    wavelength: float = WAVELENGTH

    @property
    def interactions(self) -> int:
        return self.n * self.nx * self.ny


# The five workload shapes.  "paper" is the headline shape of Table 1 / the
# abstract: a 1,920 x 1,024 hologram from 1,024 points.
WORKLOADS = {
    "small": Workload("small", 256, 256, 64,
                      "256x256 hologram, 64 points, z in [0.3,0.6] m"),
    "paper": Workload("paper", 1920, 1024, 1024,
                      "1920x1024 hologram, 1024 points, z in [0.5,1.0] m"),
    "mesh8k": Workload("mesh8k", 1920, 1080, 8192,
                       "1920x1080 hologram, 8192 mesh points, z in [0.2,1.5] m"),
    "mesh64k": Workload("mesh64k", 1920, 1080, 65536,
                        "1920x1080 hologram, 65536 mesh points, z in [0.2,1.5] m"),
    "adjoint": Workload("adjoint", 1024, 1024, 4096,
                        "1024x1024 hologram, 4096 points, perturbed from a hidden cloud"),
    "fit4k": Workload("fit4k", 3840, 2160, 16384,
                      "3840x2160 hologram, 16384 points, perturbed from a hidden cloud"),
}


def small_cloud() -> Cloud:
    return uniform_cloud(SEED_BASE + 0, 64, 256.0, 256.0, 0.3, 0.6, 0.5, 1.0)


def paper_cloud(n: int = 1024, seed: int = SEED_BASE + 1) -> Cloud:
    return uniform_cloud(seed, n, 1920.0, 1024.0, 0.5, 1.0, 0.5, 1.0)


def paper_target_cloud() -> Cloud:
    """Second cloud of the 1920x1024 shape whose hologram is the fitting target."""
    return paper_cloud(seed=SEED_BASE + 10)


def mesh_clouds() -> tuple[Cloud, Cloud]:
    """(8192-point, 65536-point) mesh clouds; the first is a prefix of the second."""
    big = mesh_cloud(SEED_BASE + 2, 65536, 1920, 1080)
    return big.take(8192), big


def adjoint_clouds() -> tuple[Cloud, Cloud]:
    """(hidden, trainable) clouds of the 1024x1024, 4096-point adjoint workload."""
    hidden = uniform_cloud(SEED_BASE + 3, 4096, 1024.0, 1024.0, 0.3, 0.6, 0.5, 1.0)
    return hidden, perturb(hidden, SEED_BASE + 4)


def fit_clouds() -> tuple[Cloud, Cloud]:
    """(hidden, trainable) clouds of the 3840x2160, 16384-point fitting workload."""
    hidden = uniform_cloud(SEED_BASE + 6, 16384, 3840.0, 2160.0, 0.3, 0.6, 0.5, 1.0)
    return hidden, perturb(hidden, SEED_BASE + 7)


def sample_pixels(seed: int, nx: int, ny: int, m: int) -> tuple[np.ndarray, np.ndarray]:
    """m seeded pixels plus the four corners and the centre (row-major unique)."""
    rng = np.random.default_rng(seed)
    px = rng.integers(0, nx, m)
    py = rng.integers(0, ny, m)
    px = np.concatenate([px, [0, nx - 1, 0, nx - 1, nx // 2]])
    py = np.concatenate([py, [0, 0, ny - 1, ny - 1, ny // 2]])
    flat = np.unique(py.astype(np.int64) * nx + px.astype(np.int64))
    return (flat % nx).astype(np.int64), (flat // nx).astype(np.int64)


def random_cloud(seed: int, n: int, nx: int, ny: int, zlo: float = 0.3, zhi: float = 0.6,
                 alo: float = -1.0, ahi: float = 1.0, margin: float = 0.0) -> Cloud:
    """Generic seeded cloud for tests (points may lie outside the aperture by ``margin``)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-margin, nx + margin, n)
    y = rng.uniform(-margin, ny + margin, n)
    z = rng.uniform(zlo, zhi, n)
    a = rng.uniform(alo, ahi, n)
    return Cloud(_f32(x), _f32(y), _f32(z), _f32(a))
