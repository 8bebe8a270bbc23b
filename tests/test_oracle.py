"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's own loop: each checks a closed form, an
invariant, an independent formulation or a high-precision brute force of
Eq. (1) (Section 1), the recurrence of Eq. (2) (Section 2.1), or, for the
adjoint, finite differences of the pinned forward.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from paper_1002_0916_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
P, LAM = W.PITCH, W.WAVELENGTH


def f32(*vals):
    return [np.asarray(v, dtype=np.float32) for v in vals]


# ---------------------------------------------------------------- forward --

def test_single_point_peak_equals_amplitude(oracle_mod):
    """A point on a grid node gives I = A there (cos 0 = 1), Eq. (1)."""
    x, y, z, a = f32([37.0], [21.0], [0.45], [0.8125])
    I = oracle_mod.forward(x, y, z, a, 64, 48)
    assert I[21, 37] == np.float64(np.float32(0.8125))
    assert np.all(np.abs(I) <= 0.8125 + 1e-15)


def test_single_point_eightfold_symmetry(oracle_mod):
    """Radial symmetry about a grid node is exact (bitwise) in the oracle."""
    x0, y0 = 20, 20
    x, y, z, a = f32([x0], [y0], [0.37], [1.0])
    I = oracle_mod.forward(x, y, z, a, 41, 41)
    for u in range(0, 21):
        for v in range(0, 21):
            vals = {I[y0 + v, x0 + u], I[y0 + v, x0 - u], I[y0 - v, x0 + u], I[y0 - v, x0 - u],
                    I[y0 + u, x0 + v], I[y0 + u, x0 - v], I[y0 - u, x0 + v], I[y0 - u, x0 - v]}
            assert len(vals) == 1, (u, v, vals)


@pytest.mark.parametrize("z", [0.3, 0.5, 1.0])
def test_fresnel_zone_plate_radii(oracle_mod, z):
    """Sign changes along a row through an on-axis point sit at the textbook
    Fresnel zone radii: the phase pi r^2 / (lambda z) (physical r) crosses
    (k + 1/2) pi at r_k = sqrt((k + 1/2) lambda z), i.e. r_k / p pixels."""
    n = 1200
    x, y, z_, a = f32([0.0], [0.0], [z], [1.0])
    row = oracle_mod.forward(x, y, z_, a, n, 1)[0]
    zf = float(np.float32(z))
    radii = []
    k = 0
    while True:
        r = math.sqrt((k + 0.5) * LAM * zf) / P
        if r >= n - 1:
            break
        radii.append(r)
        k += 1
    changes = [u for u in range(n - 1) if np.sign(row[u]) != np.sign(row[u + 1])]
    expected = [int(math.floor(r)) for r in radii]
    # Every predicted zero falls between the pixels whose signs differ; skip
    # radii that land within 1e-6 px of a pixel centre (sign undetermined).
    clean = [e for e, r in zip(expected, radii) if abs(r - round(r)) > 1e-6]
    assert set(clean) <= set(changes)
    assert len(changes) == len(expected)


def test_linearity_in_amplitude(oracle_mod):
    c = W.random_cloud(11, 40, 50, 30, alo=-1.0, ahi=1.0, margin=20)
    I1 = oracle_mod.forward(*c.astuple(), 50, 30)
    I4 = oracle_mod.forward(c.x, c.y, c.z, (4 * c.a).astype(np.float32), 50, 30)
    assert np.array_equal(I4, 4 * I1)  # power-of-two scaling is exact
    a3 = c.a.astype(np.float64) * 3.7
    I3 = oracle_mod.forward(c.x, c.y, c.z, a3, 50, 30)
    assert np.max(np.abs(I3 - 3.7 * I1)) <= 1e-13 * np.sum(np.abs(a3))


def test_superposition_and_empty(oracle_mod):
    c = W.random_cloud(12, 64, 40, 33, margin=10)
    I = oracle_mod.forward(*c.astuple(), 40, 33)
    s1, s2 = c.take(25), W.Cloud(c.x[25:], c.y[25:], c.z[25:], c.a[25:])
    I12 = oracle_mod.forward(*s1.astuple(), 40, 33) + oracle_mod.forward(*s2.astuple(), 40, 33)
    assert np.max(np.abs(I - I12)) <= 1e-12 * np.sum(np.abs(c.a))
    e = np.zeros(0, dtype=np.float32)
    assert np.array_equal(oracle_mod.forward(e, e, e, e, 7, 5), np.zeros((5, 7)))
    z = oracle_mod.forward(c.x, c.y, c.z, np.zeros_like(c.a), 40, 33)
    assert np.array_equal(z, np.zeros((33, 40)))


@pytest.mark.parametrize("name", ["tiny_near", "tiny_far"])
def test_against_stored_brute_force(oracle_mod, name):
    """Stored 40-digit brute force (tests/golden/make_brute.py, oracle/brute.py)."""
    with open(os.path.join(HERE, "golden", "brute_%s.json" % name)) as f:
        d = json.load(f)
    I = oracle_mod.forward(d["x"], d["y"], d["z"], d["a"], d["nx"], d["ny"], d["pitch"],
                           d["wavelength"])
    ref = np.array([[float(v) for v in row] for row in d["I"]])
    # FP64 relative rounding times the largest phase (~1e3 rad) bounds the error.
    assert np.max(np.abs(I - ref)) < 1e-12


def test_against_live_brute_force(oracle_mod):
    from oracle import brute

    c = W.random_cloud(13, 4, 6, 5, zlo=1e-4, zhi=4e-4, margin=3)
    I = oracle_mod.forward(*c.astuple(), 6, 5)
    ref = np.array([[float(v) for v in row] for row in brute.hologram(*c.astuple(), 6, 5, P, LAM)])
    assert np.max(np.abs(I - ref)) < 1e-12


@settings(max_examples=30, deadline=None, derandomize=True)
@given(seed=st.integers(0, 2 ** 31 - 1), n=st.integers(1, 4), nx=st.integers(1, 6),
       ny=st.integers(1, 5), z=st.sampled_from([1e-4, 1e-3, 1e-2, 0.5]),
       amp=st.sampled_from([1e-6, 1.0, 1e6]))
def test_random_clouds_against_brute_force(oracle_mod, seed, n, nx, ny, z, amp):
    """Random tiny clouds (points up to 3 px outside the grid, depths giving
    phases from ~1e-2 to ~500 rad, amplitudes over 12 decades): the oracle
    matches the 50-digit brute force within FP64 rounding of the phase."""
    from oracle import brute

    c = W.random_cloud(seed, n, nx, ny, zlo=z, zhi=2 * z, alo=-amp, ahi=amp, margin=3)
    I = oracle_mod.forward(*c.astuple(), nx, ny)
    ref = np.array([[float(v) for v in row]
                    for row in brute.hologram(*c.astuple(), nx, ny, P, LAM)])
    # |d theta| <= a few ulp(theta) with theta <= 500 rad: < 1e-12 per unit amplitude
    bound = 1e-12 * float(np.sum(np.abs(c.a.astype(np.float64))))
    assert np.max(np.abs(I - ref)) <= bound


def test_integer_translation(oracle_mod):
    """Shifting points by integers (s, t) shifts the hologram window exactly."""
    c = W.random_cloud(14, 30, 40, 30, margin=5)
    s, t = 9, 4
    I = oracle_mod.forward(*c.astuple(), 40, 30)
    xs = (c.x.astype(np.float64) + s)
    ys = (c.y.astype(np.float64) + t)
    J = oracle_mod.forward(xs, ys, c.z, c.a, 40 + s, 30 + t)
    assert np.array_equal(J[t:, s:], I)


def test_separable_identity(oracle_mod):
    """I = Re(V diag(A) U^T) with U[x,j] = exp(i P_j (x-x_j)^2) and
    V[y,j] = exp(i P_j (y-y_j)^2): an independent formulation (a complex GEMM)."""
    nx, ny = 300, 180
    c = W.random_cloud(15, 500, nx, ny, zlo=0.2, zhi=1.5, margin=50)
    I = oracle_mod.forward(*c.astuple(), nx, ny, threads=0)
    x, y, z, a = (v.astype(np.float64) for v in c.astuple())
    Pj = np.pi * P * P / (LAM * z)
    U = np.exp(1j * Pj[None, :] * (np.arange(nx)[:, None] - x[None, :]) ** 2)
    V = np.exp(1j * Pj[None, :] * (np.arange(ny)[:, None] - y[None, :]) ** 2)
    ref = ((V * a[None, :]) @ U.T).real
    assert np.max(np.abs(I - ref)) <= 1e-10 * np.sum(np.abs(a))


def test_recurrence_eq2_exact_in_rationals():
    """Eq. (2): Gamma_n = Gamma_{n-1} + delta_{n-1}, delta_n = delta_{n-1} + Delta with
    Gamma_0 = P((x_h-x_j)^2+(y_h-y_j)^2), delta_0 = P(2(x_h-x_j)+1), Delta = 2P
    reproduces the phase at x_h + n exactly."""
    Pj = Fraction(0.0012345)
    xj, yj = Fraction(float(np.float32(17.3))), Fraction(float(np.float32(-4.6)))
    xh, yh = Fraction(3), Fraction(9)
    G = Pj * ((xh - xj) ** 2 + (yh - yj) ** 2)
    d = Pj * (2 * (xh - xj) + 1)
    D = 2 * Pj
    for n in range(1, 200):
        G, d = G + d, d + D
        assert G == Pj * ((xh + n - xj) ** 2 + (yh - yj) ** 2)


def test_oracle_row_matches_recurrence(oracle_mod):
    """A hologram row from the oracle equals the row built with Eq. (2)'s phases
    (exact rationals per point, one cosine per pixel)."""
    nx = 64
    c = W.random_cloud(16, 12, nx, 8, zlo=0.3, zhi=0.6, margin=30)
    yh = 5
    row = oracle_mod.forward(*c.astuple(), nx, 8)[yh]
    acc = np.zeros(nx)
    for j in range(c.n):
        Pj = Fraction(math.pi) * Fraction(P) ** 2 / (Fraction(LAM) * Fraction(float(c.z[j])))
        xj, yj = Fraction(float(c.x[j])), Fraction(float(c.y[j]))
        G = Pj * ((0 - xj) ** 2 + (yh - yj) ** 2)
        d = Pj * (2 * (0 - xj) + 1)
        for n in range(nx):
            acc[n] += float(c.a[j]) * math.cos(float(G))
            G, d = G + d, d + 2 * Pj
    assert np.max(np.abs(row - acc)) <= 1e-11 * np.sum(np.abs(c.a))


def test_threads_bitwise_and_subset(oracle_mod):
    c = W.random_cloud(17, 50, 70, 45, margin=10)
    I1 = oracle_mod.forward(*c.astuple(), 70, 45, threads=1)
    I5 = oracle_mod.forward(*c.astuple(), 70, 45, threads=5)
    assert np.array_equal(I1, I5)
    px, py = W.sample_pixels(3, 70, 45, 100)
    vals = oracle_mod.forward_at(*c.astuple(), 70, 45, px, py, threads=3)
    assert np.array_equal(vals, I1[py, px])


def test_rejects_bad_arguments(oracle_mod):
    c = W.random_cloud(18, 4, 8, 8)
    with pytest.raises(ValueError):
        oracle_mod.forward(*c.astuple(), 0, 8)
    with pytest.raises(ValueError):
        oracle_mod.forward(*c.astuple(), 8, 8, pitch=-1.0)
    with pytest.raises(ValueError):
        oracle_mod.forward_at(*c.astuple(), 8, 8, [8], [0])


# ---------------------------------------------------------------- adjoint --

def _loss(oracle_mod, x, y, z, a, nx, ny, T):
    I = oracle_mod.forward(x, y, z, a, nx, ny)
    return 0.5 * np.sum((I - T) ** 2)


def test_adjoint_against_central_differences(oracle_mod):
    """dL/dA, dL/dx, dL/dy, dL/dz of L = 0.5 ||I - T||^2 against central FD of the
    pinned forward.  Steps: 1e-3 in pixels (x, y), 1e-3 in A, and 1e-3 pixel
    pitches (8 nm) in z."""
    nx, ny = 48, 36
    hidden = W.random_cloud(19, 10, nx, ny, zlo=0.02, zhi=0.05, alo=0.5, ahi=1.0)
    T = oracle_mod.forward(*hidden.astuple(), nx, ny)
    c = W.random_cloud(20, 10, nx, ny, zlo=0.02, zhi=0.05, alo=0.5, ahi=1.0)
    x, y, z, a = (v.astype(np.float64) for v in c.astuple())
    G = oracle_mod.forward(x, y, z, a, nx, ny) - T
    gx, gy, gz, ga = oracle_mod.adjoint(x, y, z, a, nx, ny, G)
    steps = {"x": 1e-3, "y": 1e-3, "z": 1e-3 * P, "a": 1e-3}
    grads = {"x": gx, "y": gy, "z": gz, "a": ga}
    for name, h in steps.items():
        for j in range(c.n):
            arrs = {"x": x.copy(), "y": y.copy(), "z": z.copy(), "a": a.copy()}
            arrs[name][j] += h
            lp = _loss(oracle_mod, arrs["x"], arrs["y"], arrs["z"], arrs["a"], nx, ny, T)
            arrs[name][j] -= 2 * h
            lm = _loss(oracle_mod, arrs["x"], arrs["y"], arrs["z"], arrs["a"], nx, ny, T)
            fd = (lp - lm) / (2 * h)
            scale = max(abs(fd), np.max(np.abs(grads[name])) * 1e-3)
            assert abs(grads[name][j] - fd) <= 2e-6 * scale, (name, j, grads[name][j], fd)


def test_adjoint_dot_product(oracle_mod):
    """<J v, w> = <v, J^T w> with J = dI/d(params), J v by central FD of the forward."""
    nx, ny = 40, 30
    c = W.random_cloud(21, 8, nx, ny, zlo=0.02, zhi=0.05)
    x, y, z, a = (v.astype(np.float64) for v in c.astuple())
    rng = np.random.default_rng(22)
    w = rng.standard_normal((ny, nx))
    v = {k: rng.standard_normal(8) for k in "xyza"}
    h = 1e-4
    scale = {"x": 1.0, "y": 1.0, "z": P, "a": 1.0}
    Ip = oracle_mod.forward(x + h * v["x"], y + h * v["y"], z + h * P * v["z"], a + h * v["a"],
                            nx, ny)
    Im = oracle_mod.forward(x - h * v["x"], y - h * v["y"], z - h * P * v["z"], a - h * v["a"],
                            nx, ny)
    jv = (Ip - Im) / (2 * h)
    gx, gy, gz, ga = oracle_mod.adjoint(x, y, z, a, nx, ny, w)
    lhs = np.sum(jv * w)
    rhs = (np.dot(gx, v["x"]) * scale["x"] + np.dot(gy, v["y"]) * scale["y"] +
           np.dot(gz, v["z"]) * scale["z"] + np.dot(ga, v["a"]) * scale["a"])
    assert abs(lhs - rhs) <= 1e-6 * (abs(lhs) + 1e-3)


def test_adjoint_amplitude_homogeneity(oracle_mod):
    """I is linear in A, so sum_j A_j dL/dA_j = sum_h G I for any G (Euler)."""
    nx, ny = 33, 29
    c = W.random_cloud(23, 20, nx, ny, margin=10)
    rng = np.random.default_rng(24)
    G = rng.standard_normal((ny, nx))
    I = oracle_mod.forward(*c.astuple(), nx, ny)
    _, _, _, ga = oracle_mod.adjoint(*c.astuple(), nx, ny, G)
    lhs = np.dot(c.a.astype(np.float64), ga)
    assert abs(lhs - np.sum(G * I)) <= 1e-12 * np.sum(np.abs(G)) * np.sum(np.abs(c.a))


def test_adjoint_pixel_impulse(oracle_mod):
    """G = e_pixel: A_j dL/dA_j is point j's own contribution, which is what the
    forward of the single point j gives at that pixel."""
    nx, ny = 20, 15
    c = W.random_cloud(25, 6, nx, ny, margin=5)
    G = np.zeros((ny, nx))
    G[7, 11] = 1.0
    _, _, _, ga = oracle_mod.adjoint(*c.astuple(), nx, ny, G)
    for j in range(c.n):
        single = oracle_mod.forward(c.x[j:j + 1], c.y[j:j + 1], c.z[j:j + 1], c.a[j:j + 1],
                                    nx, ny)
        assert abs(float(c.a[j]) * ga[j] - single[7, 11]) <= 1e-15


def test_adjoint_subset_and_threads_bitwise(oracle_mod):
    nx, ny = 31, 17
    c = W.random_cloud(26, 40, nx, ny, margin=5)
    G = np.random.default_rng(27).standard_normal((ny, nx))
    full = oracle_mod.adjoint(*c.astuple(), nx, ny, G, threads=1)
    par = oracle_mod.adjoint(*c.astuple(), nx, ny, G, threads=4)
    idx = np.array([39, 0, 17, 17, 5])
    sub = oracle_mod.adjoint(*c.astuple(), nx, ny, G, idx=idx, threads=2)
    for f, p_, s in zip(full, par, sub):
        assert np.array_equal(f, p_)
        assert np.array_equal(f[idx], s)
