"""Host-side checks of the C ABI (no GPU needed, no kernel launched).

The library must load, export every function that include/cgh.h declares,
size workspaces consistently, and reject bad arguments on the host before
anything is enqueued.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cgh.h")


@pytest.fixture(scope="module")
def lib():
    from paper_1002_0916_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        from paper_1002_0916_amd import build

        build.build()
    return binding.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cgh_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("cgh_forward", "cgh_forward_f64", "cgh_backward", "cgh_workspace_bytes",
                     "cgh_strerror"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_1002_0916_amd import binding

    assert sorted(binding.EXPORTED) == declared_functions()


def test_binding_constants_match_header():
    """Every numeric #define of the header has the same value in the binding
    (variants, operations, kernel ids, status codes)."""
    from paper_1002_0916_amd import binding as B

    with open(HEADER) as f:
        defines = dict(re.findall(r"^#define (CGH_[A-Z0-9_]+) (\d+)", f.read(), flags=re.M))
    checked = 0
    for macro, value in defines.items():
        # status codes keep their prefix in the binding, the rest drop it
        status = macro == "CGH_OK" or macro.startswith("CGH_E")
        attr = macro if status else macro[len("CGH_"):]
        assert hasattr(B, attr), macro
        assert getattr(B, attr) == int(value), macro
        checked += 1
    assert checked >= 20
    assert max(B.VARIANTS.values()) == int(defines["CGH_RECURRENCE"])


def test_strerror_and_version(lib):
    for code in range(5):
        assert isinstance(lib.cgh_strerror(code), bytes) and lib.cgh_strerror(code)
    assert lib.cgh_strerror(99) == b"unknown status"
    assert lib.cgh_version() >= 100


def test_workspace_bytes(lib):
    from paper_1002_0916_amd import binding as B

    f = lib.cgh_workspace_bytes
    assert f(0, 16, 16, B.PLAIN, B.OP_FORWARD) == 0
    assert f(-1, 16, 16, B.PLAIN, B.OP_FORWARD) == 0
    assert f(10, 0, 16, B.PLAIN, B.OP_FORWARD) == 0
    bad = max(B.VARIANTS.values()) + 1
    assert f(10, 16, 16, bad, B.OP_FORWARD) == 0
    assert f(10, 16, 16, -1, B.OP_FORWARD) == 0
    for v in B.SEPARABLE_IDS + (B.RECURRENCE,):
        assert f(10, 16, 16, v, B.OP_FORWARD) > 0
        assert f(10, 16, 16, v, B.OP_BACKWARD) > 0
    assert f(10, 16, 16, B.PLAIN, 9) == 0
    assert f(4000001, 16, 16, B.PLAIN, B.OP_FORWARD) == 0
    assert f(4000000, 16, 16, B.PLAIN, B.OP_BACKWARD) > 0
    p = f(1024, 1920, 1024, B.PLAIN, B.OP_FORWARD)
    c = f(1024, 1920, 1024, B.COMPENSATED, B.OP_FORWARD)
    d = f(1024, 1920, 1024, B.PLAIN, B.OP_FORWARD_F64)
    b = f(1024, 1920, 1024, B.COMPENSATED, B.OP_BACKWARD)
    assert 0 < p < c and p < d and p < b
    # the compensated forward's tables: row phases [256 row groups][N][4] and
    # column phases [30 * 64 columns][N]
    assert c - p == 256 * 1024 * 4 * 4 + 30 * 64 * 1024 * 4
    # the column table is dropped above 256 MiB (64 columns x 4M points)
    big_f = (4000000, 64, 16)
    row_tab = 8 * 4000000 * 4 * 4  # 8 row groups of 4 rows
    assert (f(*big_f, B.COMPENSATED, B.OP_FORWARD) - f(*big_f, B.PLAIN, B.OP_FORWARD)
            == row_tab)
    # 1920 columns x 65536 points (503 MB): no column table; 3840 x 16384
    # (252 MB): a column table
    mesh = (65536, 1920, 1080)
    rows_mesh = 34 * 8 * 65536 * 4 * 4
    assert f(*mesh, B.COMPENSATED, B.OP_FORWARD) - f(*mesh, B.PLAIN, B.OP_FORWARD) == rows_mesh
    fit = (16384, 3840, 2160)
    rows_fit = 68 * 8 * 16384 * 4 * 4
    assert (f(*fit, B.COMPENSATED, B.OP_FORWARD) - f(*fit, B.PLAIN, B.OP_FORWARD)
            == rows_fit + 3840 * 16384 * 4)
    # the compensated adjoint's tables: the row table, {cos, sin} of the y-phase per row
    # and point (N * Ny float2), and the column table, the x-phase per strip
    # column and point (N * ceil(Nx / 32) * 32 floats), while each fits in
    # 512 MiB; above that the kernel forms the values itself and the
    # workspace equals the plain adjoint's
    bp = f(1024, 1920, 1024, B.PLAIN, B.OP_BACKWARD)
    assert b - bp == 1024 * 1024 * 8 + 1920 * 1024 * 4
    big = (16448, 32, 4096)
    assert big[0] * big[2] * 8 > 512 << 20
    assert f(*big, B.COMPENSATED, B.OP_BACKWARD) == f(*big, B.PLAIN, B.OP_BACKWARD)
    edge = (4096, 32, 16384)  # a row table of exactly 512 MiB: still the tables
    assert (f(*edge, B.COMPENSATED, B.OP_BACKWARD) - f(*edge, B.PLAIN, B.OP_BACKWARD)
            == (512 << 20) + 32 * 4096 * 4)
    wide = (16448, 8192, 4)  # a column table above 512 MiB: none
    assert wide[0] * wide[1] * 4 > 512 << 20
    assert f(*wide, B.COMPENSATED, B.OP_BACKWARD) == f(*wide, B.PLAIN, B.OP_BACKWARD)
    wide_edge = (4096, 32768, 4)  # a column table of exactly 512 MiB: the tables
    assert (f(*wide_edge, B.COMPENSATED, B.OP_BACKWARD) - f(*wide_edge, B.PLAIN, B.OP_BACKWARD)
            == 4 * 4096 * 8 + (512 << 20))
    for v in (p, c, d, b):
        assert v % 256 == 0
    # monotone in N
    assert f(4096, 1920, 1024, B.COMPENSATED, B.OP_BACKWARD) > b


def _args(n=4):
    dummy = ctypes.c_void_p(256)
    return [dummy] * 4, n


@pytest.mark.parametrize("case", ["null", "nx", "ny", "n", "pitch", "wl", "nan", "variant",
                                  "out", "toolarge"])
def test_forward_rejects_bad_arguments(lib, case):
    from paper_1002_0916_amd import binding as B

    p = ctypes.c_void_p(256)
    args = dict(x=p, y=p, z=p, a=p, n=4, nx=8, ny=8, pitch=8e-6, wl=633e-9, v=B.PLAIN, out=p)
    if case == "null":
        args["y"] = None
    elif case == "nx":
        args["nx"] = 0
    elif case == "ny":
        args["ny"] = -3
    elif case == "n":
        args["n"] = -1
    elif case == "pitch":
        args["pitch"] = 0.0
    elif case == "wl":
        args["wl"] = -1.0
    elif case == "nan":
        args["pitch"] = float("nan")
    elif case == "variant":
        args["v"] = max(B.VARIANTS.values()) + 1
    elif case == "out":
        args["out"] = None
    elif case == "toolarge":
        args["nx"] = (1 << 20) + 1
    rc = lib.cgh_forward(args["x"], args["y"], args["z"], args["a"], args["n"], args["nx"],
                         args["ny"], args["pitch"], args["wl"], args["v"], args["out"], p,
                         1 << 30, None)
    assert rc == B.CGH_EINVAL
    # the allocation-free forward runs the same checks first
    rc = lib.cgh_forward_noalloc(args["x"], args["y"], args["z"], args["a"], args["n"],
                                 args["nx"], args["ny"], args["pitch"], args["wl"], args["v"],
                                 args["out"], None)
    assert rc == B.CGH_EINVAL
    # and so does the forward with a residual (target and residual elsewhere)
    rc = lib.cgh_forward_residual(args["x"], args["y"], args["z"], args["a"], args["n"],
                                  args["nx"], args["ny"], args["pitch"], args["wl"], args["v"],
                                  ctypes.c_void_p(512), args["out"], ctypes.c_void_p(768), p,
                                  1 << 30, None)
    assert rc == B.CGH_EINVAL


def test_forward_residual_rejects_missing_or_aliased_grids(lib):
    """cgh_forward_residual needs three distinct grids (target, hologram,
    residual) and the forward's workspace; all checked on the host."""
    from paper_1002_0916_amd import binding as B

    p = ctypes.c_void_p(256)
    t, h, r = ctypes.c_void_p(4096), ctypes.c_void_p(8192), ctypes.c_void_p(12288)

    def call(target, holo, res, ws=p, wsb=1 << 30):
        return lib.cgh_forward_residual(p, p, p, p, 100, 64, 64, 8e-6, 633e-9, B.COMPENSATED,
                                        target, holo, res, ws, wsb, None)

    for args in ((None, h, r), (t, None, r), (t, h, None), (t, h, h), (t, h, t), (t, t, r)):
        assert call(*args) == B.CGH_EINVAL, args
    need = lib.cgh_workspace_bytes(100, 64, 64, B.COMPENSATED, B.OP_FORWARD)
    assert call(t, h, r, p, need - 1) == B.CGH_EWORKSPACE
    assert call(t, h, r, None, need) == B.CGH_EWORKSPACE


def test_noalloc_rejects_problems_beyond_its_scratch(lib):
    """cgh_forward_noalloc refuses, on the host, any problem whose plan needs
    more than its static buffer; the compensated forward first drops its
    column table (the kernel forms those values itself)."""
    from paper_1002_0916_amd import binding as B

    p = ctypes.c_void_p(256)
    cap = B.NOALLOC_SCRATCH_BYTES
    assert lib.cgh_workspace_bytes(16384, 3840, 2160, B.PLAIN, B.OP_FORWARD) < cap
    # the compensated forward at 3840 x 2160, N = 16384: 142 MB of row table
    assert lib.cgh_workspace_bytes(16384, 3840, 2160, B.COMPENSATED, B.OP_FORWARD) > cap
    for v in (B.COMPENSATED, B.SEPARABLE, B.SEPARABLE_F16X3):
        rc = lib.cgh_forward_noalloc(p, p, p, p, 16384, 3840, 2160, 8e-6, 633e-9, v, p, None)
        assert rc == B.CGH_ETOOBIG, v
    # every variant fits at the paper's shape
    for v in set(B.VARIANTS.values()):
        assert lib.cgh_workspace_bytes(1024, 1920, 1024, v, B.OP_FORWARD) <= cap, v
    assert b"static buffer" in lib.cgh_strerror(B.CGH_ETOOBIG)


def test_workspace_too_small_or_misaligned(lib):
    from paper_1002_0916_amd import binding as B

    p = ctypes.c_void_p(256)
    need = lib.cgh_workspace_bytes(100, 64, 64, B.COMPENSATED, B.OP_FORWARD)
    rc = lib.cgh_forward(p, p, p, p, 100, 64, 64, 8e-6, 633e-9, B.COMPENSATED, p, p, need - 1,
                         None)
    assert rc == B.CGH_EWORKSPACE
    rc = lib.cgh_forward(p, p, p, p, 100, 64, 64, 8e-6, 633e-9, B.COMPENSATED, p, None, need,
                         None)
    assert rc == B.CGH_EWORKSPACE
    rc = lib.cgh_forward(p, p, p, p, 100, 64, 64, 8e-6, 633e-9, B.COMPENSATED, p,
                         ctypes.c_void_p(256 + 4), need, None)
    assert rc == B.CGH_EWORKSPACE
    need_b = lib.cgh_workspace_bytes(100, 64, 64, B.PLAIN, B.OP_BACKWARD)
    rc = lib.cgh_backward(p, p, p, p, 100, 64, 64, 8e-6, 633e-9, B.PLAIN, p, p, p, p, p, p,
                          need_b - 256, None)
    assert rc == B.CGH_EWORKSPACE
    need_d = lib.cgh_workspace_bytes(100, 64, 64, B.PLAIN, B.OP_FORWARD_F64)
    rc = lib.cgh_forward_f64(p, p, p, p, 100, 64, 64, 8e-6, 633e-9, p, p, need_d - 1, None)
    assert rc == B.CGH_EWORKSPACE


def test_backward_rejects_bad_arguments(lib):
    from paper_1002_0916_amd import binding as B

    p = ctypes.c_void_p(256)
    ok = dict(gh=p, gx=p, gy=p, gz=p, ga=p)
    for k in ok:
        args = dict(ok)
        args[k] = None
        rc = lib.cgh_backward(p, p, p, p, 10, 32, 32, 8e-6, 633e-9, B.PLAIN, args["gh"],
                              args["gx"], args["gy"], args["gz"], args["ga"], p, 1 << 30, None)
        assert rc == B.CGH_EINVAL, k
    bad = max(B.VARIANTS.values()) + 1
    rc = lib.cgh_backward(p, p, p, p, 10, 32, 32, 8e-6, 633e-9, bad, p, p, p, p, p, p, 1 << 30,
                          None)
    assert rc == B.CGH_EINVAL
    # n = 0 is a valid no-op that enqueues nothing
    rc = lib.cgh_backward(None, None, None, None, 0, 32, 32, 8e-6, 633e-9, B.PLAIN, p, None,
                          None, None, None, None, 0, None)
    assert rc == B.CGH_OK


def test_profile_read_rejects_bad_kernel(lib):
    from paper_1002_0916_amd import binding as B

    n = ctypes.c_int64(0)
    t = ctypes.c_double(0)
    assert lib.cgh_profile_read(-1, ctypes.byref(n), ctypes.byref(t)) == B.CGH_EINVAL
    assert lib.cgh_profile_read(B.KERNEL_COUNT, ctypes.byref(n), ctypes.byref(t)) == B.CGH_EINVAL
    assert lib.cgh_profile_read(0, None, ctypes.byref(t)) == B.CGH_EINVAL
    buf = (ctypes.c_float * 4)()
    each = lib.cgh_profile_read_each
    assert each(B.KERNEL_COUNT, ctypes.byref(n), ctypes.byref(t), buf, 4) == B.CGH_EINVAL
    assert each(0, ctypes.byref(n), ctypes.byref(t), buf, -1) == B.CGH_EINVAL
    assert each(0, ctypes.byref(n), ctypes.byref(t), None, 4) == B.CGH_EINVAL
    # nothing recorded (timing is off): zero launches, nothing written
    buf[0] = -1.0
    assert each(0, ctypes.byref(n), ctypes.byref(t), buf, 4) == B.CGH_OK
    assert n.value == 0 and t.value == 0.0 and buf[0] == -1.0


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1002_0916_amd import binding as B

    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(B.CGHError):
        B.load_library()


def test_binding_validates_tensors():
    import torch

    from paper_1002_0916_amd import binding as B

    if B._lib is None and not os.path.exists(B.LIB_PATH):
        pytest.skip("library not built")
    x = torch.zeros(4)
    with pytest.raises(ValueError):
        B.forward(x, x, x, x, 8, 8)  # CPU tensors are refused (no CPU path)
    with pytest.raises(ValueError):
        B.variant_id("fastest")


def test_header_compiles_and_links_as_c(tmp_path, lib):
    """include/cgh.h is self-contained C: the plain-C consumer builds with gcc
    against it and links against libcgh.so (run on the GPU in
    test_gpu_c_abi.py)."""
    import importlib.util
    import subprocess

    spec = importlib.util.spec_from_file_location(
        "c_abi_build", os.path.join(ROOT, "tests", "c_abi", "build.py"))
    c_build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(c_build)
    out = str(tmp_path / "check")
    subprocess.run(c_build.command(out), check=True)
    assert os.path.exists(out)
