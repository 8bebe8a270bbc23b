"""Python binding of the HIP hologram library (``include/cgh.h``).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libcgh.so``.  PyTorch provides device memory (tensors and the
workspace) and the current stream.  If the library has not been built this
module raises on first use; there is no CPU fallback.

Functions mirror the C entry points:

    forward(x, y, z, a, nx, ny, pitch, wavelength, variant) -> I  [ny, nx] fp32
    forward_f64(x, y, z, a, nx, ny, pitch, wavelength)        -> I  [ny, nx] fp64
    backward(x, y, z, a, grad, nx, ny, pitch, wavelength, variant)
                                                   -> (gx, gy, gz, ga) fp32 [n]
    forward_noalloc(x, y, z, a, nx, ny, pitch, wavelength, variant, out)
                         (cgh_forward_noalloc: no workspace, static scratch)

and ``CGHFunction`` wraps forward/backward as a ``torch.autograd.Function``
differentiable in x, y, z (metres) and a.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcgh.so")

CGH_OK, CGH_EINVAL, CGH_EWORKSPACE, CGH_EHIP, CGH_ETOOBIG = 0, 1, 2, 3, 4
NOALLOC_SCRATCH_BYTES = 64 << 20
PLAIN, COMPENSATED, SEPARABLE = 0, 1, 2
SEPARABLE_F16X3, SEPARABLE_F16, SEPARABLE_BF16 = 3, 4, 5
RECURRENCE = 6
SEPARABLE_IDS = (SEPARABLE, SEPARABLE_F16X3, SEPARABLE_F16, SEPARABLE_BF16)
OP_FORWARD, OP_FORWARD_F64, OP_BACKWARD = 0, 1, 2
KERNEL_FWD_PLAIN, KERNEL_FWD_COMPENSATED, KERNEL_FWD_F64 = 0, 1, 2
KERNEL_ADJ_PLAIN, KERNEL_ADJ_COMPENSATED = 3, 4
KERNEL_FWD_SEPARABLE, KERNEL_ADJ_SEPARABLE = 5, 6
KERNEL_FWD_RECURRENCE, KERNEL_ADJ_RECURRENCE = 7, 8
KERNEL_COUNT = 9

VARIANTS = {"plain": PLAIN, "fast": PLAIN, "compensated": COMPENSATED, "comp": COMPENSATED,
            "separable": SEPARABLE, "separable_f16x3": SEPARABLE_F16X3,
            "separable_f16": SEPARABLE_F16, "separable_bf16": SEPARABLE_BF16,
            "recurrence": RECURRENCE}

EXPORTED = ("cgh_workspace_bytes", "cgh_forward", "cgh_forward_f64", "cgh_backward",
            "cgh_strerror", "cgh_version", "cgh_profile_enable", "cgh_profile_read",
            "cgh_profile_read_each", "cgh_forward_noalloc", "cgh_forward_residual")

_lib = None
_lock = threading.Lock()


class CGHError(RuntimeError):
    pass


def load_library():
    """Loads ``libcgh.so`` (raises if it is missing: no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise CGHError("libcgh.so is not built (%s); run __graft_entry__.build() or "
                           "python paper_1002_0916_amd/build.py" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        lib.cgh_workspace_bytes.argtypes = [i64, i32, i32, i32, i32]
        lib.cgh_workspace_bytes.restype = ctypes.c_size_t
        lib.cgh_forward.argtypes = [vp, vp, vp, vp, i64, i32, i32, f64, f64, i32, vp, vp,
                                    ctypes.c_size_t, vp]
        lib.cgh_forward.restype = ctypes.c_int
        lib.cgh_forward_noalloc.argtypes = [vp, vp, vp, vp, i64, i32, i32, f64, f64, i32, vp,
                                            vp]
        lib.cgh_forward_noalloc.restype = ctypes.c_int
        lib.cgh_forward_residual.argtypes = [vp, vp, vp, vp, i64, i32, i32, f64, f64, i32, vp,
                                             vp, vp, vp, ctypes.c_size_t, vp]
        lib.cgh_forward_residual.restype = ctypes.c_int
        lib.cgh_forward_f64.argtypes = [vp, vp, vp, vp, i64, i32, i32, f64, f64, vp, vp,
                                        ctypes.c_size_t, vp]
        lib.cgh_forward_f64.restype = ctypes.c_int
        lib.cgh_backward.argtypes = [vp, vp, vp, vp, i64, i32, i32, f64, f64, i32, vp, vp, vp,
                                     vp, vp, vp, ctypes.c_size_t, vp]
        lib.cgh_backward.restype = ctypes.c_int
        lib.cgh_strerror.argtypes = [ctypes.c_int]
        lib.cgh_strerror.restype = ctypes.c_char_p
        lib.cgh_version.argtypes = []
        lib.cgh_version.restype = ctypes.c_int
        lib.cgh_profile_enable.argtypes = [i32]
        lib.cgh_profile_enable.restype = ctypes.c_int
        lib.cgh_profile_read.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(f64)]
        lib.cgh_profile_read.restype = ctypes.c_int
        lib.cgh_profile_read_each.argtypes = [i32, ctypes.POINTER(i64), ctypes.POINTER(f64),
                                              ctypes.POINTER(ctypes.c_float), i64]
        lib.cgh_profile_read_each.restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != CGH_OK:
        raise CGHError("cgh: %s (status %d)" % (load_library().cgh_strerror(rc).decode(), rc))


def variant_id(variant) -> int:
    if isinstance(variant, int):
        if variant not in set(VARIANTS.values()):
            raise ValueError("unknown variant %r" % variant)
        return variant
    try:
        return VARIANTS[variant]
    except KeyError:
        raise ValueError("unknown variant %r (%s)" % (variant, "|".join(VARIANTS))) from None


def workspace_bytes(n: int, nx: int, ny: int, variant=COMPENSATED, op: int = OP_FORWARD) -> int:
    return int(load_library().cgh_workspace_bytes(int(n), int(nx), int(ny),
                                                 variant_id(variant), int(op)))


# One workspace per (device, stream); calls on one stream are ordered, so
# they may share it.
_workspaces: dict = {}


def _workspace(device: torch.device, stream, nbytes: int):
    if nbytes == 0:
        return None, 0
    key = (device.index, stream.cuda_stream)
    buf = _workspaces.get(key)
    if buf is None or buf.numel() < nbytes:
        with torch.cuda.stream(stream):
            buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _workspaces[key] = buf
    return buf.data_ptr(), buf.numel()


def release_workspaces():
    _workspaces.clear()


def _points(x, y, z, a):
    ts = (x, y, z, a)
    for name, t in zip("xyza", ts):
        if not isinstance(t, torch.Tensor):
            raise ValueError("%s must be a torch tensor" % name)
        if t.dtype != torch.float32 or t.dim() != 1 or not t.is_contiguous():
            raise ValueError("%s must be a contiguous 1-D float32 tensor" % name)
        if t.device.type != "cuda":
            raise ValueError("%s must be on a HIP device" % name)
    n = x.shape[0]
    dev = x.device
    for name, t in zip("yza", ts[1:]):
        if t.shape[0] != n or t.device != dev:
            raise ValueError("%s must match x in length and device" % name)
    return n, dev


def _sizes(nx, ny):
    nx, ny = int(nx), int(ny)
    if nx < 1 or ny < 1:
        raise ValueError("nx and ny must be >= 1")
    return nx, ny


def forward(x, y, z, a, nx: int, ny: int, pitch: float = 8e-6, wavelength: float = 633e-9,
            variant="compensated", out: torch.Tensor | None = None) -> torch.Tensor:
    """Hologram I[ny, nx] (float32) of Eq. (1) computed by the HIP kernels."""
    lib = load_library()
    n, dev = _points(x, y, z, a)
    nx, ny = _sizes(nx, ny)
    v = variant_id(variant)
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    elif (out.dtype != torch.float32 or out.device != dev or not out.is_contiguous()
          or out.numel() != nx * ny):
        raise ValueError("out must be a contiguous float32 tensor of ny*nx on x's device")
    stream = torch.cuda.current_stream(dev)
    ws, wsb = _workspace(dev, stream, workspace_bytes(n, nx, ny, v, OP_FORWARD))
    _check(lib.cgh_forward(x.data_ptr(), y.data_ptr(), z.data_ptr(), a.data_ptr(), n, nx, ny,
                           float(pitch), float(wavelength), v, out.data_ptr(), ws, wsb,
                           stream.cuda_stream))
    return out


def forward_residual(x, y, z, a, target: torch.Tensor, nx: int, ny: int, pitch: float = 8e-6,
                     wavelength: float = 633e-9, variant="compensated",
                     out: torch.Tensor | None = None,
                     residual: torch.Tensor | None = None) -> tuple[torch.Tensor, torch.Tensor]:
    """(I, I - target) through ``cgh_forward_residual``: I as ``forward``, and
    the residual (the upstream gradient of 0.5 ||I - T||^2) in the same call."""
    lib = load_library()
    n, dev = _points(x, y, z, a)
    nx, ny = _sizes(nx, ny)
    v = variant_id(variant)

    def grid(t, name):
        if t is None:
            return torch.empty((ny, nx), dtype=torch.float32, device=dev)
        if (t.dtype != torch.float32 or t.device != dev or not t.is_contiguous()
                or t.numel() != nx * ny):
            raise ValueError("%s must be a contiguous float32 tensor of ny*nx on x's device"
                             % name)
        return t

    if target is None:
        raise ValueError("target is required")
    target = grid(target, "target")
    out = grid(out, "out")
    residual = grid(residual, "residual")
    stream = torch.cuda.current_stream(dev)
    ws, wsb = _workspace(dev, stream, workspace_bytes(n, nx, ny, v, OP_FORWARD))
    _check(lib.cgh_forward_residual(x.data_ptr(), y.data_ptr(), z.data_ptr(), a.data_ptr(), n,
                                    nx, ny, float(pitch), float(wavelength), v,
                                    target.data_ptr(), out.data_ptr(), residual.data_ptr(), ws,
                                    wsb, stream.cuda_stream))
    return out, residual


def forward_noalloc(x, y, z, a, nx: int, ny: int, pitch: float = 8e-6,
                    wavelength: float = 633e-9, variant="compensated",
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """As ``forward`` through ``cgh_forward_noalloc``: the library takes no
    workspace (its scratch is a static device buffer of
    NOALLOC_SCRATCH_BYTES per GPU).  Pass ``out`` to allocate nothing at all
    (e.g. under graph capture).  Calls that overlap on one GPU race."""
    lib = load_library()
    n, dev = _points(x, y, z, a)
    nx, ny = _sizes(nx, ny)
    v = variant_id(variant)
    if out is None:
        out = torch.empty((ny, nx), dtype=torch.float32, device=dev)
    elif (out.dtype != torch.float32 or out.device != dev or not out.is_contiguous()
          or out.numel() != nx * ny):
        raise ValueError("out must be a contiguous float32 tensor of ny*nx on x's device")
    stream = torch.cuda.current_stream(dev)
    _check(lib.cgh_forward_noalloc(x.data_ptr(), y.data_ptr(), z.data_ptr(), a.data_ptr(), n,
                                   nx, ny, float(pitch), float(wavelength), v, out.data_ptr(),
                                   stream.cuda_stream))
    return out


def forward_f64(x, y, z, a, nx: int, ny: int, pitch: float = 8e-6,
                wavelength: float = 633e-9) -> torch.Tensor:
    """Hologram I[ny, nx] (float64) from the FP64 HIP kernel."""
    lib = load_library()
    n, dev = _points(x, y, z, a)
    nx, ny = _sizes(nx, ny)
    out = torch.empty((ny, nx), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev)
    ws, wsb = _workspace(dev, stream, workspace_bytes(n, nx, ny, PLAIN, OP_FORWARD_F64))
    _check(lib.cgh_forward_f64(x.data_ptr(), y.data_ptr(), z.data_ptr(), a.data_ptr(), n, nx,
                               ny, float(pitch), float(wavelength), out.data_ptr(), ws, wsb,
                               stream.cuda_stream))
    return out


def backward(x, y, z, a, grad, nx: int, ny: int, pitch: float = 8e-6,
             wavelength: float = 633e-9, variant="compensated"):
    """(dL/dx, dL/dy, dL/dz [per metre], dL/dA) for G = dL/dI ``grad`` [ny, nx]."""
    lib = load_library()
    n, dev = _points(x, y, z, a)
    nx, ny = _sizes(nx, ny)
    v = variant_id(variant)
    if (not isinstance(grad, torch.Tensor) or grad.dtype != torch.float32
            or grad.device != dev or tuple(grad.shape) != (ny, nx)):
        raise ValueError("grad must be a float32 tensor of shape (ny, nx) on x's device")
    grad = grad.contiguous()
    gx, gy, gz, ga = (torch.empty(n, dtype=torch.float32, device=dev) for _ in range(4))
    stream = torch.cuda.current_stream(dev)
    ws, wsb = _workspace(dev, stream, workspace_bytes(n, nx, ny, v, OP_BACKWARD))
    _check(lib.cgh_backward(x.data_ptr(), y.data_ptr(), z.data_ptr(), a.data_ptr(), n, nx, ny,
                            float(pitch), float(wavelength), v, grad.data_ptr(), gx.data_ptr(),
                            gy.data_ptr(), gz.data_ptr(), ga.data_ptr(), ws, wsb,
                            stream.cuda_stream))
    return gx, gy, gz, ga


class CGHFunction(torch.autograd.Function):
    """I = CGHFunction.apply(x, y, z, a, nx, ny, pitch, wavelength, variant).

    Differentiable in x, y (pixels), z (metres) and a; the backward pass is
    ``cgh_backward``.
    """

    @staticmethod
    def forward(ctx, x, y, z, a, nx, ny, pitch=8e-6, wavelength=633e-9, variant="compensated"):
        ctx.save_for_backward(x, y, z, a)
        ctx.cfg = (int(nx), int(ny), float(pitch), float(wavelength), variant)
        return forward(x, y, z, a, nx, ny, pitch, wavelength, variant)

    @staticmethod
    def backward(ctx, grad):
        x, y, z, a = ctx.saved_tensors
        nx, ny, pitch, wavelength, variant = ctx.cfg
        gx, gy, gz, ga = backward(x, y, z, a, grad.contiguous(), nx, ny, pitch, wavelength,
                                  variant)
        return gx, gy, gz, ga, None, None, None, None, None


def profile_enable(on: bool = True):
    _check(load_library().cgh_profile_enable(1 if on else 0))


def profile_read(kernel: int):
    """(launches, total_ms) recorded for ``kernel`` since the last read."""
    launches = ctypes.c_int64(0)
    total = ctypes.c_double(0.0)
    _check(load_library().cgh_profile_read(int(kernel), ctypes.byref(launches),
                                           ctypes.byref(total)))
    return int(launches.value), float(total.value)


def profile_read_each(kernel: int, capacity: int = 4096):
    """Per-launch durations (ms, launch order) recorded for ``kernel`` since
    the last read (at most ``capacity`` of them)."""
    launches = ctypes.c_int64(0)
    total = ctypes.c_double(0.0)
    buf = (ctypes.c_float * max(capacity, 1))()
    _check(load_library().cgh_profile_read_each(int(kernel), ctypes.byref(launches),
                                                ctypes.byref(total), buf, int(capacity)))
    return [float(buf[i]) for i in range(min(int(launches.value), capacity))]
