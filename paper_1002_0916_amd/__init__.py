"""MI355X-native direct point-source computer-generated hologram library.

Computes Eq. (1) of Shimobaba et al., "Fast calculation of
computer-generated-hologram on AMD HD5000 series GPU and OpenCL" (Section 1),

    I(x_h, y_h) = sum_j A_j cos(P_j ((x_h - x_j)^2 + (y_h - y_j)^2)),
    P_j = pi p^2 / (lambda z_j),

and its adjoint, with hand-written HIP kernels for gfx950 behind a C ABI
(``include/cgh.h``).  The Python side (``binding``) only marshals arguments.

Submodules are imported lazily so that ``workloads`` can be used without the
GPU library.
"""

__all__ = ["binding", "workloads"]


def __getattr__(name):
    if name in __all__:
        import importlib

        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
