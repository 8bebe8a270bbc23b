"""FP64 CPU oracle for the direct point-source hologram sum (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The GPU library never imports it and shares no code with
it.
"""
from .cgh_oracle import (  # noqa: F401
    build,
    forward,
    forward_at,
    adjoint,
    library_path,
)
