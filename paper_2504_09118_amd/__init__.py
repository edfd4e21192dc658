"""MI355X (gfx950) Yee FDTD leapfrog for PEC box cavities.

The compute lives in libfdtd.so (hand-written HIP kernels behind the C ABI of
include/fdtd.h); this package only binds it. See ``fdtd.Solver`` for one
cavity and ``fdtd.Pool`` for continuous batching of many; ``serve`` drives a
pool with a Poisson request stream.
"""

from .fdtd import (  # noqa: F401
    DIAG_NAMES,
    FIELD_NAMES,
    KERNELS,
    FdtdError,
    Pool,
    Solver,
    field_shapes,
    load_library,
    required_bytes,
)
