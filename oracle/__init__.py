"""FP64 CPU oracle of the HLBM sweep -- test infrastructure only.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg
of ``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never does, and this package never imports the product.

The arithmetic lives in ``hlbm_oracle.c`` (plain scalar FP64 loops); this module
only compiles it and marshals numpy arrays across ctypes.
"""
from .oracle import (  # noqa: F401
    OracleConfig,
    build,
    collide_cell,
    equilibrium,
    lattice,
    max_threads,
    moments,
    observe,
    run,
    stream,
    collide,
    collide_adjoint,
    stream_adjoint,
    moments_adjoint,
    gradient,
    collide_cell_tensor,
    collide_tensor,
    run_tensor,
    collide_adjoint_tensor,
    gradient_tensor,
    stream_masked,
    run_masked,
    observe_masked,
    PERIODIC,
    WALL,
    INLET_U,
    OUTLET_RHO,
)
