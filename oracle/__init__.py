"""CPU oracle for the stencil hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct numpy implementations of what the HIP path
computes, written from the paper (Brown et al., "Fortran performance
optimisation and auto-parallelisation by leveraging MLIR-based domain
specific abstractions in Flang", SC-W 2023) and from the readings recorded
with each function. Only the tests, the smoke check and the benchmark's CPU
baseline may import this package; the product path never does, and the
oracle shares no code with it (inputs come from ``synth``).

Arrays follow the halo-padded layout of ``synth``: shape (nz+2, ny+2, nx+2),
x fastest, interior at [1:-1, 1:-1, 1:-1]. Strided views (padded pitch) are
accepted everywhere.

The functions are written with numpy elementwise operators only, so the same
code also runs on object arrays (``fractions.Fraction`` for exact arithmetic,
or a counting scalar for flop counts) -- that is how the tests pin it.
"""

from .gauss_seidel import rbgs_half, rbgs_solve, rbgs_sweep, rbgs_sweeps, red_mask  # noqa: F401
from .stencil import (  # noqa: F401
    C6_F32,
    C6_F64,
    advect_source,
    interior,
    jacobi_solve,
    jacobi_sweep,
    jacobi_sweeps,
    neighbour_sum,
    pow2_scale,
    refined_solve,
    residual,
    residual_norm,
    residual_norm_f32_storage,
    stencil_apply,
    sweep_f32,
    zero_interior,
)
