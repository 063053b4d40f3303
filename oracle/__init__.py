"""FP64 CPU oracle of the short-range step (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import this package.  It shares no code with the GPU path: its
arithmetic lives in ``crk_oracle.c`` (plain C, double precision, OpenMP over
target particles) and the Python side below only marshals arrays, loops over
boxes and expands sampled targets to the neighbourhoods their outputs
depend on.
"""
from .oracle import (  # noqa: F401
    PARAMS, build, coefficients, density, gravity, hydro, integrate,
    kernel, grav_g, s2_force, neighbours, num_threads, step, step_sampled,
    STEP_PARAMS, timestep_bins, substep_cycle, s2_form_factor, pm_long_range,
    fof_labels, velocity_gradient, RECON, compatible_update,
    fof_properties,
)
