"""FP64 CPU oracle of the D2Q37 thermal LBM update (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It shares no code with the HIP library.
"""
from .d2q37 import (  # noqa: F401
    D, NPOP, WALL_ROWS, SHELL_REPS, velocity_set, solve_isotropy, constants,
    moments, equilibrium, collide, propagate, wall_factors, thermalise, bc,
    step, run, stored, step_stored, fp16dev_reference, encode_fp16dev, decode_fp16dev, gather_sites, step_sites, totals, interface_height, rt_fields,
    init_rt,
)
