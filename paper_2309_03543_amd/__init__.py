"""MI355X corrector-system library for the one-domain Navier-Stokes-Brinkman
solver of arXiv 2309.03543: GPU assembly and PCG of the two corrector systems
behind a C ABI (include/pmcorr.h), with a thin Python binding."""
from . import binding  # noqa: F401
from .binding import (  # noqa: F401
    PM_CP1X, PM_CP1Y, PM_CP2, PM_FP64, PM_MIXED, Batch, Mesh, PMError, assemble_corrector,
    pcg_adjoint, pcg_solve, pcg_solve_batched, pm_batch_create, pm_mesh_create, pm_structure_host,
    pm_last_launch, pm_time_kernel, cp2_cross_rhs, cp2_solve_two_step, pm_time_cross,
    cp1_solve_coupled, cp1_solve_coupled_pcg, flux_average, rt0_update,
)
