"""MI355X (gfx950) stencil composition: exact composition of finite-difference
stencils and their matrix-free application in HIP kernels, inside CG solves
of a biharmonic boundary-value problem and of an implicit Cahn-Hilliard step.

The public calls mirror the C ABI in ``include/scomp.h``:
``compose_stencil``, ``apply_composed``, ``solve_biharmonic``, ``ch_step``.
"""

from ._native import (  # noqa: F401
    ApplyPlan,
    Csr,
    SC_BC_HALO,
    SC_BC_PERIODIC,
    SC_CSR_ADAPTIVE,
    SC_CSR_PERIODIC,
    SC_CSR_ROWSPLIT,
    SC_CSR_ZERO_RING,
    SC_PC_FASTPOISSON,
    SC_PC_NONE,
    SC_PREC_F32_IR,
    SC_PREC_F32_RU,
    SC_PREC_F64,
    SC_REQ_BVP,
    SC_REQ_CH_STEP,
    ScError,
    Server,
    SolveStats,
    Stencil,
    apply_composed,
    apply_varcoef,
    ch_step,
    compose_stencil,
    grid_diagnostics,
    grid_of,
    solve_biharmonic,
    solve_biharmonic_batch,
    spinodal_energy,
    spinodal_params,
    spinodal_steps,
    stencil_lincomb,
    version,
)
from . import stencils  # noqa: F401
