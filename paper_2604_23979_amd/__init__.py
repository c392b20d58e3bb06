"""MI355X-native preconditioned Krylov solver for interior-point-method linear
systems: block-Jacobi (filtered, diagonally corrected, ILU(0)-factored blocks)
preconditioned CG in FP64 or FP32-inner / FP64-refined form, GMRES(m),
BiCGSTAB, GCR(m), and the
bordered-block-diagonal preconditioner with a dense Schur complement, behind
the C ABI of include/sdsl.h.  This package is the binding of that library."""
from ._binding import (BBD, BICGSTAB, BJ, FACT_COMPLETE, FACT_ILU0, GCR, Group, DIAG_DELTA, DIAG_DROPSUM, E_BREAKDOWN, E_DEVICE, E_INVALID, E_NOMEM,
                       E_NOT_CONVERGED, E_STATE, E_STRUCTURE, FILTER_GEOMEAN, FILTER_MIN, FILTER_NONE, FP32_IR,
                       FP32_IR_RESTART,
                       FP64, GMRES, OK, PCG, PIVOT_FAIL, PIVOT_REPLACE, PIVOT_SHIFT, SIGNATURES, LIB_PATH, Options,
                       SdslError, Solver, lib, solve_batch, torch_allocator)


def from_system(sys_, options=None, stream=None, torch_memory=True):
    """Solver for an object carrying row_ptr, col, val, block_ptr, n_border
    and lowrank (such as the seeded inputs' System)."""
    return Solver(sys_.row_ptr, sys_.col, sys_.val, sys_.block_ptr, n_border=getattr(sys_, "n_border", 0),
                  lowrank=getattr(sys_, "lowrank", None), options=options, stream=stream,
                  torch_memory=torch_memory)
