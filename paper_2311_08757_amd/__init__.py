"""MI355X library for the smallest eigenpair of periodic Schroedinger operators
on anisotropically long boxes: sigma-shifted inverse iteration with CG
preconditioned by two-level additive Schwarz and the PerFact coarse space
(Theisen & Stamm, arXiv 2311.08757).  The compute path is the HIP library
libddeig.so (include/ddeig.h); this package only binds it."""
from .ddeig import (assemble, cell_shift, set_shift, debug_force_breakdown, apply_op, apply_precond, pcg_solve,
                    apply_schwarz, stationary_ras, gmres_solve, PREC_KINDS,
                    inverse_iteration, lopcg, profile_kernel, profile_iteration,
                    ITERATION_PARTS, potential_form, potential_form_noalloc, query,
                    eig_grad, shift_grad, solve_grad, batch_eig_grad, batch_solve_grad,
                    Batch, batch_create, batch_query, batch_pcg_solve, batch_inverse_iteration, status_string, load_library, DdeigError, Problem,
                    EXPORTS, LIB_PATH)

__all__ = ["assemble", "cell_shift", "set_shift", "debug_force_breakdown", "apply_op", "apply_precond", "pcg_solve",
           "apply_schwarz", "stationary_ras", "gmres_solve", "PREC_KINDS",
           "inverse_iteration", "lopcg", "profile_kernel", "profile_iteration",
           "ITERATION_PARTS", "potential_form", "potential_form_noalloc", "eig_grad",
           "shift_grad", "solve_grad", "batch_eig_grad", "batch_solve_grad", "query", "Batch", "batch_create",
           "batch_query", "batch_pcg_solve", "batch_inverse_iteration", "status_string", "load_library", "DdeigError",
           "Problem", "EXPORTS", "LIB_PATH"]
