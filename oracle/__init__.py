"""CPU FP64 oracle (test infrastructure only; see ``oracle.condensed_ipm``)."""
from .condensed_ipm import (  # noqa: F401
    Reduced, Result, reduce_problem, reduce_general, inputs, condensed_step, condensed_matrix, residuals,
    fraction_to_boundary, kkt_error, initial_point, solve, simulate, sparse_objective,
    objective, STATUS_CONVERGED, STATUS_MAX_ITER, STATUS_SMALL_STEP,
)
