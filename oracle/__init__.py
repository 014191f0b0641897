"""CPU FP64 oracle (test infrastructure only; see reference.py)."""

from .reference import (  # noqa: F401
    CSR,
    Factors,
    SolveResult,
    apply_alg2,
    apply_alg3,
    csr_from_scipy,
    dense_S,
    extract,
    factor,
    factor_problem,
    ilup,
    level_sets,
    levels,
    lower_solve,
    pcgls,
    prescale,
    to_csc,
    true_residual,
    upper_solve,
    validate,
)
