"""CPU FP64 oracle for the adaptive s-step CG method (TEST INFRASTRUCTURE).

This package is test infrastructure, not part of the product: only the
tests, the smoke check and the benchmark's CPU-baseline leg may import it.
The GPU library never calls it and shares no code with it.

It is a plain, slow, readable implementation of what the paper computes,
in numpy/scipy FP64:

* ``hscg``         -- Hestenes-Stiefel CG (Algorithm 1).
* ``ritz``         -- the Lanczos tridiagonal from the CG coefficients (1.1),
                      its Cholesky factor (4.1) and the incremental extremal
                      Ritz value estimates of Algorithms 3 and 4, plus the psi
                      recurrence (4.5).
* ``basis``        -- basis parameters (monomial, Newton/Leja (2.7),
                      Chebyshev (2.8)), the s-step basis (2.2)-(2.3) and the
                      change-of-basis matrix (2.5).
* ``sstep``        -- the improved adaptive s-step CG (Algorithm 5).

Columns of the s-step basis are kept in the paper's order Y = [P, R]
(P = s+1 columns, R = s columns).  Every place where the paper is silent or
inconsistent follows a documented reading; each is marked "Reading:" in the
code.
"""
from .hscg import hscg
from .ritz import (lanczos_tridiagonal, lanczos_cholesky_factor, MaxRitzEstimate,
                   MinRitzEstimate, psi_update)
from .basis import (leja_reference_points, params_monomial, params_newton,
                    params_chebyshev, make_params, polynomial_columns, sstep_basis,
                    change_of_basis, sub_indices)
from .sstep import adaptive_sstep_cg, select_stilde, UNIT_ROUNDOFF, Outcome

__all__ = [
    "hscg", "lanczos_tridiagonal", "lanczos_cholesky_factor", "MaxRitzEstimate",
    "MinRitzEstimate", "psi_update", "leja_reference_points", "params_monomial",
    "params_newton", "params_chebyshev", "make_params", "polynomial_columns",
    "sstep_basis", "change_of_basis", "sub_indices", "adaptive_sstep_cg", "select_stilde",
    "UNIT_ROUNDOFF", "Outcome",
]
