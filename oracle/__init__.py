"""Plain FP64 CPU oracle for SPMESL -- test infrastructure only.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the HIP library:
the arithmetic lives in ``spmesl_oracle.c`` (plain C, compiled with gcc) and
this package only builds and calls it.
"""
from .api import (  # noqa: F401
    build, lib_path, standardize, scaled_lasso, spmesl, spmesl_columns, spmesl_subset,
    symmetrize, lambda_ub, lambda_univ, lambda_pb,
)
