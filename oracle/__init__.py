"""Plain CPU oracle for the Chebyshev--Jacobi transform.

TEST INFRASTRUCTURE ONLY: tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import this package; the product library
never does.  It shares no code with the HIP path.

`cjt_oracle.c` holds the arithmetic (long double, O(N^2) direct sums of the
paper's definitions); this module builds it with gcc and wraps it with ctypes.
"""
from .oracle import (  # noqa: F401
    build,
    forward,
    inverse,
    inverse_shifted,
    shift_coefficients,
    jacobi_to_jacobi,
    point_values,
    point_values_rows,
    jacobi_column,
    moments,
    cc_weights,
    norm_consts,
    version,
    default_threads,
)
