"""FP64 CPU oracle for shifted Cholesky QR and the block append.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The HIP library never uses it, and
it never uses the HIP library.
"""
from .cholqr import (  # noqa: F401
    U64, OK, NOT_CONVERGED, BREAKDOWN, ENONFINITE, RECOMPUTE, NO_SHIFT, FIXED, VARIANTS,
    gram, gram_append, schur, fro_dist_identity, lambda_max, shift_orth,
    shift_append_first, cholesky_upper, apply_inverse, default_opts, orth,
    append, panel, loo, rrr, rcr,
)
