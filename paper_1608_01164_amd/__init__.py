"""hQDWH on MI355X: spectral projectors of symmetric banded matrices in HODLR format.

Thin Python binding over the C ABI in ``include/hq.h`` (library ``libhqdwh.so`` next to this file).
Every step of the computation runs in the library's HIP kernels; this package only marshals
arguments (torch tensors are used for device memory and streams).  Importing it does not load the
library; the first call does, and raises if the library has not been built.
"""
from .binding import (  # noqa: F401
    HODLR, Info, Opts, LibraryMissing, HQError, lib, hodlr_build, qdwh_sign, spectral_projector,
    spectral_projector_batched,
    shift_for_count, test_gemm, test_qr_r, test_recompress, test_from_dense, test_product,
    test_cholesky_inverse, test_q_factors, test_q_dense_host, profile, profile_read, KCLASSES,
    Predictor, predictor_rows, tuning, set_tuning, HMatrix, hodlr_to_hmatrix, iteration_records,
    cholesky_solve,
)
