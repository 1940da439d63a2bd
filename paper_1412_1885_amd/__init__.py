"""Randomized Tucker compression (RandTucker2i) and FFCP on MI355X.

Python binding of the C ABI in include/rtucker.h; every step of the method
runs in the HIP library ``librtucker.so`` built by
``python -m paper_1412_1885_amd.build``.  The library is loaded on first use
and its absence is an error (there is no CPU fallback).
"""

from ._binding import (  # noqa: F401
    RtError, NonFiniteInput, lib, version, status_string, last_error,
    tucker_desc, tucker_rand_workspace, tucker_rand, bf16_copy_shape,
    ffcp_desc, ffcp_workspace, ffcp, ffcp_noalloc, ffcp_dense_workspace, ffcp_dense, ttm, cp_fit_dense,
    rt_tucker_rand, rt_ffcp, rt_ttm, rt_cp_fit_dense, rt_stream_pass,
    stream_pass, profile_enable, profile_read,
    sequential_desc, tucker_sequential, gaussian_matrix,
    LIB_PATH, TUCKER_INFO_DTYPE, FFCP_INFO_DTYPE,
    MLP, mlp_desc,
)
