"""Python binding of libmsrep: the equal-nnz partitioned SpMV of msRep
(arXiv 2209.07552) on one MI355X.

This module only marshals arguments: torch tensors on the GPU are passed to
the C ABI (include/msrep.h) as raw device pointers together with torch's
current HIP stream.  Every step of the computation runs in the library's HIP
kernels; there is no CPU fallback.  Importing works without a GPU (for
building and for symbol checks); calling a compute entry point without a GPU
or without the built library raises.
"""
from __future__ import annotations

from ._abi import (  # noqa: F401
    BF16, COO, COO_ANY, COO_COL, CSC, CSR, F32, F64, PART_DTYPE, Mat, MsrepError, Partition, Tune, lib_path,
    load_library, msrep_autotune, msrep_build_partition, msrep_convert, msrep_last_error,
    msrep_lptr_bound, msrep_plan_create, SPLIT_NNZ, SPLIT_ROWS, msrep_serve, msrep_spmm, msrep_spmm_ws_bytes,
    msrep_spmv, msrep_spmv_batched, msrep_spmv_noalloc, msrep_spmv_noalloc_max_parts,
    msrep_spmv_prepare, msrep_spmv_prepared, msrep_spmv_ws_bytes, msrep_timing,
    msrep_timing_only, msrep_timing_read, msrep_probe_stream,
    msrep_validate, mat_from_csr, exported_symbols,
)
