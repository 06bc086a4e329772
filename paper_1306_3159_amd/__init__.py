"""blob_rd: MI355X (gfx950) linear solves of the reactive blob model of arXiv:1306.3159.

The compute path is the HIP library ``libblob_rd.so`` (C ABI declared in
``include/blob_rd.h``). This package only marshals arguments: PyTorch
provides device memory and streams, every step of a solve runs in the
library's kernels. There is no CPU fallback: if the library is missing the
import of :mod:`paper_1306_3159_amd.native` fails loudly.
"""
from .native import (BlobRD, Net, NET_PARAMS, Batch, solve_streams, solve_batched, weights_blob, blob_params,
                     PRECOND_BLOB_BYTES, BlobRDError, NotConverged, Stats,
                     load_library, FP64, MIXED, PRECOND_NONE, PRECOND_DIAGONAL, PRECOND_LEARNED, SOLVER_SCHUR,
                     SOLVER_BLOCK, SOLVER_BLOCK_LEARNED, BOUNDARY_PERIODIC, BOUNDARY_DIRICHLET)

__all__ = ["BlobRD", "Net", "NET_PARAMS", "Batch", "solve_streams", "solve_batched", "weights_blob", "blob_params",
           "PRECOND_BLOB_BYTES", "BlobRDError", "NotConverged", "Stats",
           "load_library", "FP64", "MIXED", "PRECOND_NONE", "PRECOND_DIAGONAL", "PRECOND_LEARNED", "SOLVER_SCHUR",
           "SOLVER_BLOCK", "SOLVER_BLOCK_LEARNED", "BOUNDARY_PERIODIC", "BOUNDARY_DIRICHLET"]
