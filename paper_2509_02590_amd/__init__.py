"""MI355X (gfx950) hot path of Well-Connected Clusters (arXiv 2509.02590).

The computation runs in hand-written HIP kernels behind the C ABI of include/wcc.h; this
package is only its Python binding (PyTorch supplies device memory and streams).
Importing it fails loudly when the library has not been built.
"""
from ._lib import (CRIT, EXEC, MODE, RECORD_DTYPE, Params, Stats, WccError, cluster_csr, lib,  # noqa: F401
                   make_csr, mincut_split, mincut_split_batch, params, release, threshold, wcc_run)

__all__ = ["wcc_run", "mincut_split", "mincut_split_batch", "cluster_csr", "threshold", "params",
           "WccError", "RECORD_DTYPE", "release"]
