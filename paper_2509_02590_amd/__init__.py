"""MI355X (gfx950) hot path of Well-Connected Clusters (arXiv 2509.02590).

The computation runs in hand-written HIP kernels behind the C ABI of include/wcc.h; this
package is only its Python binding (PyTorch supplies device memory and streams).
Importing it fails loudly when the library has not been built.
"""
from ._lib import (CRIT, EXEC, MODE, RECORD_DTYPE, ExecConfig, Params, Stats, WccError, autotune,  # noqa: F401
                   ccr_components, cluster_csr, cm_run, cda,
                   get_exec_config, lib, make_csr, mincut_split, mincut_split_batch, params, release,
                   Server, set_exec_config, threshold, wcc_run)

__all__ = ["wcc_run", "mincut_split", "mincut_split_batch", "cluster_csr", "threshold", "params",
           "WccError", "RECORD_DTYPE", "release", "get_exec_config", "set_exec_config", "autotune", "Server", "ccr_components",
           "cm_run", "cda"]
