"""lgmg: unsmoothed-aggregation multigrid for graph Laplacians on one MI355X.

The method is that of Konolige & Brown, "A Parallel Solver for Graph
Laplacians" (PASC'18).  All arithmetic runs in the HIP library liblgmg.so
(C ABI in include/lgmg.h); :mod:`.lgmg` is its ctypes binding.
"""

from . import lgmg  # noqa: F401
from .lgmg import (  # noqa: F401
    LgError,
    lg_cycle,
    lg_default_opts,
    lg_export_coarsest,
    lg_export_level,
    lg_export_setup_data,
    lg_hierarchy_bytes,
    lg_hierarchy_stats,
    lg_profile_enable,
    lg_profile_read,
    lg_setup,
    lg_setup_ms,
    lg_solve,
    lg_spmv,
)
