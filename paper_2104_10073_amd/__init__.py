"""Multi-function direct Monte Carlo integration on MI355X (gfx950).

The method (ZMCintegral multi-function integrations): many integrands that
differ in form, dimension and box domain, each integrated by direct Monte
Carlo, each result a value with a standard error.  The work runs in the HIP
library ``libzmc.so`` (C ABI in ``include/zmc.h``); this package is its
binding plus the seeded workload generator.
"""

from . import runs, workloads
from ._native import (GRID_AXIS_DTYPE, MC_FAMILY_USER0, MC_MAX_GRID_AXES, MC_MAX_USER_FAMILIES, MC_NO_GRAPH, MC_NO_PROMOTE, MC_RESIDENT, MC_SCHED_FAIR, MC_SCHED_FIFO, MC_SCHED_SRPT, MC_VALIDATE_ONLY, PREC_FP32, PREC_FP64, RESULT_DTYPE, Context, McError,
                      load, segment_samples, version)

__all__ = ["runs", "workloads", "Context", "GRID_AXIS_DTYPE", "MC_MAX_GRID_AXES", "MC_FAMILY_USER0", "MC_MAX_USER_FAMILIES", "McError", "PREC_FP32", "PREC_FP64", "RESULT_DTYPE", "MC_NO_GRAPH",
           "MC_VALIDATE_ONLY", "MC_NO_PROMOTE", "MC_RESIDENT", "MC_SCHED_FAIR", "MC_SCHED_FIFO", "MC_SCHED_SRPT", "load", "segment_samples", "version"]
