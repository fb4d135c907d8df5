"""MI355X (gfx950) community-quality scoring: Q, Qds, the six measures of Section
II-B3, and the partition-comparison metrics of Section II-A, computed by hand-written
HIP kernels behind a C ABI (``include/cq.h``).  ``cq`` is the ctypes binding."""
from . import cq  # noqa: F401  (fails loudly if libcq.so has not been built)
from .cq import (  # noqa: F401
    CQError, Context, Graph, compare_partitions, score_partition,
)
