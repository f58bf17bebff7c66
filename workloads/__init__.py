"""Seeded input generators shared by the oracle tests, the GPU tests and the bench.

This package holds inputs only: CSS code definitions (parity-check matrices),
seeded permutations of the check nodes, and the batch shapes of each workload.
It contains none of the decoder's arithmetic (no BP, no subtree search, no
selection, no failure test, no noise sampler); both the oracle and the HIP
library receive what is generated here as plain arrays.
"""

from .codes import (  # noqa: F401
    CSSCode,
    bb_code,
    bb72,
    bb144,
    bb288,
    qc882,
    steane7,
    surface13,
    toric18,
    fig2_matrix,
    to_csr,
)
from .perms import check_permutations  # noqa: F401
from .configs import WORKLOADS, workload  # noqa: F401
