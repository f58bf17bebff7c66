"""The benchmark and parity workloads: code, number of bases L, iteration cap T,
normalisation alpha, error rates, shot counts and seeds.

Noise is code-capacity depolarizing: each qubit independently suffers X, Y or Z
with probability p/3 each.  X and Z parts are decoded separately.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, Tuple

from . import codes


@dataclasses.dataclass(frozen=True)
class Workload:
    key: str
    code: Callable[[], "codes.CSSCode"]
    L: int
    T: int
    alpha: float
    ps: Tuple[float, ...]
    shots: int
    seed: int
    basis_mode: str  # "subtrees": distinct maximal subtrees; "ramp": uneven prefixes
    perm_seed: int = 0
    description: str = ""


WORKLOADS = {
    "bb72_L4_T20": Workload(
        "bb72_L4_T20", codes.bb72, L=4, T=20, alpha=0.75, ps=(0.05,), shots=10_000,
        seed=1, basis_mode="subtrees",
        description="[[72,12,6]] BB, p=0.05, L=4 subtree bases, T=20, alpha=0.75"),
    "bb144_L16_T50": Workload(
        "bb144_L16_T50", codes.bb144, L=16, T=50, alpha=0.875,
        ps=(0.02, 0.04, 0.06, 0.08), shots=1_000_000, seed=1, basis_mode="subtrees",
        description="[[144,12,12]] BB, L=16 subtree bases, T=50, alpha=0.875"),
    "bb288_L32_T100": Workload(
        "bb288_L32_T100", codes.bb288, L=32, T=100, alpha=0.875, ps=(0.03,),
        shots=10_000_000, seed=1, basis_mode="ramp",
        description="[[288,12,18]] BB, L=32 uneven bases (0..m rows), T=100"),
    "qc882_L64_T100": Workload(
        "qc882_L64_T100", codes.qc882, L=64, T=100, alpha=0.875,
        ps=(0.01, 0.02, 0.03), shots=1_000_000, seed=1, basis_mode="ramp",
        description="n=882 k=24 QC stand-in, L=64 uneven bases, T=100"),
    "bb144_weighted_T25": Workload(
        "bb144_weighted_T25", codes.bb144, L=16, T=25, alpha=0.875, ps=(0.05,),
        shots=1_000_000, seed=1, basis_mode="subtrees",
        description="[[144,12,12]] weighted BP, T=25 unrolled, L=16"),
}


def workload(key: str) -> Workload:
    return WORKLOADS[key]
