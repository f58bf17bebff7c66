"""Shared test helpers: workload construction (inputs only) and comparisons."""

from __future__ import annotations

import re
import os

import numpy as np

from workloads import codes, check_permutations
from workloads.configs import WORKLOADS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    """Function names declared in include/mbbp.h."""
    with open(os.path.join(ROOT, "include", "mbbp.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(mbbp_[a-z_]+)\s*\(", text)))


def perms_for(h: np.ndarray, wl) -> np.ndarray:
    count = max(wl.L, 8)
    return check_permutations(h.shape[0], count, seed=wl.perm_seed)


def bases_for(h: np.ndarray, wl, builder):
    """Representations of h for workload wl, built by `builder` (oracle or library)."""
    return builder(h, wl.basis_mode, wl.L, perms_for(h, wl))


def f32(x: float) -> float:
    return float(np.float32(x))


def tie_shots(margin: np.ndarray, thresh: float = 1e-3) -> np.ndarray:
    """(shot, representation) instances whose FP64 run came within `thresh` of a sign
    flip at some evaluated sign or decision."""
    return (margin[..., 0] < thresh) | (margin[..., 1] < thresh)
