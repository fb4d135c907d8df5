"""Parity bar between the library's outputs and the oracle's -- TEST INFRASTRUCTURE ONLY.

Integers (counts, tables) must match bit for bit.  A binary64 value g passes against the
oracle's o when

    |g - o| <= 1e-12 |o|   or   |g - o| <= 4 * 2^-52 * S

where S is the magnitude of the terms that cancel inside that value (Q = sum of
|E_c^in|/|E| minus sum of (D_c/2|E|)^2, so S <= 2; VI and NMI add entropy terms each at
most ln n; NVD is 1 minus a ratio).  Sums of terms of one sign and ratios of exact
integers have S = 0: they are held to 1e-12 relative alone.  The second bound only matters for values near zero: both sides carry a
rounding error of a few units of 2^-53 times S, whatever the order they sum in, so a
purely relative bar is meaningless there.  Per-community arrays take S per community
(0 for a single ratio of exact integers, so those are held to 1e-12 relative alone).
"""
from __future__ import annotations

import math

import numpy as np

REL = 1e-12
EPS4 = 4.0 * 2.0 ** -52

SCORE_INT = ("n", "m", "K", "num_pairs", "sum_ein", "sum_eout")
SCORE_FLT = ("Q", "Qds", "split_penalty", "mean_intra_edges", "mean_intra_density", "mean_contraction",
             "mean_inter_edges", "mean_expansion", "mean_conductance")
CMP_INT = ("n", "Ka", "Kb", "nnz", "a11", "a10", "a01", "a00", "A")
CMP_FLT = ("VI", "NMI", "F", "NVD", "RI", "ARI", "JI")

# magnitude of the cancelling terms of each scalar (see the module docstring); 0 for
# sums of terms of one sign and ratios of exact integers, which are held to 1e-12
# relative alone
SCORE_SCALE = {"Q": 2.0, "Qds": 3.0}


def cmp_scale(key: str, n: int) -> float:
    if key in ("VI", "NMI"):
        return 4.0 * math.log(max(n, 2))
    return {"ARI": 2.0, "NVD": 1.0}.get(key, 0.0)


def fclose(g: float, o: float, scale: float = 0.0) -> bool:
    if math.isnan(g) or math.isnan(o):
        return math.isnan(g) and math.isnan(o)
    return abs(g - o) <= max(REL * abs(o), EPS4 * scale)


def score_mismatches(gpu: dict, orc: dict) -> list[str]:
    bad = [f"{k}: gpu {gpu[k]} oracle {orc[k]}" for k in SCORE_INT if int(gpu[k]) != int(orc[k])]
    for k in SCORE_FLT:
        if not fclose(float(gpu[k]), float(orc[k]), SCORE_SCALE.get(k, 0.0)):
            bad.append(f"{k}: gpu {gpu[k]!r} oracle {orc[k]!r}")
    if gpu.get("device_flags", 0):
        bad.append(f"device_flags {gpu['device_flags']}")
    return bad


def compare_mismatches(gpu: dict, orc: dict) -> list[str]:
    bad = [f"{k}: gpu {gpu[k]} oracle {orc[k]}" for k in CMP_INT if int(gpu[k]) != int(orc[k])]
    n = int(orc["n"])
    for k in CMP_FLT:
        if not fclose(float(gpu[k]), float(orc[k]), cmp_scale(k, n)):
            bad.append(f"{k}: gpu {gpu[k]!r} oracle {orc[k]!r}")
    return bad


def array_mismatch(g: np.ndarray, o: np.ndarray, scale: np.ndarray | float = 0.0) -> float:
    """Largest excess of |g - o| over the per-element bound (<= 0 means all pass)."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    if g.shape != o.shape:
        return math.inf
    if g.size == 0:
        return 0.0
    bound = np.maximum(REL * np.abs(o), EPS4 * np.asarray(scale, np.float64))
    return float(np.max(np.abs(g - o) - bound))


def per_community_scales(ein, degsum, intra_density, qds_term, total: float):
    """S per community for q_term and qds_term.  total = |E| (or W when weighted; ein and
    degsum are then w_in and the strength s(c)).  q_term = ein/total - (degsum/2total)^2;
    qds_term = (ein/total) d - (degsum d/2total)^2 - p with p >= 0 the community's share
    of the split penalty, recovered here from the oracle's own values."""
    ein = np.asarray(ein, np.float64)
    ds = np.asarray(degsum, np.float64)
    d = np.asarray(intra_density, np.float64)
    a = ein / total
    b = (ds / (2.0 * total)) ** 2
    sq = a + b
    a2 = a * d
    b2 = (ds * d / (2.0 * total)) ** 2
    p = np.abs(a2 - b2 - np.asarray(qds_term, np.float64))
    return sq, a2 + b2 + p
