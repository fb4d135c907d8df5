"""Shared helpers for the GPU parity tests: run the library and the oracle on the
same seeded input and compare (integers bit-exact, binary64 within tolerance)."""
import math
import sys

import numpy as np

# Floating-point tolerance: 1e-12 relative; an absolute floor of 1e-13 for values
# near zero (Q, ARI and NMI of unrelated partitions), where both sides carry absolute
# rounding error of order 1e-16 times the magnitude of the cancelling terms.
REL = 1e-12
ABS = 1e-13

SCORE_INT = ("n", "m", "K", "num_pairs", "sum_ein", "sum_eout")
SCORE_FLT = ("Q", "Qds", "split_penalty", "mean_intra_edges", "mean_intra_density", "mean_contraction",
             "mean_inter_edges", "mean_expansion", "mean_conductance")
CMP_INT = ("n", "Ka", "Kb", "nnz", "a11", "a10", "a01", "a00", "A")
CMP_FLT = ("VI", "NMI", "F", "NVD", "RI", "ARI", "JI")


def note(msg: str) -> None:
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def fclose(g: float, o: float, rel=REL, abs_=ABS) -> bool:
    return abs(g - o) <= max(rel * abs(o), abs_) or (math.isnan(g) and math.isnan(o))


def check_score(gpu: dict, orc: dict, what: str = ""):
    bad = []
    for k in SCORE_INT:
        if int(gpu[k]) != int(orc[k]):
            bad.append(f"{k}: gpu {gpu[k]} oracle {orc[k]}")
    for k in SCORE_FLT:
        if not fclose(float(gpu[k]), float(orc[k])):
            bad.append(f"{k}: gpu {gpu[k]!r} oracle {orc[k]!r}")
    if gpu.get("device_flags", 0):
        bad.append(f"device_flags {gpu['device_flags']}")
    assert not bad, f"{what}: " + "; ".join(bad)


def check_compare(gpu: dict, orc: dict, what: str = ""):
    bad = []
    for k in CMP_INT:
        if int(gpu[k]) != int(orc[k]):
            bad.append(f"{k}: gpu {gpu[k]} oracle {orc[k]}")
    for k in CMP_FLT:
        if not fclose(float(gpu[k]), float(orc[k])):
            bad.append(f"{k}: gpu {gpu[k]!r} oracle {orc[k]!r}")
    assert not bad, f"{what}: " + "; ".join(bad)


def check_per_community(pc: dict, o) -> None:
    for k in ("size", "degsum", "ein", "eout"):
        g = pc[k].cpu().numpy()
        assert np.array_equal(g, getattr(o, k)), k
    for k in ("intra_density", "contraction", "expansion", "conductance", "q_term", "qds_term"):
        g = pc[k].cpu().numpy()
        e = getattr(o, k)
        tol = np.maximum(REL * np.abs(e), ABS)
        assert (np.abs(g - e) <= tol).all(), (k, float(np.max(np.abs(g - e))))


def sort_rows(t) -> np.ndarray:
    a = t.cpu().numpy() if hasattr(t, "cpu") else np.asarray(t)
    if a.size == 0:
        return a.reshape(0, 3)
    idx = np.lexsort((a[:, 1], a[:, 0]))
    return a[idx]
