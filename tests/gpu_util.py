"""Shared helpers for the GPU parity tests: run the library and the oracle on the
same seeded input and compare (integers bit-exact, binary64 within tolerance)."""
import math
import sys

import numpy as np

from oracle.parity import (  # noqa: F401  (re-exported for the tests)
    CMP_FLT, CMP_INT, EPS4, REL, SCORE_FLT, SCORE_SCALE, SCORE_INT, array_mismatch, compare_mismatches, fclose,
    per_community_scales, score_mismatches,
)


def note(msg: str) -> None:
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def check_score(gpu: dict, orc: dict, what: str = ""):
    bad = score_mismatches(gpu, orc)
    assert not bad, f"{what}: " + "; ".join(bad)


def check_compare(gpu: dict, orc: dict, what: str = ""):
    bad = compare_mismatches(gpu, orc)
    assert not bad, f"{what}: " + "; ".join(bad)


def check_per_community(pc: dict, o, m: int) -> None:
    """Per-community outputs against the oracle: integers bit for bit, ratios of exact
    integers within 1e-12 relative, the Eq. (8) and Eq. (9) brackets with the
    near-zero bound scaled by their own terms."""
    for k in ("size", "degsum", "ein", "eout"):
        g = pc[k].cpu().numpy()
        assert np.array_equal(g, getattr(o, k)), k
    for k in ("intra_density", "contraction", "expansion", "conductance"):
        ex = array_mismatch(pc[k].cpu().numpy(), getattr(o, k))
        assert ex <= 0, (k, ex)
    s_q, s_qds = per_community_scales(o.ein, o.degsum, o.intra_density, o.qds_term, float(m))
    for k, s in (("q_term", s_q), ("qds_term", s_qds)):
        ex = array_mismatch(pc[k].cpu().numpy(), getattr(o, k), s)
        assert ex <= 0, (k, ex)


def sort_rows(t) -> np.ndarray:
    a = t.cpu().numpy() if hasattr(t, "cpu") else np.asarray(t)
    if a.size == 0:
        return a.reshape(0, 3)
    idx = np.lexsort((a[:, 1], a[:, 0]))
    return a[idx]


def table_equal(t, ref: np.ndarray, width: int) -> bool:
    """An exported (i, j, count) table (GPU tensor, rows in any order) equals the
    oracle's table (rows ascending by (i, j)).  Sorted on the GPU: tables of the
    100M-node graph hold over 10^8 rows."""
    import torch

    if t is None or int(t.shape[0]) != int(ref.shape[0]):
        return False
    if ref.shape[0] == 0:
        return True
    key = t[:, 0] * int(width) + t[:, 1]
    key, order = torch.sort(key)
    cnt = t[:, 2][order]
    rkey = ref[:, 0].astype(np.int64) * int(width) + ref[:, 1].astype(np.int64)
    return bool(np.array_equal(key.cpu().numpy(), rkey) and np.array_equal(cnt.cpu().numpy(), ref[:, 2]))
