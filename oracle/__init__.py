"""CPU oracle for community-quality metrics -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct C implementation (``cq_oracle.c``) of what the
paper defines: Q (Eq. 8), Qds (Eq. 9), the six measures of Section II-B3 (also on
edge-weighted graphs, with the densities kept unweighted), and VI, NMI, F-measure,
NVD, RI, ARI, JI (Eqs. 1-7).  It is the independent reference
the GPU library is checked against and shares no code with it.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import
this package; the product path never does.

``build()`` compiles ``cq_oracle.c`` with gcc into ``liborcq.so`` next to it;
:func:`lib` loads it (building it first if it is absent).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cq_oracle.c")
_SO = os.path.join(_HERE, "liborcq.so")

ORC_OK = 0
ORC_E_ARG = -1
ORC_E_LABEL = -2
ORC_E_GRAPH = -3
ORC_E_NOEDGES = -6
ORC_E_CAPACITY = -10
ORC_E_NOMEM = -11


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


class _ScoreResult(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "m", "K", "num_pairs", "sum_ein", "sum_eout")] + [
        (k, ctypes.c_double)
        for k in (
            "Q", "Qds", "split_penalty", "mean_intra_edges", "mean_intra_density",
            "mean_contraction", "mean_inter_edges", "mean_expansion", "mean_conductance",
        )
    ]


class _ScoreWResult(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "m", "K", "num_pairs", "sum_ein", "sum_eout")] + [
        (k, ctypes.c_double)
        for k in (
            "W", "sum_w_in", "sum_w_out", "Q", "Qds", "split_penalty", "mean_intra_edges", "mean_intra_density",
            "mean_contraction", "mean_inter_edges", "mean_expansion", "mean_conductance",
        )
    ]


class _CompareResult(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "Ka", "Kb", "nnz", "a11", "a10", "a01", "a00", "A")] + [
        (k, ctypes.c_double) for k in ("VI", "NMI", "F", "NVD", "RI", "ARI", "JI")
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_LIB = None


def load(path: str) -> ctypes.CDLL:
    """Load an oracle build from ``path`` (the tests also load deliberately broken copies)."""
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    L.orc_score.restype = ctypes.c_int
    L.orc_score.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_int32, ctypes.POINTER(_ScoreResult)] + [P] * 13 + [ctypes.c_int64]
    if hasattr(L, "orc_score_w"):
        L.orc_score_w.restype = ctypes.c_int
        L.orc_score_w.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int32, ctypes.POINTER(_ScoreWResult)] + [P] * 13 + [ctypes.c_int64]
    L.orc_compare.restype = ctypes.c_int
    L.orc_compare.argtypes = [ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_int32, ctypes.POINTER(_CompareResult), P, P, P, ctypes.c_int64]
    return L


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        _LIB = load(_SO)
    return _LIB


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


@dataclass
class ScoreOut:
    result: dict
    size: np.ndarray
    degsum: np.ndarray
    ein: np.ndarray
    eout: np.ndarray
    intra_density: np.ndarray
    contraction: np.ndarray
    expansion: np.ndarray
    conductance: np.ndarray
    q_term: np.ndarray
    qds_term: np.ndarray
    pairs: np.ndarray | None  # (num_pairs, 3) int64: ci, cj, |E_ci,cj| with ci < cj, ascending


@dataclass
class ScoreWOut:
    result: dict
    strength: np.ndarray
    w_in: np.ndarray
    w_out: np.ndarray
    intra_density: np.ndarray
    contraction: np.ndarray
    expansion: np.ndarray
    conductance: np.ndarray
    q_term: np.ndarray
    qds_term: np.ndarray
    pairs: np.ndarray | None  # (num_pairs, 3) int64: ci, cj, |E_ci,cj| with ci < cj, ascending
    pair_w: np.ndarray | None  # (num_pairs,) float64: w(ci, cj) in the same order


@dataclass
class CompareOut:
    result: dict
    cells: np.ndarray | None  # (nnz, 3) int64: i, j, |c_i ∩ c'_j|, ascending


def score(row_ptr, col_idx, labels, num_labels: int, *, want_pairs: bool = True, _lib=None) -> ScoreOut:
    """Score a partition of a symmetric CSR graph (Section II-B)."""
    rp, ci, lab = _i32(row_ptr), _i32(col_idx), _i32(labels)
    n = lab.shape[0]
    if rp.shape[0] != n + 1:
        raise ValueError("row_ptr must have n+1 entries")
    L = int(num_labels)
    arrs_i = [np.zeros(max(L, 1), np.int64) for _ in range(4)]
    arrs_d = [np.zeros(max(L, 1), np.float64) for _ in range(6)]
    m = int(rp[-1]) // 2 if n > 0 else 0
    cap = min(m, L * (L - 1) // 2) if want_pairs else 0
    pi = np.zeros(max(cap, 1), np.int32)
    pj = np.zeros(max(cap, 1), np.int32)
    pc = np.zeros(max(cap, 1), np.int64)
    res = _ScoreResult()
    rc = (_lib or lib()).orc_score(
        n, _ptr(rp), _ptr(ci), _ptr(lab), L, ctypes.byref(res),
        *[_ptr(a) for a in arrs_i], *[_ptr(a) for a in arrs_d],
        _ptr(pi), _ptr(pj), _ptr(pc), cap,
    )
    if rc != ORC_OK:
        raise OracleError(rc, "score")
    r = {k: getattr(res, k) for k, _ in _ScoreResult._fields_}
    pairs = None
    if want_pairs:
        npairs = r["num_pairs"]
        pairs = np.stack([pi[:npairs].astype(np.int64), pj[:npairs].astype(np.int64), pc[:npairs]], axis=1)
    return ScoreOut(r, *[a[:L] for a in arrs_i], *[a[:L] for a in arrs_d], pairs)


def score_w(row_ptr, col_idx, weights, labels, num_labels: int, *, want_pairs: bool = True, _lib=None) -> ScoreWOut:
    """Score a partition of an edge-weighted symmetric CSR graph: Eqs. 8-9 and the six
    measures with weight sums in place of edge counts, densities unweighted."""
    rp, ci, lab = _i32(row_ptr), _i32(col_idx), _i32(labels)
    w = np.ascontiguousarray(np.asarray(weights), dtype=np.float32)
    n = lab.shape[0]
    if rp.shape[0] != n + 1 or w.shape[0] != ci.shape[0]:
        raise ValueError("row_ptr must have n+1 entries and weights one per entry")
    L = int(num_labels)
    arrs = [np.zeros(max(L, 1), np.float64) for _ in range(9)]
    m = int(rp[-1]) // 2 if n > 0 else 0
    cap = min(m, L * (L - 1) // 2) if want_pairs else 0
    pi = np.zeros(max(cap, 1), np.int32)
    pj = np.zeros(max(cap, 1), np.int32)
    pc = np.zeros(max(cap, 1), np.int64)
    pw = np.zeros(max(cap, 1), np.float64)
    res = _ScoreWResult()
    rc = (_lib or lib()).orc_score_w(
        n, _ptr(rp), _ptr(ci), _ptr(w), _ptr(lab), L, ctypes.byref(res),
        *[_ptr(a) for a in arrs], _ptr(pi), _ptr(pj), _ptr(pc), _ptr(pw), cap,
    )
    if rc != ORC_OK:
        raise OracleError(rc, "weighted score")
    r = {k: getattr(res, k) for k, _ in _ScoreWResult._fields_}
    pairs = pair_w = None
    if want_pairs:
        k = r["num_pairs"]
        pairs = np.stack([pi[:k].astype(np.int64), pj[:k].astype(np.int64), pc[:k]], axis=1)
        pair_w = pw[:k].copy()
    return ScoreWOut(r, *[a[:L] for a in arrs], pairs, pair_w)


def compare(labels_a, num_labels_a: int, labels_b, num_labels_b: int, *, want_cells: bool = True, _lib=None) -> CompareOut:
    """Compare ground truth C (labels_a) with detected C' (labels_b) (Section II-A)."""
    la, lb = _i32(labels_a), _i32(labels_b)
    N = la.shape[0]
    if lb.shape[0] != N:
        raise ValueError("label arrays differ in length")
    cap = N if want_cells else 0
    ci = np.zeros(max(cap, 1), np.int32)
    cj = np.zeros(max(cap, 1), np.int32)
    cn = np.zeros(max(cap, 1), np.int64)
    res = _CompareResult()
    rc = (_lib or lib()).orc_compare(N, _ptr(la), int(num_labels_a), _ptr(lb), int(num_labels_b), ctypes.byref(res), _ptr(ci), _ptr(cj), _ptr(cn), cap)
    if rc != ORC_OK:
        raise OracleError(rc, "compare")
    r = {k: getattr(res, k) for k, _ in _CompareResult._fields_}
    cells = None
    if want_cells:
        k = r["nnz"]
        cells = np.stack([ci[:k].astype(np.int64), cj[:k].astype(np.int64), cn[:k]], axis=1)
    return CompareOut(r, cells)
