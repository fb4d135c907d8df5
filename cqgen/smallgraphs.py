"""Small deterministic graphs for special cases (cliques, stars, rings, G(n,p))."""
from __future__ import annotations

import numpy as np


def csr_from_edges(n: int, edges) -> tuple[np.ndarray, np.ndarray]:
    """Symmetric int32 CSR (rows sorted) from undirected edges; drops loops and repeats."""
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    if e.size:
        e = e[e[:, 0] != e[:, 1]]
        lo = np.minimum(e[:, 0], e[:, 1])
        hi = np.maximum(e[:, 0], e[:, 1])
        und = np.unique(lo * n + hi)
        lo, hi = und // n, und % n
        src = np.concatenate([lo, hi])
        dst = np.concatenate([hi, lo])
        key = np.sort(src * n + dst)
        rows, cols = key // n, key % n
    else:
        rows = cols = np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, np.int64)
    row_ptr[1:] = np.cumsum(np.bincount(rows, minlength=n))
    return row_ptr.astype(np.int32), cols.astype(np.int32)


def complete_graph(n: int):
    return csr_from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def cliques_graph(sizes):
    """Disjoint cliques; returns (row_ptr, col_idx, labels by clique)."""
    edges, labels, off = [], [], 0
    for c, s in enumerate(sizes):
        edges += [(off + i, off + j) for i in range(s) for j in range(i + 1, s)]
        labels += [c] * s
        off += s
    rp, ci = csr_from_edges(off, edges)
    return rp, ci, np.asarray(labels, np.int32)


def star_graph(leaves: int):
    return csr_from_edges(leaves + 1, [(0, i) for i in range(1, leaves + 1)])


def ring_graph(n: int):
    return csr_from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def erdos_renyi(n: int, p: float, seed: int):
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    mask = rng.random(iu[0].size) < p
    return csr_from_edges(n, np.stack([iu[0][mask], iu[1][mask]], axis=1))
