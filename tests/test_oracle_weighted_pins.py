"""Pins for the weighted score of the oracle (Eqs. 8-9 and Section II-B3 with edge
weights; the densities d_c and d_{ci,cj} keep unweighted counts, as the paper notes
for weighted networks).

Independent routes: a hand-derived example in exact fractions, the unweighted oracle
(every weight 1), networkx's weighted modularity, dense weighted adjacency algebra,
and invariants (scaling every weight, pair weights summing to inter weights)."""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle
from cqgen import CONFIGS, csr_from_edges, erdos_renyi, lfr_graph, perturb_labels, random_labels

REL = 1e-12


def close(a, b, rel=REL, abs_=1e-13):
    return abs(a - b) <= max(rel * abs(b), abs_)


def weights_for(rp, ci, seed, lo=0.25, hi=4.0):
    """Symmetric float32 weights: one value per undirected edge, stored in both rows."""
    rng = np.random.default_rng(seed)
    n = len(rp) - 1
    w = np.zeros(len(ci), np.float32)
    rows = np.repeat(np.arange(n), np.diff(rp))
    a, b = np.minimum(rows, ci), np.maximum(rows, ci)
    key = a.astype(np.int64) * n + b
    uniq, inv = np.unique(key, return_inverse=True)
    vals = rng.uniform(lo, hi, len(uniq)).astype(np.float32)
    w[:] = vals[inv]
    return w


def two_triangles_weighted():
    # triangle A = {0,1,2} with weights 1, 1, 2; triangle B = {3,4,5} with weights 1;
    # bridge 2-3 with weight 3
    edges = {(0, 1): 1, (1, 2): 1, (0, 2): 2, (3, 4): 1, (4, 5): 1, (3, 5): 1, (2, 3): 3}
    rp, ci = csr_from_edges(6, list(edges))
    w = np.array([edges[(min(u, v), max(u, v))] for u in range(6) for v in ci[rp[u]:rp[u + 1]]], np.float32)
    return rp, ci, w


def test_two_triangles_weighted(orc):
    rp, ci, w = two_triangles_weighted()
    o = orc.score_w(rp, ci, w, [0, 0, 0, 1, 1, 1], 2)
    r = o.result
    # W = 4 + 3 + 3 = 10; w_in(A) = 4, s(A) = 2*4 + 3 = 11; w_in(B) = 3, s(B) = 9;
    # Q = 4/10 - (11/20)^2 + 3/10 - (9/20)^2 = 39/200.
    # d_A = d_B = 1 (unweighted: 3 edges among 3 nodes), d_AB = 1/(3*3), w(A,B) = 3:
    # each bracket loses (3/20)(1/9) = 1/60, so Qds = 39/200 - 1/30 = 97/600.
    want = {
        "W": Fr(10), "sum_w_in": Fr(7), "sum_w_out": Fr(6), "Q": Fr(39, 200), "Qds": Fr(97, 600),
        "split_penalty": Fr(1, 30), "mean_intra_edges": Fr(7, 2), "mean_intra_density": Fr(1),
        "mean_contraction": Fr(7, 3), "mean_inter_edges": Fr(3), "mean_expansion": Fr(1),
        "mean_conductance": Fr(10, 33),  # (3/11 + 3/9) / 2
    }
    for k, v in want.items():
        assert close(r[k], float(v)), (k, r[k], float(v))
    assert (r["m"], r["K"], r["num_pairs"], r["sum_ein"], r["sum_eout"]) == (7, 2, 1, 6, 2)
    assert np.allclose(o.strength, [11, 9]) and np.allclose(o.w_in, [4, 3]) and np.allclose(o.w_out, [3, 3])
    assert o.pairs.tolist() == [[0, 1, 1]] and o.pair_w.tolist() == [3.0]


def _cases():
    out = []
    g = lfr_graph(CONFIGS["tiny_1k"], 1)
    lab = g.labels.numpy()
    out.append(("tiny GT", g.row_ptr.numpy(), g.col_idx.numpy(), lab, g.num_labels))
    out.append(("tiny 20%", g.row_ptr.numpy(), g.col_idx.numpy(),
                perturb_labels(g.labels, g.num_labels, 0.2, 7).numpy(), g.num_labels))
    for seed in (1, 2, 3):
        rp, ci = erdos_renyi(120, 0.06, seed)
        out.append((f"er{seed}", rp, ci, random_labels(120, 9, seed).numpy(), 12))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c[0])
def test_unit_weights_equal_unweighted(orc, case):
    _, rp, ci, lab, L = case
    u = orc.score(rp, ci, lab, L).result
    w = orc.score_w(rp, ci, np.ones(len(ci), np.float32), lab, L)
    r = w.result
    for k in ("n", "m", "K", "num_pairs", "sum_ein", "sum_eout"):
        assert r[k] == u[k], k
    assert r["W"] == u["m"] and r["sum_w_in"] == u["sum_ein"] and r["sum_w_out"] == u["sum_eout"]
    for k in ("Q", "Qds", "split_penalty", "mean_intra_edges", "mean_intra_density", "mean_contraction",
              "mean_inter_edges", "mean_expansion", "mean_conductance"):
        assert close(r[k], u[k]), (k, r[k], u[k])


def _dense(rp, ci, w, lab, L):
    """Weighted adjacency algebra: S is the node-community indicator, A the weighted and
    B the 0/1 adjacency; S^T A S holds 2 w_in on the diagonal and w(ci,cj) off it,
    S^T B S the same counts unweighted."""
    n = len(rp) - 1
    A = np.zeros((n, n))
    B = np.zeros((n, n))
    for u in range(n):
        for e in range(rp[u], rp[u + 1]):
            A[u, ci[e]] = w[e]
            B[u, ci[e]] = 1.0
    S = np.zeros((n, L))
    S[np.arange(n), lab] = 1.0
    WA, WB = S.T @ A @ S, S.T @ B @ S
    sz = S.sum(0)
    W = A.sum() / 2
    s = A.sum(1) @ S
    live = sz > 0
    d = np.where(sz >= 2, WB.diagonal() / np.maximum(sz * (sz - 1), 1), 0.0)
    q = np.sum((WA.diagonal() / 2 / W - (s / (2 * W)) ** 2)[live])
    dij = WB / np.maximum(np.outer(sz, sz), 1)
    off = WA * dij / (2 * W)
    np.fill_diagonal(off, 0.0)
    qds = np.sum((WA.diagonal() / 2 / W * d - (s / (2 * W) * d) ** 2 - off.sum(1))[live])
    return W, q, qds


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_against_dense_weighted_algebra(orc, seed):
    rp, ci = erdos_renyi(60, 0.12, seed)
    w = weights_for(rp, ci, 100 + seed)
    lab = random_labels(60, 6, seed).numpy()
    r = orc.score_w(rp, ci, w, lab, 8).result
    W, q, qds = _dense(rp, ci, w.astype(np.float64), lab, 8)
    assert close(r["W"], W) and close(r["Q"], q) and close(r["Qds"], qds)


def test_networkx_weighted_modularity(orc):
    nx = pytest.importorskip("networkx")
    g = lfr_graph(CONFIGS["tiny_1k"], 2)
    rp, ci = g.row_ptr.numpy(), g.col_idx.numpy()
    w = weights_for(rp, ci, 9)
    lab = perturb_labels(g.labels, g.num_labels, 0.1, 3).numpy()
    G = nx.Graph()
    G.add_nodes_from(range(len(rp) - 1))
    for u in range(len(rp) - 1):
        for e in range(rp[u], rp[u + 1]):
            if u < ci[e]:
                G.add_edge(u, int(ci[e]), weight=float(w[e]))
    comms = [set(np.flatnonzero(lab == c).tolist()) for c in np.unique(lab)]
    want = nx.community.modularity(G, comms, weight="weight")
    assert close(orc.score_w(rp, ci, w, lab, g.num_labels).result["Q"], want, rel=1e-10)


def test_invariants(orc):
    g = lfr_graph(CONFIGS["tiny_1k"], 3)
    rp, ci = g.row_ptr.numpy(), g.col_idx.numpy()
    w = weights_for(rp, ci, 5)
    lab = perturb_labels(g.labels, g.num_labels, 0.15, 4).numpy()
    a = orc.score_w(rp, ci, w, lab, g.num_labels)
    b = orc.score_w(rp, ci, w * np.float32(4.0), lab, g.num_labels)  # exact in float32
    for k in ("Q", "Qds", "split_penalty", "mean_intra_density", "mean_conductance"):
        assert close(b.result[k], a.result[k]), k
    for k in ("W", "sum_w_in", "sum_w_out", "mean_intra_edges", "mean_contraction", "mean_inter_edges", "mean_expansion"):
        assert close(b.result[k], 4 * a.result[k]), k
    # strength = 2 w_in + w_out; pair weights add up to each side's inter weight
    assert np.allclose(a.strength, 2 * a.w_in + a.w_out, rtol=1e-12)
    acc = np.zeros(g.num_labels)
    np.add.at(acc, a.pairs[:, 0], a.pair_w)
    np.add.at(acc, a.pairs[:, 1], a.pair_w)
    assert np.allclose(acc, a.w_out, rtol=1e-12, atol=1e-9)
    assert close(a.result["W"], float(np.sum(w.astype(np.float64))) / 2)


def test_rejects_bad_weights(orc):
    rp, ci, w = two_triangles_weighted()
    for bad in (0.0, -1.0, np.inf, np.nan):
        w2 = w.copy()
        w2[3] = bad
        with pytest.raises(oracle.OracleError) as e:
            orc.score_w(rp, ci, w2, [0, 0, 0, 1, 1, 1], 2)
        assert e.value.code == oracle.ORC_E_GRAPH
