"""Pins for the oracle's no-ground-truth scoring (Section II-B: Eqs. 8, 9 and the six
measures of Section II-B3).

Nothing here re-types the oracle's formulas.  The oracle is held against:
  * hand-derived worked examples (exact fractions, derivations in comments),
  * closed forms (one community, all singletons, disjoint cliques, complete graph),
  * the textbook modularity (1/2m) sum_ij [A_ij - k_i k_j / 2m] delta(c_i, c_j)
    from a dense adjacency matrix, and networkx's modularity,
  * community counts from the dense block product S^T A S (S = membership matrix),
  * invariants (degree sums, pair-count row sums, relabelling and node permutation).
"""
from fractions import Fraction as Fr

import networkx as nx
import numpy as np
import pytest

from cqgen import cliques_graph, complete_graph, csr_from_edges, erdos_renyi, lfr_graph, CONFIGS, star_graph, ring_graph

REL = 1e-12


def close(a, b, rel=REL, abs_=1e-14):
    return abs(float(a) - float(b)) <= max(rel * abs(float(b)), abs_)


def dense(rp, ci):
    n = len(rp) - 1
    A = np.zeros((n, n), np.int64)
    for u in range(n):
        for e in range(rp[u], rp[u + 1]):
            A[u, ci[e]] += 1
    return A


TWO_TRIANGLES = [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)]


def test_two_triangles_by_triangle(orc):
    # m = 7; each triangle: |E_in| = 3, |E_out| = 1 (the bridge), degree sum 7, d = 1.
    # Q = 2 [3/7 - (7/14)^2] = 5/14.
    # pair density d_01 = 1/(3*3); per community Qds bracket = 3/7 - 1/4 - (1/14)(1/9) = 43/252.
    rp, ci = csr_from_edges(6, TWO_TRIANGLES)
    o = orc.score(rp, ci, [0, 0, 0, 1, 1, 1], 2)
    r = o.result
    assert r["m"] == 7 and r["K"] == 2 and r["num_pairs"] == 1
    assert close(r["Q"], Fr(5, 14))
    assert close(r["Qds"], 2 * Fr(43, 252))
    assert close(r["split_penalty"], Fr(1, 63))
    assert close(r["mean_intra_edges"], 3) and close(r["mean_intra_density"], 1)
    assert close(r["mean_contraction"], 2) and close(r["mean_inter_edges"], 1)
    assert close(r["mean_expansion"], Fr(1, 3)) and close(r["mean_conductance"], Fr(1, 7))
    assert o.pairs.tolist() == [[0, 1, 1]]


def test_two_triangles_three_pairs(orc):
    # communities {0,1}, {2,3}, {4,5}: |E_in| = 1 each; degree sums 4, 6, 4; |E_out| = 2, 4, 2.
    # Q = 3/7 - (16 + 36 + 16)/196 = 4/49.
    # |E_01| = 2 (0-2, 1-2), |E_12| = 2 (3-4, 3-5); d = 1 for all; d_01 = d_12 = 1/2.
    # Qds = [1/7 - 4/49 - 1/14] + [1/7 - 9/49 - 1/7] + [1/7 - 4/49 - 1/14] = -10/49.
    rp, ci = csr_from_edges(6, TWO_TRIANGLES)
    o = orc.score(rp, ci, [0, 0, 1, 1, 2, 2], 3)
    r = o.result
    assert close(r["Q"], Fr(4, 49))
    assert close(r["Qds"], Fr(-10, 49))
    assert close(r["split_penalty"], Fr(2, 7))
    assert r["num_pairs"] == 2
    assert o.eout.tolist() == [2, 4, 2] and o.degsum.tolist() == [4, 6, 4]
    assert close(r["mean_inter_edges"], Fr(8, 3)) and close(r["mean_expansion"], Fr(4, 3))
    assert close(r["mean_conductance"], Fr(5, 9))
    assert o.pairs.tolist() == [[0, 1, 2], [1, 2, 2]]


def test_star_unequal_sizes(orc):
    # star, centre 0, leaves 1..4 (m = 4); communities {0,1,2}, {3}, {4}.
    # c0: |E_in| = 2, degree sum 6, |E_out| = 2, d = 2*2/(3*2) = 2/3; singletons: d = 0.
    # Q = [2/4 - (6/8)^2] + 2 [0 - (1/8)^2] = -3/32.
    # |E_01| = |E_02| = 1, d_01 = d_02 = 1/3.
    # Qds: c0 = (1/2)(2/3) - ((3/4)(2/3))^2 - 2 (1/8)(1/3) = 0; c1 = c2 = -(1/8)(1/3); total -1/12.
    rp, ci = star_graph(4)
    o = orc.score(rp, ci, [0, 0, 0, 1, 2], 3)
    r = o.result
    assert close(r["Q"], Fr(-3, 32))
    assert close(r["Qds"], Fr(-1, 12))
    assert close(o.qds_term[0], 0.0) and close(o.qds_term[1], Fr(-1, 24))
    assert close(r["mean_intra_edges"], Fr(2, 3)) and close(r["mean_intra_density"], Fr(2, 9))
    assert close(r["mean_contraction"], Fr(4, 9)) and close(r["mean_inter_edges"], Fr(4, 3))
    assert close(r["mean_expansion"], Fr(8, 9)) and close(r["mean_conductance"], Fr(7, 9))
    assert close(r["split_penalty"], Fr(1, 6))


def test_empty_label_ids_are_not_communities(orc):
    rp, ci = csr_from_edges(6, TWO_TRIANGLES)
    a = orc.score(rp, ci, [0, 0, 1, 1, 2, 2], 3).result
    b = orc.score(rp, ci, [6, 6, 1, 1, 4, 4], 9).result
    assert b["K"] == 3
    for k in ("Q", "Qds", "split_penalty", "mean_conductance", "mean_intra_density", "num_pairs"):
        assert close(a[k], b[k])


def test_isolated_node_community(orc):
    # node 3 has no edges and is its own community: degree sum 0 -> conductance 0, d = 0.
    rp, ci = csr_from_edges(4, [(0, 1), (1, 2), (0, 2)])
    o = orc.score(rp, ci, [0, 0, 0, 1], 2)
    assert o.conductance[1] == 0.0 and o.intra_density[1] == 0.0 and o.degsum[1] == 0
    # triangle alone as one community: Q = 3/3 - (6/6)^2 = 0, Qds = 1*1 - 1 = 0
    assert close(o.result["Q"], 0.0) and close(o.result["Qds"], 0.0)


@pytest.mark.parametrize("n", [5, 12, 30])
def test_complete_graph_one_community(orc, n):
    rp, ci = complete_graph(n)
    r = orc.score(rp, ci, np.zeros(n, np.int32), 1).result
    assert r["Q"] == 0.0            # Eq. 8 with one community is 1 - 1
    assert close(r["Qds"], 0.0)     # d = 1: Qds = d(1 - d) = 0
    assert r["num_pairs"] == 0 and close(r["mean_conductance"], 0.0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_one_community_closed_form(orc, seed):
    # one community holding every node: Q = 0, Qds = d (1 - d) with d = 2m / (n (n-1)).
    rp, ci = erdos_renyi(40, 0.2, seed)
    n = 40
    r = orc.score(rp, ci, np.zeros(n, np.int32), 1).result
    d = Fr(2 * r["m"], n * (n - 1))
    assert abs(r["Q"]) < 1e-15
    assert close(r["Qds"], d * (1 - d))


@pytest.mark.parametrize("seed", [4, 5])
def test_all_singletons(orc, seed):
    # every node alone: Q = -sum_u (k_u / 2m)^2 ; Qds = -1 exactly (d_c = 0, each edge is a
    # pair of singletons with pair density 1, and the ordered pairs sum to 2m / 2m).
    rp, ci = erdos_renyi(50, 0.15, seed)
    n = 50
    r = orc.score(rp, ci, np.arange(n, dtype=np.int32), n).result
    k = np.diff(rp).astype(np.int64)
    twom = int(rp[-1])
    assert close(r["Q"], -sum(Fr(int(x) * int(x), twom * twom) for x in k))
    assert close(r["Qds"], -1.0)
    assert r["num_pairs"] == r["m"]


def test_disjoint_cliques(orc):
    # cliques partitioned by clique: no boundary edges, d = 1, so Qds = Q = sum (E_c/m)(1 - E_c/m).
    sizes = [3, 4, 6, 9]
    rp, ci, lab = cliques_graph(sizes)
    r = orc.score(rp, ci, lab, len(sizes)).result
    m = r["m"]
    E = [s * (s - 1) // 2 for s in sizes]
    q = sum(Fr(e, m) * (1 - Fr(e, m)) for e in E)
    assert close(r["Q"], q) and close(r["Qds"], q)
    assert r["num_pairs"] == 0 and r["sum_eout"] == 0


def test_ring_halves(orc):
    # ring of 10 split into two arcs of 5: each arc has 4 internal edges, 2 boundary edges,
    # degree sum 10. Q = 2 [4/10 - (10/20)^2] = 3/10.
    rp, ci = ring_graph(10)
    r = orc.score(rp, ci, [0] * 5 + [1] * 5, 2).result
    assert close(r["Q"], Fr(3, 10))


def _textbook_q(A, lab):
    k = A.sum(1).astype(np.float64)
    twom = k.sum()
    same = lab[:, None] == lab[None, :]
    return float(((A - np.outer(k, k) / twom) * same).sum() / twom)


def _random_cases():
    rng = np.random.default_rng(7)
    cases = []
    for i in range(12):
        n = int(rng.integers(6, 90))
        p = float(rng.uniform(0.03, 0.4))
        rp, ci = erdos_renyi(n, p, 100 + i)
        if rp[-1] == 0:
            continue
        L = int(rng.integers(1, n + 3))
        lab = rng.integers(0, L, n).astype(np.int32)
        cases.append((rp, ci, lab, L))
    g = lfr_graph(CONFIGS["tiny_1k"], 3)
    cases.append((g.row_ptr.numpy(), g.col_idx.numpy(), g.labels.numpy(), g.num_labels))
    return cases


@pytest.mark.parametrize("case", _random_cases(), ids=lambda c: f"n{len(c[0]) - 1}_L{c[3]}")
def test_against_dense_adjacency(orc, case):
    rp, ci, lab, L = case
    n = len(rp) - 1
    o = orc.score(rp, ci, lab, L)
    A = dense(rp, ci)
    # textbook modularity and networkx
    assert close(o.result["Q"], _textbook_q(A, lab), rel=1e-11, abs_=1e-13)
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from((u, int(ci[e])) for u in range(n) for e in range(rp[u], rp[u + 1]))
    comms = [set(np.nonzero(lab == c)[0].tolist()) for c in range(L) if (lab == c).any()]
    assert close(o.result["Q"], nx.community.modularity(G, comms), rel=1e-11, abs_=1e-13)
    # counts from S^T A S
    S = np.zeros((n, L), np.int64)
    S[np.arange(n), lab] = 1
    B = S.T @ A @ S
    assert (o.ein * 2 == np.diag(B)).all()
    assert (o.eout == B.sum(1) - np.diag(B)).all()
    assert (o.degsum == B.sum(1)).all()
    assert (o.size == S.sum(0)).all()
    iu = np.triu_indices(L, 1)
    nz = B[iu] > 0
    expect = np.stack([iu[0][nz], iu[1][nz], B[iu][nz]], axis=1)
    assert np.array_equal(o.pairs, expect)
    assert o.result["num_pairs"] == int(nz.sum())
    # invariants
    assert o.degsum.sum() == 2 * o.result["m"]
    ne = o.size > 0
    assert ((o.conductance[ne] >= 0) & (o.conductance[ne] <= 1)).all()
    assert np.allclose(o.contraction[ne] + o.expansion[ne], o.degsum[ne] / o.size[ne], rtol=1e-14)


def test_relabel_and_node_permutation_invariance(orc):
    g = lfr_graph(CONFIGS["tiny_1k"], 5)
    rp, ci, lab, L = g.row_ptr.numpy(), g.col_idx.numpy(), g.labels.numpy(), g.num_labels
    base = orc.score(rp, ci, lab, L).result
    rng = np.random.default_rng(0)
    perm_lab = rng.permutation(L + 5)[:L].astype(np.int32)          # injective relabel into a larger id space
    r1 = orc.score(rp, ci, perm_lab[lab], L + 5).result
    # node permutation: new id of node u is pi[u]
    n = len(rp) - 1
    pi = rng.permutation(n)
    inv = np.argsort(pi)
    edges = [(pi[u], pi[ci[e]]) for u in range(n) for e in range(rp[u], rp[u + 1]) if u < ci[e]]
    rp2, ci2 = csr_from_edges(n, edges)
    lab2 = lab[inv]
    r2 = orc.score(rp2, ci2, lab2, L).result
    for r in (r1, r2):
        for k in ("Q", "Qds", "split_penalty", "mean_intra_density", "mean_conductance", "mean_expansion"):
            assert close(r[k], base[k], rel=1e-13), k
        for k in ("K", "num_pairs", "sum_ein", "sum_eout", "m"):
            assert r[k] == base[k]


def test_pair_rows_sum_to_boundary(orc):
    g = lfr_graph(CONFIGS["tiny_1k"], 9)
    o = orc.score(g.row_ptr.numpy(), g.col_idx.numpy(), g.labels.numpy(), g.num_labels)
    acc = np.zeros(g.num_labels, np.int64)
    np.add.at(acc, o.pairs[:, 0], o.pairs[:, 2])
    np.add.at(acc, o.pairs[:, 1], o.pairs[:, 2])
    assert np.array_equal(acc, o.eout)


def test_error_codes(orc):
    rp, ci = csr_from_edges(6, TWO_TRIANGLES)
    with pytest.raises(orc.OracleError) as e:
        orc.score(rp, ci, [0, 0, 0, 1, 1, 2], 2)
    assert e.value.code == orc.ORC_E_LABEL
    rp0, ci0 = csr_from_edges(3, [])
    with pytest.raises(orc.OracleError) as e:
        orc.score(rp0, ci0, [0, 0, 0], 1)
    assert e.value.code == orc.ORC_E_NOEDGES
