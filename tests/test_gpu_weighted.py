"""GPU parity for edge-weighted scoring: cq_graph_load_weighted + cq_score_partition
against the oracle's weighted score (Eqs. 8-9 and the measures of Section II-B3 with
weight sums in place of edge counts; the densities d_c and d_{ci,cj} keep the
unweighted counts, as the paper notes for weighted networks).

Integer counts and the pair table must match bit for bit, W exactly; binary64 values
within the tolerance in tests/gpu_util.py."""
import numpy as np
import pytest
import torch

import oracle
from cqgen import CONFIGS, csr_from_edges, edge_weights, erdos_renyi, lfr_graph, perturb_labels, random_labels
from tests.gpu_util import SCORE_SCALE, array_mismatch, check_score, fclose, note, per_community_scales, sort_rows

pytestmark = pytest.mark.gpu

ORDERS = ["input", "blocked", "unblocked"]
WEIGHT_MIN = 2.0 ** -32
WEIGHT_MAX = 2.0 ** 32


@pytest.fixture(scope="module")
def cq():
    from paper_1507_05492_amd import cq as mod

    return mod


@pytest.fixture(scope="module")
def ctx(cq):
    c = cq.Context(0)
    yield c
    c.close()


def open_weighted(cq, ctx, rp_t, ci_t, w_t, order, validate=False):
    g = cq.Graph(ctx, rp_t, ci_t, validate=validate, reorder=(order != "input"), blocks=(order == "blocked"),
                 weights=w_t)
    want = {"input": 0, "blocked": cq.CQ_GRAPH_REORDER, "unblocked": cq.CQ_GRAPH_REORDER | cq.CQ_GRAPH_NO_BLOCKS}[order]
    assert g.stats["reordered"] == want and g.stats["weighted"] == 1
    return g


def check_weighted(r: dict, o, what: str, per_comm=None, pairs=None):
    """r: the library's result; o: oracle.score_w output."""
    check_score(r, o.result, what)
    assert r["weighted"] == 1, what
    bad = []
    for gk, ok in (("total_weight", "W"), ("sum_w_in", "sum_w_in"), ("sum_w_out", "sum_w_out")):
        if not fclose(float(r[gk]), float(o.result[ok])):
            bad.append(f"{gk}: gpu {r[gk]!r} oracle {o.result[ok]!r}")
    assert not bad, f"{what}: " + "; ".join(bad)
    if per_comm is not None:
        # ratios and positive weight sums: 1e-12 relative; the Eq. (8) and (9) brackets with
        # the near-zero bound scaled by their own terms
        s_q, s_qds = per_community_scales(o.w_in, o.strength, o.intra_density, o.qds_term, float(o.result["W"]))
        for k, s in (("intra_density", 0.0), ("contraction", 0.0), ("expansion", 0.0), ("conductance", 0.0),
                     ("w_in", 0.0), ("strength", 0.0), ("q_term", s_q), ("qds_term", s_qds)):
            ex = array_mismatch(per_comm[k].cpu().numpy(), getattr(o, k), s)
            assert ex <= 0, (what, k, ex)
        # integer per-community fields are the unweighted counts
        size = per_comm["size"].cpu().numpy()
        ein = per_comm["ein"].cpu().numpy()
        eout = per_comm["eout"].cpu().numpy()
        assert int(size.sum()) == r["n"] and int(ein.sum()) == r["sum_ein"] and int(eout.sum()) == r["sum_eout"], what
    if pairs is not None:
        assert np.array_equal(sort_rows(pairs), o.pairs), f"{what}: pair table differs"


def run_case(cq, ctx, rp, ci, w, lab, L, what, *, order="input", validate=True, per_comm=True, pairs=True):
    what = f"{what} [{order} graph]"
    note(what)
    rp_t = torch.as_tensor(np.asarray(rp, np.int32)).cuda()
    ci_t = torch.as_tensor(np.asarray(ci, np.int32)).cuda()
    w_t = torch.as_tensor(np.asarray(w, np.float32)).cuda()
    lab_t = torch.as_tensor(np.asarray(lab, np.int32)).cuda()
    g = open_weighted(cq, ctx, rp_t, ci_t, w_t, order, validate=validate)
    o = oracle.score_w(np.asarray(rp), np.asarray(ci), np.asarray(w, np.float32), np.asarray(lab), L, want_pairs=pairs)
    assert fclose(g.stats["total_weight"], o.result["W"]), (what, g.stats["total_weight"], o.result["W"])
    cap = max(1, int(o.result["num_pairs"])) if pairs else 0
    r, pc, pt = cq.score_partition(g, lab_t, L, per_community=per_comm, pairs_capacity=cap)
    torch.cuda.synchronize()
    check_weighted(r, o, what, pc if per_comm else None, pt if pairs else None)
    g.close()
    return r, o


def weights_np(rp, ci, seed, **kw):
    return edge_weights(torch.as_tensor(np.asarray(rp)), torch.as_tensor(np.asarray(ci)), seed, **kw).numpy()


def lfr_case(name, seed):
    g = lfr_graph(CONFIGS[name], seed)
    return g.row_ptr.numpy(), g.col_idx.numpy(), g.labels.numpy(), g.num_labels


@pytest.mark.parametrize("order", ORDERS)
def test_two_triangles(cq, ctx, order):
    # two triangles joined by one bridge, weights chosen by hand
    edges = {(0, 1): 1, (1, 2): 1, (0, 2): 2, (3, 4): 1, (4, 5): 1, (3, 5): 1, (2, 3): 3}
    rp, ci = csr_from_edges(6, list(edges))
    w = np.array([edges[(min(u, int(v)), max(u, int(v)))] for u in range(6) for v in ci[rp[u]:rp[u + 1]]], np.float32)
    r, o = run_case(cq, ctx, rp, ci, w, [0, 0, 0, 1, 1, 1], 2, "two triangles", order=order)
    assert r["total_weight"] == 10.0 and r["sum_w_in"] == 7.0 and r["sum_w_out"] == 6.0


@pytest.mark.parametrize("order", ORDERS)
def test_tiny_lfr(cq, ctx, order):
    rp, ci, lab, L = lfr_case("tiny_1k", 1)
    w = weights_np(rp, ci, 31)
    run_case(cq, ctx, rp, ci, w, lab, L, "tiny_1k weighted ground truth", order=order)
    pert = perturb_labels(torch.as_tensor(lab), L, 0.10, 101).numpy()
    run_case(cq, ctx, rp, ci, w, pert, L, "tiny_1k weighted perturbed 10%", order=order)


@pytest.mark.parametrize("order", ORDERS)
@pytest.mark.parametrize("name", ["m100k_mu0.1", "m100k_mu0.5"])
def test_m100k(cq, ctx, name, order):
    rp, ci, lab, L = lfr_case(name, 11)
    w = weights_np(rp, ci, 41)
    run_case(cq, ctx, rp, ci, w, lab, L, f"{name} weighted ground truth", order=order)
    pert = perturb_labels(torch.as_tensor(lab), L, 0.30, 1030).numpy()
    run_case(cq, ctx, rp, ci, w, pert, L, f"{name} weighted perturbed 30%", order=order, per_comm=False)


def test_extreme_weights_and_special_partitions(cq, ctx):
    rp, ci = erdos_renyi(400, 0.04, 5)
    n = 400
    w = weights_np(rp, ci, 9, values=[WEIGHT_MIN, 1.0, WEIGHT_MAX, 3.0e-7, 5.0e8])
    lab = random_labels(n, 12, 3).numpy()
    run_case(cq, ctx, rp, ci, w, lab, 12, "weights 2^-32 .. 2^32")
    w1 = weights_np(rp, ci, 10)
    run_case(cq, ctx, rp, ci, w1, np.zeros(n, np.int32), 1, "one community")
    run_case(cq, ctx, rp, ci, w1, np.arange(n, dtype=np.int32), n, "all singletons")
    run_case(cq, ctx, rp, ci, w1, random_labels(n, 40, 7).numpy() * 3, 120, "sparse label ids")
    rp2, ci2 = csr_from_edges(5, [(0, 1), (1, 2)])  # nodes 3, 4 isolated
    run_case(cq, ctx, rp2, ci2, np.array([0.5, 0.5, 2.0, 2.0], np.float32), [0, 0, 1, 2, 2], 3,
             "isolated-node communities")


def test_unit_weights_match_unweighted(cq, ctx):
    rp, ci, lab, L = lfr_case("m100k_mu0.3", 11)
    rp_t = torch.as_tensor(rp).cuda()
    ci_t = torch.as_tensor(ci).cuda()
    lab_t = torch.as_tensor(lab).cuda()
    note("m100k_mu0.3 unit weights vs the unweighted path")
    gu = cq.Graph(ctx, rp_t, ci_t)
    gw = cq.Graph(ctx, rp_t, ci_t, weights=torch.ones(len(ci), dtype=torch.float32, device="cuda"))
    assert gw.stats["total_weight"] == gw.stats["m"] == gu.stats["m"] and gu.stats["weighted"] == 0
    ru, _, _ = cq.score_partition(gu, lab_t, L)
    rw, _, _ = cq.score_partition(gw, lab_t, L)
    assert ru["weighted"] == 0 and ru["total_weight"] == ru["m"]
    assert ru["sum_w_in"] == ru["sum_ein"] and ru["sum_w_out"] == ru["sum_eout"]
    for k in ("n", "m", "K", "num_pairs", "sum_ein", "sum_eout"):
        assert ru[k] == rw[k], k
    assert rw["sum_w_in"] == ru["sum_ein"] and rw["sum_w_out"] == ru["sum_eout"]
    for k in ("Q", "Qds", "split_penalty", "mean_intra_edges", "mean_intra_density", "mean_contraction",
              "mean_inter_edges", "mean_expansion", "mean_conductance"):
        assert fclose(rw[k], ru[k], SCORE_SCALE.get(k, 0.0)), (k, rw[k], ru[k])
    gu.close()
    gw.close()


@pytest.mark.parametrize("order", ORDERS)
def test_random_labels_compact_staging(cq, ctx, order):
    """Random labels on a column-blocked weighted graph: nearly every entry has another
    label, so the own-span tiles' staging buffer overflows and the second pass stages;
    200 ids leave each bucket of the node pass few enough labels for its atomic totals,
    3000 ids make every bucket write a histogram row."""
    rp, ci, lab, L = lfr_case("m100k_mu0.3", 14)
    w = weights_np(rp, ci, 61)
    n = len(rp) - 1
    for nl, seed in ((200, 21), (3000, 22)):
        labr = random_labels(n, nl, seed).numpy()
        run_case(cq, ctx, rp, ci, w, labr, nl, f"random labels, {nl} ids", order=order, per_comm=False)


def test_label_id_limits(cq, ctx):
    rp, ci, lab, L = lfr_case("m100k_mu0.3", 12)
    w = weights_np(rp, ci, 51)
    n = len(rp) - 1
    lab2 = (lab.astype(np.int64) * 7919 % 20011).astype(np.int32)  # beyond the node-pass LDS histograms
    run_case(cq, ctx, rp, ci, w, lab2, 20011, "relabelled into 20011 ids", per_comm=False)
    lab3 = random_labels(n, 32768, 5).numpy()  # the largest label space of the weighted group pass
    for order in ORDERS:
        run_case(cq, ctx, rp, ci, w, lab3, 32768, "random labels, 32768 ids", order=order, per_comm=False)
    note("32769 ids are rejected")
    g = cq.Graph(ctx, torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(), weights=torch.as_tensor(w).cuda())
    lab_t = torch.as_tensor(lab).cuda()
    with pytest.raises(cq.CQError) as e:
        cq.score_partition(g, lab_t, 32769)
    assert e.value.status == cq.CQ_E_INVALID_ARG
    g.close()


def test_load_errors(cq, ctx):
    rp, ci = erdos_renyi(300, 0.05, 3)
    rp_t = torch.as_tensor(rp).cuda()
    ci_t = torch.as_tensor(ci).cuda()
    w = weights_np(rp, ci, 2)
    for bad, what in ((0.0, "zero"), (-1.0, "negative"), (float("nan"), "NaN"), (float("inf"), "inf"),
                      (2.0 ** 33, "2^33"), (2.0 ** -33, "2^-33"), (2.0 ** 40, "2^40")):
        note(f"weight {what} is rejected")
        wb = w.copy()
        wb[17] = bad
        with pytest.raises(cq.CQError) as e:
            cq.Graph(ctx, rp_t, ci_t, weights=torch.as_tensor(wb).cuda())
        assert e.value.status == cq.CQ_E_GRAPH_FORMAT, what
    note("unequal weights on the two entries of an edge")
    wa = w.copy()
    wa[rp[0]] = 2.0 * w[rp[0]]  # the first entry of row 0 only; its mirror keeps the old weight
    with pytest.raises(cq.CQError) as e:
        cq.Graph(ctx, rp_t, ci_t, validate=True, weights=torch.as_tensor(wa).cuda())
    assert e.value.status == cq.CQ_E_GRAPH_FORMAT
    # a weighted load checks the mirror weights whether or not validation was asked for
    with pytest.raises(cq.CQError) as e:
        cq.Graph(ctx, rp_t, ci_t, validate=False, weights=torch.as_tensor(wa).cuda())
    assert e.value.status == cq.CQ_E_GRAPH_FORMAT
    g = cq.Graph(ctx, rp_t, ci_t, validate=False, weights=torch.as_tensor(w).cuda())
    assert g.stats["validated"] == cq.CQ_VALIDATE_GRAPH
    g.close()
    note("null weights")
    with pytest.raises(cq.CQError) as e:
        cq.cq_graph_load_weighted(ctx.handle, len(rp) - 1, len(ci), rp_t.data_ptr(), ci_t.data_ptr(), None, 0)
    assert e.value.status == cq.CQ_E_INVALID_ARG
    with pytest.raises(ValueError):
        cq.Graph(ctx, rp_t, ci_t, weights=torch.ones(len(ci) - 2, dtype=torch.float32, device="cuda"))


def test_label_error_and_batch_and_server(cq, ctx):
    rp, ci, lab, L = lfr_case("tiny_1k", 2)
    w = weights_np(rp, ci, 61)
    rp_t = torch.as_tensor(rp).cuda()
    ci_t = torch.as_tensor(ci).cuda()
    g = cq.Graph(ctx, rp_t, ci_t, weights=torch.as_tensor(w).cuda())
    lab_t = torch.as_tensor(lab).cuda()
    note("weighted: label out of range")
    bad = lab_t.clone()
    bad[7] = L + 2
    r, _, _ = cq.score_partition(g, bad, L, allow=(cq.CQ_E_LABEL_RANGE,))
    assert r["status"] == cq.CQ_E_LABEL_RANGE
    note("weighted: batch plans refuse weighted graphs")
    with pytest.raises(cq.CQError) as e:
        cq.Batch(ctx, [(g, lab_t, L)], autotune=False)
    assert e.value.status == cq.CQ_E_INVALID_ARG
    note("weighted: server requests run alone and match a direct call")
    direct, _, _ = cq.score_partition(g, lab_t, L)
    direct = dict(direct)
    direct.pop("status")
    srv = cq.Server(ctx, num_slots=2, max_batch=8, memory_budget=1 << 30, small_nnz=1_000_000)
    h = lab_t.cpu().pin_memory()
    tickets = [srv.submit_score(g, h, L) for _ in range(3)]
    o = oracle.score_w(rp, ci, w, lab, L, want_pairs=False)
    for t in tickets:
        out = srv.wait(t)
        assert out["status"] == cq.CQ_OK and out["score"] == direct
        check_weighted(out["score"], o, "weighted served request vs oracle")
    assert srv.stats()["grouped_requests"] == 0
    srv.close()
    g.close()


def test_deterministic_and_workspace_reuse(cq, ctx):
    rp, ci, lab, L = lfr_case("m100k_mu0.5", 11)
    pert = perturb_labels(torch.as_tensor(lab), L, 0.30, 1030).cuda()
    w = torch.as_tensor(weights_np(rp, ci, 71)).cuda()
    rp_t = torch.as_tensor(rp).cuda()
    ci_t = torch.as_tensor(ci).cuda()
    for order in ORDERS:
        note(f"weighted m100k_mu0.5 perturbed 30%: repeated runs [{order} graph]")
        g = open_weighted(cq, ctx, rp_t, ci_t, w, order)
        ws = torch.empty(g.workspace_size(L), dtype=torch.uint8, device="cuda")
        first = None
        for i in range(4):
            ws.fill_(255 if i % 2 else 0)
            r, _, _ = cq.score_partition(g, pert, L, workspace=ws)
            r = dict(r)
            if first is None:
                first = r
            assert r == first, (order, i)
        g.close()


def test_full_size_l10m(cq, ctx):
    """10M-node LFR graph with weights: counts exact, the pair table exact, metrics within
    tolerance, for every storage order."""
    note("weighted l10m: generating on the GPU")
    gr = lfr_graph(CONFIGS["l10m"], 21, device="cuda")
    w = edge_weights(gr.row_ptr, gr.col_idx, 81)
    rp, ci, lab = gr.row_ptr.cpu().numpy(), gr.col_idx.cpu().numpy(), gr.labels.cpu().numpy()
    wn = w.cpu().numpy()
    note(f"weighted l10m: n={gr.n} nnz={gr.nnz} K={gr.num_labels}; oracle")
    o = oracle.score_w(rp, ci, wn, lab, gr.num_labels)
    del rp, ci, wn
    for order in ORDERS:
        note(f"weighted l10m: GPU, {order} graph")
        g = open_weighted(cq, ctx, gr.row_ptr, gr.col_idx, w, order)
        assert fclose(g.stats["total_weight"], o.result["W"])
        r, pc, pt = cq.score_partition(g, gr.labels, gr.num_labels, per_community=True,
                                       pairs_capacity=int(o.result["num_pairs"]))
        check_weighted(r, o, f"weighted l10m [{order} graph]", pc, pt)
        g.close()
