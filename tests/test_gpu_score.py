"""GPU parity: cq_score_partition against the oracle (Section II-B, Eqs. 8-9, II-B3).

Counts, per-community integers and the pair table |E_{ci,cj}| must match bit for bit;
binary64 metrics within the tolerance in tests/gpu_util.py."""
import numpy as np
import pytest
import torch

import oracle
from cqgen import CONFIGS, LFRParams, csr_from_edges, erdos_renyi, lfr_graph, perturb_labels, random_labels, star_graph
from tests.gpu_util import check_per_community, check_score, note, sort_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cq():
    from paper_1507_05492_amd import cq as mod

    return mod


@pytest.fixture(scope="module")
def ctx(cq):
    c = cq.Context(0)
    yield c
    c.close()


# graph storage: the caller's order, renumbered with column blocks, renumbered without
ORDERS = ["input", "blocked", "unblocked"]


def open_graph(cq, ctx, rp_t, ci_t, order, validate=False):
    g = cq.Graph(ctx, rp_t, ci_t, validate=validate, reorder=(order != "input"), blocks=(order == "blocked"))
    want = {"input": 0, "blocked": cq.CQ_GRAPH_REORDER, "unblocked": cq.CQ_GRAPH_REORDER | cq.CQ_GRAPH_NO_BLOCKS}[order]
    assert g.stats["reordered"] == want
    return g


def run_case(cq, ctx, rp, ci, lab, L, what, *, validate=True, pairs=True, per_comm=True, reorder="input",
             expect_staging=None):
    what = f"{what} [{reorder} graph]"
    note(what)
    rp_t = torch.as_tensor(np.asarray(rp, np.int32)).cuda()
    ci_t = torch.as_tensor(np.asarray(ci, np.int32)).cuda()
    lab_t = torch.as_tensor(np.asarray(lab, np.int32)).cuda()
    g = open_graph(cq, ctx, rp_t, ci_t, reorder, validate=validate)
    o = oracle.score(np.asarray(rp), np.asarray(ci), np.asarray(lab), L, want_pairs=pairs)
    cap = max(1, int(o.result["num_pairs"])) if pairs else 0
    r, pc, pt = cq.score_partition(g, lab_t, L, per_community=per_comm, pairs_capacity=cap)
    torch.cuda.synchronize()
    check_score(r, o.result, what)
    if per_comm:
        check_per_community(pc, o, int(o.result["m"]))
    if pairs:
        assert np.array_equal(sort_rows(pt), o.pairs), f"{what}: pair table differs"
    if expect_staging is not None:
        assert g.last_staging == expect_staging, (what, g.last_staging)
    g.close()
    return r, o


def lfr_case(name, seed):
    g = lfr_graph(CONFIGS[name], seed)
    return g.row_ptr.numpy(), g.col_idx.numpy(), g.labels.numpy(), g.num_labels


@pytest.mark.parametrize("reorder", ORDERS)
def test_tiny_lfr_ground_truth_and_perturbed(cq, ctx, reorder):
    rp, ci, lab, L = lfr_case("tiny_1k", 1)
    run_case(cq, ctx, rp, ci, lab, L, "tiny_1k seed1 ground truth", reorder=reorder)
    pert = perturb_labels(torch.as_tensor(lab), L, 0.10, 101).numpy()
    run_case(cq, ctx, rp, ci, pert, L, "tiny_1k seed1 perturbed 10%", reorder=reorder)


@pytest.mark.parametrize("reorder", ORDERS)
@pytest.mark.parametrize("name", ["m100k_mu0.1", "m100k_mu0.3", "m100k_mu0.5"])
def test_m100k(cq, ctx, name, reorder):
    rp, ci, lab, L = lfr_case(name, 11)
    run_case(cq, ctx, rp, ci, lab, L, f"{name} ground truth", reorder=reorder)
    for pct in (5, 30):
        pert = perturb_labels(torch.as_tensor(lab), L, pct / 100, 1000 + pct).numpy()
        run_case(cq, ctx, rp, ci, pert, L, f"{name} perturbed {pct}%", per_comm=False, reorder=reorder)


def test_special_partitions(cq, ctx):
    rp, ci = erdos_renyi(300, 0.05, 3)
    n = 300
    run_case(cq, ctx, rp, ci, np.zeros(n, np.int32), 1, "one community")
    run_case(cq, ctx, rp, ci, np.arange(n, dtype=np.int32), n, "all singletons (small tables)")
    lab = random_labels(n, 40, 7).numpy() * 3  # ids 0, 3, 6, ...: most label ids empty
    run_case(cq, ctx, rp, ci, lab, 120, "sparse label ids")
    rp2, ci2 = csr_from_edges(5, [(0, 1), (1, 2)])  # nodes 3, 4 isolated
    run_case(cq, ctx, rp2, ci2, [0, 0, 1, 2, 2], 3, "isolated-node communities")


def test_many_labels_global_paths(cq, ctx):
    # more label ids than fit LDS: global-atomic node pass and hash-only group tables
    rp, ci, lab, L = lfr_case("m100k_mu0.3", 12)
    n = len(rp) - 1
    run_case(cq, ctx, rp, ci, np.arange(n, dtype=np.int32), n, "all singletons n=1e5", pairs=True)
    lab2 = (lab.astype(np.int64) * 7919 % 40009).astype(np.int32)  # injective relabel into 40009 ids
    run_case(cq, ctx, rp, ci, lab2, 40009, "relabelled into 40009 ids")
    run_case(cq, ctx, rp, ci, lab2, 40009, "relabelled into 40009 ids", reorder="blocked")
    run_case(cq, ctx, rp, ci, lab2, 40009, "relabelled into 40009 ids", reorder="unblocked")
    lab3 = (lab.astype(np.int64) * 7919 % 70001).astype(np.int32)  # ids beyond 16 bits: 32-bit staging
    run_case(cq, ctx, rp, ci, lab3, 70001, "relabelled into 70001 ids", reorder="blocked")
    run_case(cq, ctx, rp, ci, lab3, 70001, "relabelled into 70001 ids", reorder="unblocked")


@pytest.mark.parametrize("reorder", ORDERS)
def test_random_labels_compact_staging(cq, ctx, reorder):
    """Random labels: nearly every entry has another label, so on a column-blocked graph
    the own-span tiles' staging buffer overflows and the second pass stages; 200 ids
    leave each bucket of the node pass few enough labels for its atomic totals, 3000 ids
    make every bucket write a histogram row."""
    rp, ci, lab, L = lfr_case("m100k_mu0.3", 15)
    n = len(rp) - 1
    for nl, seed in ((200, 23), (3000, 24)):
        labr = random_labels(n, nl, seed).numpy()
        if reorder != "blocked":
            run_case(cq, ctx, rp, ci, labr, nl, f"random labels, {nl} ids", reorder=reorder, per_comm=False)
            continue
        # both stagings of a column-blocked graph: the blocks (forced), and the row-major
        # copy the call picks for labels out of the stored order
        for frac, want in ((2.0, cq.CQ_STAGING_BLOCKS), (1 / 16, cq.CQ_STAGING_ROWS)):
            cq.cq_context_set_row_staging(ctx.handle, frac)
            try:
                run_case(cq, ctx, rp, ci, labr, nl, f"random labels, {nl} ids, row staging from {frac}", reorder=reorder,
                         per_comm=False, expect_staging=want)
            finally:
                cq.cq_context_set_row_staging(ctx.handle, 1 / 16)


def test_staging_choice_on_blocked_graphs(cq, ctx):
    """A column-blocked graph counts the label changes along its stored order: the ground
    truth (runs) keeps the blocks, 30 % reassigned nodes or random labels take the
    row-major copy, and forcing either choice gives the same result bit for bit."""
    rp, ci, lab, L = lfr_case("m100k_mu0.3", 16)
    n = len(rp) - 1
    cases = [("ground truth", lab, cq.CQ_STAGING_BLOCKS),
             ("1% reassigned", perturb_labels(torch.as_tensor(lab), L, 0.01, 161).numpy(), None),
             ("30% reassigned", perturb_labels(torch.as_tensor(lab), L, 0.30, 162).numpy(), cq.CQ_STAGING_ROWS),
             ("random", random_labels(n, L, 163).numpy(), cq.CQ_STAGING_ROWS)]
    rp_t = torch.as_tensor(np.asarray(rp, np.int32)).cuda()
    ci_t = torch.as_tensor(np.asarray(ci, np.int32)).cuda()
    g = open_graph(cq, ctx, rp_t, ci_t, "blocked")
    for what, lb, want in cases:
        note(f"staging choice: {what}")
        o = oracle.score(rp, ci, lb, L)
        lab_t = torch.as_tensor(np.asarray(lb, np.int32)).cuda()
        cap = max(1, int(o.result["num_pairs"]))
        r, pc, pt = cq.score_partition(g, lab_t, L, per_community=True, pairs_capacity=cap)
        assert want is None or g.last_staging == want, (what, g.last_staging)
        check_score(r, o.result, what)
        check_per_community(pc, o, int(o.result["m"]))
        assert np.array_equal(sort_rows(pt), o.pairs), what
        for frac, forced in ((-1.0, cq.CQ_STAGING_ROWS), (2.0, cq.CQ_STAGING_BLOCKS)):
            cq.cq_context_set_row_staging(ctx.handle, frac)
            try:
                r2, pc2, pt2 = cq.score_partition(g, lab_t, L, per_community=True, pairs_capacity=cap)
            finally:
                cq.cq_context_set_row_staging(ctx.handle, 1 / 16)
            assert g.last_staging == forced, (what, frac)
            assert r2 == r, (what, frac)
            for k in ("size", "degsum", "ein", "eout", "intra_density", "contraction", "expansion", "conductance",
                      "q_term", "qds_term"):
                assert torch.equal(pc2[k], pc[k]), (what, frac, k)
            assert np.array_equal(sort_rows(pt2), o.pairs), (what, frac)
    g.close()


def test_wide_counter_wraps(cq, ctx):
    # 40003 label ids select 16-bit LDS counters for large segments.  Community 0 is
    # joined completely to communities 40000 and 40001 (300 x 300 edges each), so both
    # of its counters pass 65535 (even label: low-half wrap with a carry; odd: high half).
    k = 300
    A = np.arange(k)
    B = np.arange(k, 2 * k)
    C = np.arange(2 * k, 3 * k)
    edges = [(int(u), int(v)) for u in A for v in np.concatenate([B, C])]
    edges += [(int(B[i]), int(B[i + 1])) for i in range(k - 1)] + [(int(C[i]), int(C[i + 1])) for i in range(k - 1)]
    rp, ci = csr_from_edges(3 * k, edges)
    lab = np.concatenate([np.zeros(k), np.full(k, 40000), np.full(k, 40001)]).astype(np.int32)
    for order in ORDERS:
        run_case(cq, ctx, rp, ci, lab, 40003, "complete bipartite 300x600, labels 0/40000/40001", reorder=order)


def test_hub_split_classes(cq, ctx):
    # a hub adjacent to 20000 singleton communities: its table needs residue classes;
    # labels that are all multiples of 8 force classes to overflow and split again.
    leaves = 20000
    rp, ci = star_graph(leaves)
    n = leaves + 1
    run_case(cq, ctx, rp, ci, np.arange(n, dtype=np.int32), n, "star 20000 singletons")
    lab = (np.arange(n, dtype=np.int64) * 8).astype(np.int32)
    for order in ORDERS:
        run_case(cq, ctx, rp, ci, lab, 8 * n, "star 20000 singletons, labels = 8i", reorder=order)


def test_graph_order(cq, ctx):
    # the stored order of a renumbered graph is a permutation of the caller's ids
    rp, ci, lab, L = lfr_case("m100k_mu0.3", 11)
    rp_t = torch.as_tensor(rp).cuda()
    ci_t = torch.as_tensor(ci).cuda()
    for order in ("blocked", "unblocked"):
        note(f"stored order [{order} graph]")
        g = open_graph(cq, ctx, rp_t, ci_t, order)
        perm = g.order().cpu().numpy()
        assert np.array_equal(np.sort(perm), np.arange(len(rp) - 1))
        g.close()
    g = open_graph(cq, ctx, rp_t, ci_t, "input")
    with pytest.raises(cq.CQError) as e:
        g.order()
    assert e.value.status == cq.CQ_E_INVALID_ARG
    g.close()


@pytest.mark.parametrize("reorder", ORDERS)
def test_errors(cq, ctx, reorder):
    rp, ci = erdos_renyi(50, 0.2, 1)
    g = open_graph(cq, ctx, torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda(), reorder, validate=True)
    lab = torch.zeros(50, dtype=torch.int32, device="cuda")
    lab[7] = 5
    note("label out of range")
    r, _, _ = cq.score_partition(g, lab, 5, allow=(cq.CQ_E_LABEL_RANGE,))
    assert r["status"] == cq.CQ_E_LABEL_RANGE
    lab[7] = -1
    r, _, _ = cq.score_partition(g, lab, 5, allow=(cq.CQ_E_LABEL_RANGE,))
    assert r["status"] == cq.CQ_E_LABEL_RANGE
    note("workspace too small")
    lab[7] = 0
    ws = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(cq.CQError) as e:
        cq.score_partition(g, lab, 5, workspace=ws)
    assert e.value.status == cq.CQ_E_WORKSPACE
    note("workspace not 16-byte aligned")
    big = torch.empty(g.workspace_size(5) + 64, dtype=torch.uint8, device="cuda")
    with pytest.raises(cq.CQError) as e:
        cq.score_partition(g, lab, 5, workspace=big[8:])
    assert e.value.status == cq.CQ_E_INVALID_ARG
    r, _, _ = cq.score_partition(g, lab, 5, workspace=big[16:])  # 16-byte offsets are fine
    assert r["status"] == cq.CQ_OK
    note("pair export too small")
    lab2 = torch.as_tensor(np.arange(50, dtype=np.int32) % 7).cuda()
    r, _, pt = cq.score_partition(g, lab2, 7, pairs_capacity=2, allow=(cq.CQ_E_CAPACITY,))
    assert r["status"] == cq.CQ_E_CAPACITY and r["num_pairs"] > 2
    o = oracle.score(rp, ci, lab2.cpu().numpy(), 7)
    assert r["num_pairs"] == o.result["num_pairs"]
    g.close()
    note("graph checks")
    rp_bad = torch.as_tensor(np.array([0, 2, 1, 4], np.int32)).cuda()
    ci_bad = torch.as_tensor(np.array([1, 2, 0, 0], np.int32)).cuda()
    with pytest.raises(cq.CQError) as e:
        cq.Graph(ctx, rp_bad, ci_bad)
    assert e.value.status == cq.CQ_E_GRAPH_FORMAT
    rp_a, ci_a = np.array([0, 1, 1, 2], np.int32), np.array([1, 0], np.int32)  # 0->1, 2->0: not symmetric
    with pytest.raises(cq.CQError) as e:
        cq.Graph(ctx, torch.as_tensor(rp_a).cuda(), torch.as_tensor(ci_a).cuda(), validate=True)
    assert e.value.status == cq.CQ_E_GRAPH_FORMAT
    rp0, ci0 = csr_from_edges(4, [])
    g0 = cq.Graph(ctx, torch.as_tensor(rp0).cuda(), torch.zeros(1, dtype=torch.int32, device="cuda")[:0])
    with pytest.raises(cq.CQError) as e:
        cq.score_partition(g0, torch.zeros(4, dtype=torch.int32, device="cuda"), 1)
    assert e.value.status == cq.CQ_E_NO_EDGES


def test_unblocked_label_moves(cq, ctx):
    """A renumbered graph of more than 2^20 nodes stored without column blocks moves the
    caller's labels to the stored order in two passes (by super-bucket of 2^20 stored ids,
    the last one partial): the result equals the input-order graph's bit for bit and the
    oracle's; a label out of range, on either side of a super-bucket boundary, is
    reported."""
    n = (1 << 20) + 300_001
    g = lfr_graph(LFRParams(n, 6, 30, 2.0, 1.0, 20, 200, 0.3), 4500, device="cuda")
    Gu = open_graph(cq, ctx, g.row_ptr, g.col_idx, "unblocked")
    Gi = open_graph(cq, ctx, g.row_ptr, g.col_idx, "input")
    lab = perturb_labels(g.labels, g.num_labels, 0.15, 4501).contiguous()
    note("unblocked 1.35M-node graph: 15 % reassigned")
    ru, _, _ = cq.score_partition(Gu, lab, g.num_labels)
    ri, _, _ = cq.score_partition(Gi, lab, g.num_labels)
    assert ru == ri
    o = oracle.score(g.row_ptr.cpu().numpy(), g.col_idx.cpu().numpy(), lab.cpu().numpy(), g.num_labels, want_pairs=False)
    check_score(ru, o.result, "unblocked 1.35M-node graph")
    for u in (0, (1 << 20) - 1, 1 << 20, n - 1):
        bad = lab.clone()
        bad[u] = g.num_labels
        r, _, _ = cq.score_partition(Gu, bad, g.num_labels, allow=(cq.CQ_E_LABEL_RANGE,))
        assert r["status"] == cq.CQ_E_LABEL_RANGE, u
    Gu.close()
    Gi.close()


@pytest.mark.parametrize("pct", [0, 30])
def test_deterministic_and_workspace_reuse(cq, ctx, pct):
    rp, ci, lab, L = lfr_case("m100k_mu0.5", 13)
    if pct:
        lab = perturb_labels(torch.as_tensor(lab), L, pct / 100, 77).numpy()
    note(f"m100k_mu0.5 perturbed {pct}%: repeated runs, plain and reordered graph")
    rp_t, ci_t = torch.as_tensor(rp).cuda(), torch.as_tensor(ci).cuda()
    graphs = [open_graph(cq, ctx, rp_t, ci_t, order) for order in ORDERS]
    assert graphs[1].stats["owned_bytes"] > graphs[2].stats["owned_bytes"] > 0
    lab_t = torch.as_tensor(lab).cuda()
    ws = ctx.workspace(max(g.workspace_size(L) for g in graphs))
    first, _, _ = cq.score_partition(graphs[0], lab_t, L)
    o = oracle.score(rp, ci, lab, L).result
    check_score(first, o, f"m100k_mu0.5 perturbed {pct}%")
    for _ in range(4):
        for g in graphs:
            # a workspace full of 0xFF: a staged slot the kernels fail to write reads as
            # an out-of-range label and changes the counts
            ws.fill_(255)
            again, _, _ = cq.score_partition(g, lab_t, L, workspace=ws)
            assert again == first  # bitwise: the stored node order changes no bit of the result
    for g in graphs:
        g.close()


def test_full_size_l10m(cq, ctx):
    """10M-node LFR graph (avg degree 20, max 1000, mu 0.3): every count exact, the
    whole pair table exact, metrics within tolerance, in the launch configuration the
    benchmark times."""
    note("l10m: generating on the GPU")
    gr = lfr_graph(CONFIGS["l10m"], 21, device="cuda")
    rp, ci, lab = gr.row_ptr.cpu().numpy(), gr.col_idx.cpu().numpy(), gr.labels.cpu().numpy()
    note(f"l10m: n={gr.n} nnz={gr.nnz} K={gr.num_labels}; oracle")
    o = oracle.score(rp, ci, lab, gr.num_labels)
    graphs = {}
    for reorder in ORDERS:
        note(f"l10m: GPU, {reorder} graph")
        g = graphs[reorder] = open_graph(cq, ctx, gr.row_ptr, gr.col_idx, reorder)
        r, pc, pt = cq.score_partition(g, gr.labels, gr.num_labels, per_community=True,
                                       pairs_capacity=int(o.result["num_pairs"]))
        check_score(r, o.result, f"l10m reorder={reorder}")
        check_per_community(pc, o, int(o.result["m"]))
        assert np.array_equal(sort_rows(pt), o.pairs)
        if reorder == "blocked":
            assert g.last_staging == cq.CQ_STAGING_BLOCKS  # the ground truth follows the stored order
    # 30 % of the nodes reassigned: the column-blocked graph stages through its row-major
    # copy; forcing the blocks gives the same bits
    pert = perturb_labels(gr.labels, gr.num_labels, 0.30, 2130)
    note("l10m 30% reassigned: oracle")
    op = oracle.score(rp, ci, pert.cpu().numpy(), gr.num_labels)
    gb = graphs["blocked"]
    r30, _, pt30 = cq.score_partition(gb, pert, gr.num_labels, pairs_capacity=int(op.result["num_pairs"]))
    assert gb.last_staging == cq.CQ_STAGING_ROWS
    check_score(r30, op.result, "l10m 30% reassigned [blocked graph, row-major staging]")
    assert np.array_equal(sort_rows(pt30), op.pairs)
    cq.cq_context_set_row_staging(ctx.handle, 2.0)
    try:
        r30b, _, _ = cq.score_partition(gb, pert, gr.num_labels)
    finally:
        cq.cq_context_set_row_staging(ctx.handle, 1 / 16)
    assert gb.last_staging == cq.CQ_STAGING_BLOCKS and r30b == r30
    # label ids beyond the LDS histograms: global-atomic node pass after the staged move
    lab2 = (lab.astype(np.int64) * 7919 % 40009).astype(np.int32)
    note("l10m relabelled into 40009 ids: oracle")
    o2 = oracle.score(rp, ci, lab2, 40009)
    lab2_t = torch.as_tensor(lab2).cuda()
    for reorder, g in graphs.items():
        note(f"l10m relabelled into 40009 ids: GPU, {reorder} graph")
        r, _, _ = cq.score_partition(g, lab2_t, 40009)
        check_score(r, o2.result, f"l10m 40009 ids reorder={reorder}")
        g.close()


def test_graph_stats_degree_bins(cq, ctx):
    """cq_graph_get_stats: n, 2|E|, maximum degree and the power-of-two degree histogram
    (bin 0: isolated nodes; bin b: degrees in [2^(b-1), 2^b))."""
    g = lfr_graph(CONFIGS["m100k_mu0.3"], 17)
    rp = g.row_ptr.numpy().astype(np.int64)
    deg = np.diff(rp)
    rp2 = np.concatenate([rp, [rp[-1], rp[-1]]])  # two isolated nodes at the end
    G = cq.Graph(ctx, torch.as_tensor(rp2.astype(np.int32)).cuda(), g.col_idx.cuda())
    st = G.stats
    deg2 = np.concatenate([deg, [0, 0]])
    want = np.zeros(32, np.int64)
    for d in deg2:
        want[0 if d == 0 else int(d).bit_length()] += 1
    assert st["n"] == len(deg2) and st["nnz"] == int(rp[-1]) and st["max_degree"] == int(deg.max())
    assert st["degree_bins"] == want.tolist()
    G.close()
