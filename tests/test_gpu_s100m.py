"""GPU parity at the largest size: the 100M-node LFR-style graph (average degree 10,
maximum 1,000, community sizes 50-10,000, mixing 0.3; the paper's largest
no-ground-truth network size, Section IV) scored in the caller's order and in the
stored locality order the benchmark uses (no column blocks above 2^24 nodes: the
global-atomic node pass and the unblocked edge pass at 53k labels), and two 10^8-node
partitions compared (Section II-A).  Every count, the whole pair table and the whole
contingency table bit for bit; metrics within the tolerance of oracle/parity.py."""
import numpy as np
import pytest
import torch

import oracle
from cqgen import CONFIGS, lfr_graph, perturb_labels
from tests.gpu_util import check_compare, check_per_community, check_score, note, table_equal

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


@pytest.fixture(scope="module")
def big():
    note("s100m: generating on the GPU")
    g = lfr_graph(CONFIGS["s100m"], 21, device="cuda")
    torch.cuda.synchronize()
    note(f"s100m: n={g.n} nnz={g.nnz} K={g.num_labels} max degree {g.stats['max_degree']}")
    return g


def test_score_s100m(cq, ctx, big):
    g = big
    rp, ci, lab = g.row_ptr.cpu().numpy(), g.col_idx.cpu().numpy(), g.labels.cpu().numpy()
    note("s100m score: oracle (one thread, whole graph)")
    o = oracle.score(rp, ci, lab, g.num_labels)
    del rp, ci
    npairs = int(o.result["num_pairs"])
    for order in ("unblocked", "input"):
        note(f"s100m score: GPU, {order} graph")
        G = cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=(order != "input"))
        want = cq.CQ_GRAPH_REORDER | cq.CQ_GRAPH_NO_BLOCKS if order != "input" else 0
        assert G.stats["reordered"] == want
        r, pc, pt = cq.score_partition(G, g.labels, g.num_labels, per_community=True, pairs_capacity=npairs)
        check_score(r, o.result, f"s100m {order}")
        check_per_community(pc, o, int(o.result["m"]))
        assert table_equal(pt, o.pairs, g.num_labels), f"s100m {order}: pair table differs"
        del pc, pt
        G.close()
        torch.cuda.empty_cache()


def test_compare_1e8(cq, ctx, big):
    g = big
    pert = perturb_labels(g.labels, g.num_labels, 0.10, 1010)
    a, b = g.labels.cpu().numpy(), pert.cpu().numpy()
    note(f"1e8-node compare: n={g.n} K={g.num_labels}; oracle")
    o = oracle.compare(a, g.num_labels, b, g.num_labels, want_cells=True)
    note("1e8-node compare: GPU")
    r, ct = cq.compare_partitions(ctx, g.labels, g.num_labels, pert, g.num_labels, cells_capacity=int(o.result["nnz"]))
    check_compare(r, o.result, "1e8 GT vs 10%")
    assert table_equal(ct, o.cells, g.num_labels), "1e8 compare: contingency table differs"
