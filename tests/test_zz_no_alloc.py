"""GPU: cq_score_partition_noalloc, the scoring entry point for callers that cannot
allocate device memory, uses the library's per-device scratch array in place of a
caller workspace and gives the results of cq_score_partition bit for bit (and so the
oracle's, Section II-B), on two calls in a row with the second input smaller, in both
graph storages; a call that needs more than the array holds is refused."""
import numpy as np
import pytest
import torch

import oracle
from cqgen import CONFIGS, lfr_graph, perturb_labels
from tests.gpu_util import check_score, note, table_equal

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


def _case(cq, ctx, g, lab, storage, what):
    note(f"noalloc: {what}, {storage} graph")
    G = cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=(storage != "input"), blocks=(storage == "blocked"))
    L = g.num_labels
    need = G.workspace_size(L)
    assert need <= cq.CQ_SCRATCH_BYTES, (what, need)
    o = oracle.score(g.row_ptr.cpu().numpy(), g.col_idx.cpu().numpy(), lab.cpu().numpy(), L)
    cap = int(o.result["num_pairs"])
    ref, pc_ref, pt_ref = cq.score_partition(G, lab, L, per_community=True, pairs_capacity=cap)
    got, pc, pt = cq.score_partition(G, lab, L, per_community=True, pairs_capacity=cap, noalloc=True)
    assert got == ref, what
    for k in pc_ref:
        if k not in ("w_in", "strength"):  # weighted graphs only; not written here
            assert torch.equal(pc[k], pc_ref[k]), (what, k)
    check_score(got, o.result, what)
    assert table_equal(pt, o.pairs, L), what
    G.close()


@pytest.mark.parametrize("storage", ["input", "blocked"])
def test_noalloc_matches_workspace_call(cq, ctx, storage):
    big = lfr_graph(CONFIGS["m100k_mu0.3"], 11, device="cuda")
    pert = perturb_labels(big.labels, big.num_labels, 0.15, 1115)
    _case(cq, ctx, big, pert, storage, "100k nodes, 15% reassigned")
    small = lfr_graph(CONFIGS["tiny_1k"], 1, device="cuda")
    _case(cq, ctx, small, small.labels, storage, "1k nodes, ground truth (after a larger call)")


def test_noalloc_refuses_oversize(cq, ctx):
    n = 12_000_000  # a ring: 2n stored entries, whose staging alone outgrows the array
    idx = torch.arange(n, dtype=torch.int64, device="cuda")
    col = torch.stack([(idx - 1) % n, (idx + 1) % n], dim=1).sort(dim=1).values.reshape(-1).to(torch.int32)
    rp = (2 * torch.arange(n + 1, dtype=torch.int64, device="cuda")).to(torch.int32)
    G = cq.Graph(ctx, rp, col)
    lab = torch.zeros(n, dtype=torch.int32, device="cuda")
    assert G.workspace_size(1) > cq.CQ_SCRATCH_BYTES
    note("noalloc: a 12M-node ring is refused")
    r, _, _ = cq.score_partition(G, lab, 1, noalloc=True, allow=(cq.CQ_E_WORKSPACE,))
    assert r["status"] == cq.CQ_E_WORKSPACE
    # the workspace entry point still scores it
    r, _, _ = cq.score_partition(G, lab, 1)
    assert r["status"] == cq.CQ_OK and r["K"] == 1 and r["Q"] == 0.0
    G.close()
    _ = np
