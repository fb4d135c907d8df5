"""GPU: batched scoring (many graphs x partitions in one HIP graph replay) gives, for
every task, the same result as scoring that task alone (bit for bit), and matches the
oracle; replays pick up new label contents; the tuning cache is reused."""
import os

import numpy as np
import pytest
import torch

import oracle
from cqgen import LFRParams, lfr_graph, perturb_labels
from tests.gpu_util import check_score, note

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


def make_tasks(cq, ctx, ngraphs=10, seed=500):
    rng = np.random.default_rng(seed)
    graphs, tasks, host = [], [], []
    for i in range(ngraphs):
        n = int(np.exp(rng.uniform(np.log(2000), np.log(60000))))
        avg = float(rng.uniform(10, 30))
        mu = float(rng.uniform(0.1, 0.5))
        p = LFRParams(n, avg, int(5 * avg), 2.0, 1.0, 20, max(40, min(1000, n // 5)), mu)
        g = lfr_graph(p, seed + i, device="cuda")
        G = cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=(i % 2 == 0))
        graphs.append((g, G))
        parts = [g.labels] + [perturb_labels(g.labels, g.num_labels, f, 31000 + 10 * i + k)
                              for k, f in enumerate((0.05, 0.15, 0.30))]
        if i == 3:  # a fifth partition of the same graph, with sparse label ids: opens a second group
            parts.append((g.labels.long() * 3).to(torch.int32))
        for k, lab in enumerate(parts):
            L = g.num_labels * (3 if k == 4 else 1)
            lab = lab.contiguous()
            tasks.append((G, lab, L))
            host.append((g, lab, L))
    return graphs, tasks, host


def test_batch_equals_single_and_oracle(cq, ctx):
    note("batch: building 10 graphs x 4-5 partitions")
    graphs, tasks, host = make_tasks(cq, ctx)
    for use_graph in (True, False):
        note(f"batch: use_graph={use_graph}")
        b = cq.Batch(ctx, tasks, autotune=True, use_graph=use_graph)
        assert b.tuning["num_groups"] == 11
        if use_graph:
            assert b.tuning["graph_nodes"] >= 9
        res = b.run_sync()
        for i, (G, lab, L) in enumerate(tasks):
            single, _, _ = cq.score_partition(G, lab, L)
            single.pop("status")
            r = dict(res[i])
            r.pop("status")
            assert r == single, f"task {i}"
        b.close()
    note("batch vs oracle on a few tasks")
    b = cq.Batch(ctx, tasks, autotune=False)
    res = b.run_sync()
    for i in (0, 5, 14, 17, len(tasks) - 1):
        g, lab, L = host[i]
        o = oracle.score(g.row_ptr.cpu().numpy(), g.col_idx.cpu().numpy(), lab.cpu().numpy(), L, want_pairs=False)
        check_score(res[i], o.result, f"batch task {i}")
    b.close()


def test_graph_replays_track_label_contents(cq, ctx):
    graphs, tasks, host = make_tasks(cq, ctx, ngraphs=4, seed=900)
    b = cq.Batch(ctx, tasks, autotune=False, use_graph=True)
    originals = [lab.clone() for _, lab, _ in tasks]
    for rep in range(4):
        note(f"replay {rep}")
        # eager work between replays: rewrite every label array in place
        for k, (G, lab, L) in enumerate(tasks):
            src = originals[(k + rep) % len(originals)]
            if src.numel() == lab.numel() and int(src.max()) < L:
                lab.copy_(src)
        torch.cuda.synchronize()
        expect = [cq.score_partition(G, lab, L)[0] for G, lab, L in tasks]
        res = b.run_sync()
        for i in range(len(tasks)):
            e = dict(expect[i]); e.pop("status")
            r = dict(res[i]); r.pop("status")
            assert r == e, (rep, i)
    b.close()


def test_large_task_spread_over_xcds(cq, ctx):
    """A graph large enough that its node chunks and edge tiles are dealt to all eight
    XCDs (more than 1/16 of the batch's work), beside small graphs that go whole to one
    XCD, and the large graph's partitions alone (every task dealt): each task equals its
    single call bit for bit."""
    note("batch: one 300k-node graph x 4 partitions + 3 small graphs")
    big = lfr_graph(LFRParams(300_000, 16, 80, 2.0, 1.0, 20, 1000, 0.3), 4100, device="cuda")
    Gb = cq.Graph(ctx, big.row_ptr, big.col_idx, reorder=True)
    big_tasks = [(Gb, big.labels.contiguous(), big.num_labels)] + [
        (Gb, perturb_labels(big.labels, big.num_labels, f, 4110 + k).contiguous(), big.num_labels)
        for k, f in enumerate((0.05, 0.15, 0.30))]
    small = []
    for i in range(3):
        g = lfr_graph(LFRParams(3000 + 500 * i, 12, 60, 2.0, 1.0, 20, 300, 0.2), 4200 + i, device="cuda")
        small.append((g, cq.Graph(ctx, g.row_ptr, g.col_idx, reorder=(i != 1))))
    small_tasks = [(G, g.labels.contiguous(), g.num_labels) for g, G in small]
    for tasks in (big_tasks + small_tasks, big_tasks):
        b = cq.Batch(ctx, tasks, autotune=False, use_graph=True)
        res = b.run_sync()
        for i, (G, lab, L) in enumerate(tasks):
            single, _, _ = cq.score_partition(G, lab, L)
            single.pop("status")
            r = dict(res[i])
            r.pop("status")
            assert r == single, f"task {i} of {len(tasks)}"
        b.close()
    o = oracle.score(big.row_ptr.cpu().numpy(), big.col_idx.cpu().numpy(), big_tasks[3][1].cpu().numpy(), big.num_labels,
                     want_pairs=False)
    b = cq.Batch(ctx, big_tasks, autotune=False)
    check_score(b.run_sync()[3], o.result, "dealt batch task, 30 % reassigned")
    b.close()


def test_tuning_cache_and_errors(cq, ctx, tmp_path, monkeypatch):
    monkeypatch.setenv("CQ_TUNE_CACHE", str(tmp_path / "tune.jsonl"))
    graphs, tasks, _ = make_tasks(cq, ctx, ngraphs=3, seed=1300)
    b1 = cq.Batch(ctx, tasks, autotune=True)
    assert b1.tuning["from_cache"] == 0 and b1.tuning["tuned_ms"] > 0
    b2 = cq.Batch(ctx, tasks, autotune=True)
    assert b2.tuning["from_cache"] == 1
    assert (b2.tuning["gather_rows"], b2.tuning["group_blocks_per_cu"]) == (b1.tuning["gather_rows"], b1.tuning["group_blocks_per_cu"])
    assert os.path.exists(tmp_path / "tune.jsonl")
    b1.close(); b2.close()
    note("batch label error")
    G, lab, L = tasks[1]
    bad = lab.clone()
    bad[5] = L + 3
    b3 = cq.Batch(ctx, [tasks[0], (G, bad, L)], autotune=False)
    res = b3.run_sync(allow=(cq.CQ_E_LABEL_RANGE,))
    assert res[0]["status"] == cq.CQ_E_LABEL_RANGE and res[0]["device_flags"] == 0 and res[1]["device_flags"] != 0
    b3.close()
    with pytest.raises(cq.CQError) as e:
        cq.Batch(ctx, [(G, lab, 20000)], autotune=False)
    assert e.value.status == cq.CQ_E_INVALID_ARG
