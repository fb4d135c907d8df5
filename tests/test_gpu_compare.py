"""GPU parity: cq_compare_partitions against the oracle (Section II-A, Eqs. 1-7).

Pair counts and the contingency table must match bit for bit; binary64 metrics within
the tolerance in tests/gpu_util.py."""
import numpy as np
import pytest
import torch

import oracle
from cqgen import CONFIGS, lfr_graph, perturb_labels, random_labels
from tests.gpu_util import check_compare, note, sort_rows

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


def run_cmp(cq, ctx, a, La, b, Lb, what, cells=True):
    note(what)
    a = np.asarray(a, np.int32)
    b = np.asarray(b, np.int32)
    o = oracle.compare(a, La, b, Lb, want_cells=cells)
    cap = int(o.result["nnz"]) if cells else 0
    r, ct = cq.compare_partitions(ctx, torch.as_tensor(a).cuda(), La, torch.as_tensor(b).cuda(), Lb, cells_capacity=cap)
    check_compare(r, o.result, what)
    if cells:
        assert np.array_equal(sort_rows(ct), o.cells), f"{what}: contingency table differs"
    return r, o


def test_tiny_lfr(cq, ctx):
    g = lfr_graph(CONFIGS["tiny_1k"], 1)
    lab = g.labels
    pert = perturb_labels(lab, g.num_labels, 0.10, 101)
    run_cmp(cq, ctx, lab.numpy(), g.num_labels, pert.numpy(), g.num_labels, "tiny_1k GT vs 10%")


@pytest.mark.parametrize("name", ["m100k_mu0.1", "m100k_mu0.3", "m100k_mu0.5"])
def test_m100k_sweep(cq, ctx, name):
    g = lfr_graph(CONFIGS[name], 11)
    for pct in (5, 10, 15, 20, 25, 30):
        pert = perturb_labels(g.labels, g.num_labels, pct / 100, 1000 + pct)
        run_cmp(cq, ctx, g.labels.numpy(), g.num_labels, pert.numpy(), g.num_labels, f"{name} GT vs {pct}%",
                cells=(pct in (5, 30)))


def test_identical_symmetric_relabelled(cq, ctx):
    a = random_labels(20000, 300, 1).numpy()
    r, _ = run_cmp(cq, ctx, a, 300, a, 300, "identical")
    assert r["ARI"] == 1.0 and r["NVD"] == 0.0 and abs(r["NMI"] - 1.0) < 1e-15 and r["VI"] == 0.0
    b = random_labels(20000, 150, 2).numpy()
    r1, _ = run_cmp(cq, ctx, a, 300, b, 150, "random vs random")
    r2, _ = run_cmp(cq, ctx, b, 150, a, 300, "random vs random, swapped")
    for k in ("NMI", "NVD", "RI", "ARI", "JI", "VI"):
        assert abs(r1[k] - r2[k]) <= 1e-13 * max(1.0, abs(r1[k])), k
    perm = np.random.default_rng(0).permutation(500)[:300].astype(np.int32)
    r3, _ = run_cmp(cq, ctx, perm[a], 500, a, 300, "relabelled copy")
    assert r3["ARI"] == 1.0 and r3["NVD"] == 0.0


def test_degenerate(cq, ctx):
    n = 5000
    one = np.zeros(n, np.int32)
    sing = np.arange(n, dtype=np.int32)
    run_cmp(cq, ctx, one, 1, one, 1, "one vs one")
    run_cmp(cq, ctx, sing, n, sing, n, "singletons vs singletons")
    run_cmp(cq, ctx, one, 1, sing, n, "one vs singletons")
    run_cmp(cq, ctx, np.array([0, 1], np.int32), 2, np.array([0, 0], np.int32), 1, "n=2")


def test_many_labels(cq, ctx):
    # label spaces beyond LDS: global node pass, hash group tables, class splitting
    n = 200000
    a = random_labels(n, 30000, 3).numpy()
    b = ((a.astype(np.int64) * 37 + random_labels(n, 3, 4).numpy()) % 90001).astype(np.int32)
    run_cmp(cq, ctx, a, 30000, b, 90001, "30000 x 90001 labels")
    big = np.zeros(n, np.int32)
    run_cmp(cq, ctx, big, 1, (np.arange(n) * 8).astype(np.int32), 8 * n, "one row, 2e5 cells, labels = 8i")


def test_wide_counter_wraps(cq, ctx):
    # 32768 < Lb <= 65535 selects 16-bit LDS counters; cells above 65535 wrap them and
    # must come back exact through the correction log, or through the hash path once
    # the log is full.  The first node's label is the register-counted one.
    n = 200000
    a = np.zeros(n, np.int32)
    b = np.where(np.arange(n) % 2 == 0, 40000, 40001).astype(np.int32)
    b[0] = 5
    run_cmp(cq, ctx, a, 1, b, 40003, "one row, two cells of 1e5 (even+odd label wraps)")
    b2 = np.full(n, 40000, np.int32)
    b2[0] = 5
    b2[1:70000] = 40001
    run_cmp(cq, ctx, a, 1, b2, 40003, "even label 130000 entries, odd 69999")
    n3 = 8_700_000  # 40000 holds ~132 * 65536 entries: more wraps than the log holds
    a3 = np.zeros(n3, np.int32)
    b3 = np.full(n3, 40000, np.int32)
    b3[0] = 7
    b3[1::97] = 40001
    run_cmp(cq, ctx, a3, 1, b3, 40003, "log overflow: 8.7e6 entries in two cells")


def test_wave_groups(cq, ctx):
    """Ground-truth groups of fewer than 2,048 nodes are counted one per wave, larger ones
    by a whole workgroup: groups on both sides of the split, a wave group whose 2,046
    other nodes all carry distinct detected labels (its table nearly full), singletons,
    and a group of one repeated label, against the oracle with the whole table."""
    rng = np.random.default_rng(5)
    sizes = [2047, 2048, 2049, 1, 1, 300, 1500, 4000, 2046]
    a = np.repeat(np.arange(len(sizes), dtype=np.int32), sizes)
    b = np.zeros_like(a)
    off = np.concatenate([[0], np.cumsum(sizes)])
    Lb = 9000
    b[off[0]:off[1]] = np.arange(2047) + 10               # every node its own detected label
    b[off[1]:off[2]] = rng.integers(0, 7, 2048)           # few labels, large counts
    b[off[2]:off[3]] = rng.integers(0, Lb, 2049)
    b[off[5]:off[6]] = 3                                  # one label only
    b[off[6]:off[7]] = rng.integers(0, 40, 1500)
    b[off[7]:off[8]] = rng.integers(0, Lb, 4000)
    b[off[8]:off[9]] = np.concatenate([[5] * 1000, rng.integers(100, 8000, 1046)])
    perm = rng.permutation(len(a))
    run_cmp(cq, ctx, a[perm], len(sizes), b[perm], Lb, "groups around the wave split")
    # m100k ground truth against a random partition: every small group is full of distinct labels
    g = lfr_graph(CONFIGS["m100k_mu0.3"], 19)
    rl = random_labels(g.n, 20000, 191).numpy()
    run_cmp(cq, ctx, g.labels.numpy(), g.num_labels, rl, 20000, "m100k ground truth vs 20000 random labels")


def test_full_size_l10m(cq, ctx):
    """The comparison the benchmark times: ground truth of the 10M-node graph against 10 %
    of its nodes reassigned.  Every pair count and the whole contingency table exact."""
    note("l10m compare: generating on the GPU")
    g = lfr_graph(CONFIGS["l10m"], 21, device="cuda")
    pert = perturb_labels(g.labels, g.num_labels, 0.10, 1010)
    a, b = g.labels.cpu().numpy(), pert.cpu().numpy()
    note(f"l10m compare: n={g.n} K={g.num_labels}; oracle")
    o = oracle.compare(a, g.num_labels, b, g.num_labels, want_cells=True)
    note("l10m compare: GPU")
    r, ct = cq.compare_partitions(ctx, g.labels, g.num_labels, pert, g.num_labels, cells_capacity=int(o.result["nnz"]))
    check_compare(r, o.result, "l10m GT vs 10%")
    assert np.array_equal(sort_rows(ct), o.cells), "l10m: contingency table differs"


def test_errors(cq, ctx):
    a = torch.zeros(10, dtype=torch.int32, device="cuda")
    b = torch.zeros(10, dtype=torch.int32, device="cuda")
    b[3] = 9
    note("compare label out of range")
    r, _ = cq.compare_partitions(ctx, a, 1, b, 2, allow=(cq.CQ_E_LABEL_RANGE,))
    assert r["status"] == cq.CQ_E_LABEL_RANGE
    with pytest.raises(cq.CQError) as e:
        cq.compare_partitions(ctx, a[:1], 1, b[:1], 2)
    assert e.value.status == cq.CQ_E_INVALID_ARG


def test_band_path_edges(cq, ctx):
    """Both label spaces fit 16 bits: contingency cells counted per band of ground-truth
    labels.  Bands cut at 128 labels with most labels empty, tables that split into
    residue classes over two levels, a few rows sharing one large band, the largest
    valid detected label, labels out of range on either side and an export table that
    is too small."""
    n = 300_000
    a = random_labels(n, 65535, 31).numpy()
    b = random_labels(n, 65535, 32).numpy()
    run_cmp(cq, ctx, a, 65535, b, 65535, "65535 x 65535 random labels (class splits)")
    sparse = (random_labels(n, 500, 33).numpy() * 131).astype(np.int32)  # 500 used of 65,500 ids
    run_cmp(cq, ctx, sparse, 65500, a, 65535, "500 labels spread over 65500 ids")
    a3 = random_labels(400_000, 3, 34).numpy()
    b3 = ((a3.astype(np.int64) * 1000 + random_labels(400_000, 1000, 35).numpy()) % 65535).astype(np.int32)
    run_cmp(cq, ctx, a3, 3, b3, 65535, "three rows in one band, 3000 cells")
    run_cmp(cq, ctx, random_labels(50_000, 7, 36).numpy(), 7, np.full(50_000, 65534, np.int32), 65535,
            "largest valid detected label")
    a4 = torch.as_tensor(random_labels(20_000, 50, 37).numpy()).cuda()
    b4 = torch.as_tensor(random_labels(20_000, 60, 38).numpy()).cuda()
    bad_a = a4.clone()
    bad_a[5] = 50
    note("band path: ground-truth label out of range")
    r, _ = cq.compare_partitions(ctx, bad_a, 50, b4, 60, allow=(cq.CQ_E_LABEL_RANGE,))
    assert r["status"] == cq.CQ_E_LABEL_RANGE
    bad_b = b4.clone()
    bad_b[7] = 60
    note("band path: detected label out of range")
    r, _ = cq.compare_partitions(ctx, a4, 50, bad_b, 60, allow=(cq.CQ_E_LABEL_RANGE,))
    assert r["status"] == cq.CQ_E_LABEL_RANGE
    o = oracle.compare(a4.cpu().numpy(), 50, b4.cpu().numpy(), 60)
    note("band path: cell table one short")
    r, _ = cq.compare_partitions(ctx, a4, 50, b4, 60, cells_capacity=int(o.result["nnz"]) - 1,
                                 allow=(cq.CQ_E_CAPACITY,))
    assert r["status"] == cq.CQ_E_CAPACITY
