"""The LFR-style generator realises the workload shapes it is asked for: a simple
symmetric graph whose mean degree, maximum degree and mixing fraction match the
parameters (rejected stubs are rewired rather than dropped), and community sizes in
range.  Inputs only: the generator holds none of the metrics' arithmetic."""
import numpy as np
import pytest
import torch

from cqgen import CONFIGS, LFRParams, lfr_graph


def _shape(g):
    rp = g.row_ptr.numpy().astype(np.int64)
    ci = g.col_idx.numpy().astype(np.int64)
    lab = g.labels.numpy()
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    return rp, ci, lab, rows


@pytest.mark.parametrize("name", ["m100k_mu0.1", "m100k_mu0.3", "m100k_mu0.5"])
def test_realised_shape(name):
    p = CONFIGS[name]
    g = lfr_graph(p, 11)
    rp, ci, lab, rows = _shape(g)
    deg = np.diff(rp)
    assert abs(deg.mean() - p.avg_degree) <= 0.02 * p.avg_degree, deg.mean()
    assert deg.max() >= 0.95 * p.max_degree and deg.max() <= p.max_degree
    mu = float(np.mean(lab[rows] != lab[ci]))
    assert abs(mu - p.mu) <= 0.02, mu
    sizes = np.bincount(lab, minlength=g.num_labels)
    assert sizes.min() >= p.min_comm and sizes.max() <= p.max_comm
    # stubs dropped after rewiring are a small share of those drawn
    assert g.stats["stubs_dropped"] <= 0.01 * g.stats["stubs_drawn"]


def test_simple_symmetric_csr():
    g = lfr_graph(CONFIGS["m100k_mu0.3"], 12)
    rp, ci, lab, rows = _shape(g)
    assert (rows != ci).all(), "self-loop"
    key = rows * g.n + ci
    assert (np.diff(key) > 0).all(), "rows unsorted or repeated entries"
    rev = np.sort(ci * g.n + rows)
    assert np.array_equal(rev, key), "not symmetric"


def test_hubs_reach_max_degree():
    """Config L's degree range (avg 20, max 1000) on a 1M-node graph: hubs keep their
    drawn degree, which dropping repeated pairs would cut by a fifth."""
    p = LFRParams(1_000_000, 20, 1_000, 2.0, 1.0, 50, 5_000, 0.3)
    torch.set_num_threads(8)
    g = lfr_graph(p, 21)
    deg = np.diff(g.row_ptr.numpy().astype(np.int64))
    assert abs(deg.mean() - 20) <= 0.4, deg.mean()
    assert deg.max() >= 990


def test_seeded():
    a = lfr_graph(CONFIGS["tiny_1k"], 5)
    b = lfr_graph(CONFIGS["tiny_1k"], 5)
    assert torch.equal(a.col_idx, b.col_idx) and torch.equal(a.labels, b.labels)
