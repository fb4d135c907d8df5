"""The multi-threaded CPU baseline the benchmark times on the host's cores gives the
oracle's results (counts bit for bit, binary64 values to the parity bar of
oracle/parity.py) at any thread count, so its timings are of the same computation."""
import numpy as np
import pytest

import cpubase
import oracle
from cqgen import CONFIGS, lfr_graph, perturb_labels, random_labels
from oracle.parity import score_mismatches


def _check(rp, ci, lab, L, what):
    o = oracle.score(rp, ci, lab, L, want_pairs=False).result
    for t in (1, 3, 8):
        r = cpubase.score(rp, ci, lab, L, t)
        bad = score_mismatches(r, o)
        assert not bad, f"{what}, {t} threads: " + "; ".join(bad)


@pytest.mark.parametrize("name,seed", [("tiny_1k", 1), ("m100k_mu0.3", 11), ("m100k_mu0.5", 13)])
def test_lfr_ground_truth_and_perturbed(name, seed):
    g = lfr_graph(CONFIGS[name], seed)
    rp, ci, lab = g.row_ptr.numpy(), g.col_idx.numpy(), g.labels.numpy()
    _check(rp, ci, lab, g.num_labels, f"{name} ground truth")
    pert = perturb_labels(g.labels, g.num_labels, 0.3, 77).numpy()
    _check(rp, ci, pert, g.num_labels, f"{name} 30% reassigned")


def test_special_partitions():
    g = lfr_graph(CONFIGS["tiny_1k"], 3)
    rp, ci = g.row_ptr.numpy(), g.col_idx.numpy()
    n = g.n
    _check(rp, ci, np.zeros(n, np.int32), 1, "one community")
    _check(rp, ci, np.arange(n, dtype=np.int32), n, "all singletons")
    _check(rp, ci, random_labels(n, 3000, 5).numpy(), 3000, "random labels, many unused ids")


def test_errors():
    g = lfr_graph(CONFIGS["tiny_1k"], 3)
    lab = g.labels.numpy().copy()
    lab[5] = g.num_labels
    with pytest.raises(RuntimeError):
        cpubase.score(g.row_ptr.numpy(), g.col_idx.numpy(), lab, g.num_labels, 4)
