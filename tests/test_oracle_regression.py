"""The oracle still produces the outputs recorded by tests/golden/make_oracle_regression.py
(same seeded inputs): any change to its arithmetic shows up here and must cite the passage
of the paper that justifies it."""
import json
import os

import pytest

from cqgen import CONFIGS, lfr_graph, perturb_labels

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_example_inputs_are_the_ones_the_pins_use(orc):
    w = json.load(open(os.path.join(GOLDEN, "worked_examples.json")))
    from tests import test_oracle_score_pins as SP

    assert [tuple(e) for e in w["two_triangles"]["edges"]] == SP.TWO_TRIANGLES
    assert w["compare_6"]["ground_truth"] == [0, 0, 0, 1, 1, 1]


def test_oracle_regression_tiny(orc):
    ref = json.load(open(os.path.join(GOLDEN, "oracle_tiny_1k.json")))
    g = lfr_graph(CONFIGS["tiny_1k"], ref["graph_seed"])
    pert = perturb_labels(g.labels, g.num_labels, ref["perturbation"], ref["perturbation_seed"])
    rp, ci, lab = g.row_ptr.numpy(), g.col_idx.numpy(), g.labels.numpy()
    got = {
        "score_ground_truth": orc.score(rp, ci, lab, g.num_labels).result,
        "score_perturbed": orc.score(rp, ci, pert.numpy(), g.num_labels).result,
        "compare": orc.compare(lab, g.num_labels, pert.numpy(), g.num_labels).result,
    }
    for part, vals in got.items():
        for k, v in vals.items():
            assert v == pytest.approx(ref[part][k], rel=1e-15, abs=1e-15), (part, k)
