"""Writes tests/golden/oracle_tiny_1k.json: the oracle's outputs on the seeded 1,000-node
LFR-style graph (seed 1) and its 10%-perturbed partition (seed 101).  Calls only the
oracle and the input generator; the file guards against unnoticed drift of the oracle.

    python tests/golden/make_oracle_regression.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from cqgen import CONFIGS, lfr_graph, perturb_labels  # noqa: E402


def main():
    g = lfr_graph(CONFIGS["tiny_1k"], 1)
    pert = perturb_labels(g.labels, g.num_labels, 0.10, 101)
    rp, ci, lab = g.row_ptr.numpy(), g.col_idx.numpy(), g.labels.numpy()
    s_gt = oracle.score(rp, ci, lab, g.num_labels).result
    s_pt = oracle.score(rp, ci, pert.numpy(), g.num_labels).result
    c = oracle.compare(lab, g.num_labels, pert.numpy(), g.num_labels).result
    out = {"workload": "tiny_1k", "graph_seed": 1, "perturbation_seed": 101, "perturbation": 0.10,
           "score_ground_truth": s_gt, "score_perturbed": s_pt, "compare": c}
    with open(os.path.join(HERE, "oracle_tiny_1k.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
