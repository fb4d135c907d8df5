"""The pins are sharp: each plausible slip planted in a copy of the oracle (a dropped
factor, a wrong sign, a transposed operand, a lost square...) must make at least one
pin fail.  The mutants are built with gcc into a temporary directory on the CPU and
never touch the real oracle build.
"""
import os
import subprocess
import types
from functools import partial

import numpy as np
import pytest

import oracle
from tests import test_oracle_compare_pins as CP
from tests import test_oracle_score_pins as SP
from tests import test_oracle_weighted_pins as WP

SRC = os.path.join(os.path.dirname(oracle.__file__), "cq_oracle.c")

MUTANTS = {
    "penalty_factor": ("double term = (double)eij / (2.0 * (double)m) * dij;", "double term = (double)eij / ((double)m) * dij;"),
    "q_square": ("qt = (double)e_in / (double)m - tot * tot;", "qt = (double)e_in / (double)m - tot;"),
    "q_total": ("double tot = (double)(2 * e_in + e_out) / (2.0 * (double)m);", "double tot = (double)(e_in + e_out) / (2.0 * (double)m);"),
    "qds_sign": ("qdt = (double)e_in / (double)m * dens[c] - tdc * tdc - ns_get(&pen[c]);",
                 "qdt = (double)e_in / (double)m * dens[c] - tdc * tdc + ns_get(&pen[c]);"),
    "density": ("((double)nc[c] * (double)(nc[c] - 1)) : 0.0;\n  }\n\n  /* split penalty",
                "((double)nc[c] * (double)(nc[c])) : 0.0;\n  }\n\n  /* split penalty"),
    "pair_density_operand": ("((double)nc[ci] * (double)nc[cj]);\n    double term = (double)eij",
                             "((double)nc[ci] * (double)nc[ci]);\n    double term = (double)eij"),
    "pair_key_orient": ("if (cu < cv) keys[kk++]", "if (cu > cv) keys[kk++]"),
    "conductance": ("(double)e_out / (double)(2 * e_in + e_out) : 0.0", "(double)e_out / (double)(e_in + e_out) : 0.0"),
    "expansion": ("expa = (double)e_out / (double)nc[c];", "expa = (double)e_in / (double)nc[c];"),
    "contraction": ("contr = 2.0 * (double)e_in / (double)nc[c];", "contr = (double)e_in / (double)nc[c];"),
    "nmi_operand": ("log((double)nij * Nd / ((double)a[i] * (double)b[j]))", "log((double)nij * Nd / ((double)a[i] * (double)a[i]))"),
    "vi_square": ("log((double)nij * (double)nij / ((double)a[i] * (double)b[j]))", "log((double)nij / ((double)a[i] * (double)b[j]))"),
    "entropy_b": ("ns_add(&hb, (double)b[j] / Nd * log((double)b[j] / Nd));", "ns_add(&hb, (double)b[j] / Nd * log((double)b[j]));"),
    "f_operand": ("double f = 2.0 * (double)nij / (double)(a[i] + b[j]);", "double f = 2.0 * (double)nij / (double)(a[i] + a[i]);"),
    "nvd_colmax": ("if (nij > colmax[j]) colmax[j] = nij;", "if (nij > colmax[j]) colmax[j] = 0;"),
    "nvd_scale": ("/ (2.0 * Nd);   /* Eq. 4 */", "/ (Nd);   /* Eq. 4 */"),
    "a11_choose": ("a11 += choose2(nij);", "a11 += nij;"),
    "ari_half": ("double dd = 0.5 * (", "double dd = 1.0 * ("),
    "ji_numerator": ("out->JI = dj != 0 ? (double)a11 / (double)dj : 1.0;", "out->JI = dj != 0 ? (double)(a11 + a00) / (double)dj : 1.0;"),
    # weighted score
    "w_total_half": ("double W = ns_get(&Wsum) / 2.0;", "double W = ns_get(&Wsum);"),
    "w_q_square": ("qt = wi / W - tot * tot;", "qt = wi / W - tot;"),
    "w_strength": ("double tot = sc / (2.0 * W);", "double tot = (sc - wo) / (2.0 * W);"),
    "w_in_half": ("double wi = ns_get(&win2[c]) / 2.0,", "double wi = ns_get(&win2[c]),"),
    "w_density_weighted": ("dens[c] = nc[c] >= 2 ? (2.0 * (double)e_in) / ((double)nc[c] * (double)(nc[c] - 1)) : 0.0;  /* unweighted count */",
                           "dens[c] = nc[c] >= 2 ? ns_get(&win2[c]) / ((double)nc[c] * (double)(nc[c] - 1)) : 0.0;"),
    "w_pair_density_weighted": ("double dij = (double)eij / ((double)nc[ci] * (double)nc[cj]);   /* unweighted density */",
                                "double dij = ns_get(&wij) / ((double)nc[ci] * (double)nc[cj]);"),
    "w_pair_weight": ("keys[kk].w = (double)w[e];", "keys[kk].w = 1.0;"),
    "w_conductance": ("cond = sc > 0.0 ? wo / sc : 0.0;", "cond = sc > 0.0 ? wo / (sc - wo) : 0.0;"),
}


def _build_mutant(tmpdir, name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = os.path.join(tmpdir, f"m_{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    so = os.path.join(tmpdir, f"m_{name}.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", path, "-o", so, "-lm"])
    lib = oracle.load(so)
    ns = types.SimpleNamespace(**{k: getattr(oracle, k) for k in dir(oracle) if k.startswith("ORC_") or k == "OracleError"})
    ns.score = partial(oracle.score, _lib=lib)
    ns.compare = partial(oracle.compare, _lib=lib)
    ns.score_w = partial(oracle.score_w, _lib=lib)
    return ns


def _pins(orc):
    SP.test_two_triangles_by_triangle(orc)
    SP.test_two_triangles_three_pairs(orc)
    SP.test_star_unequal_sizes(orc)
    SP.test_all_singletons(orc, 4)
    SP.test_disjoint_cliques(orc)
    SP.test_one_community_closed_form(orc, 1)
    for case in SP._random_cases()[:4]:
        SP.test_against_dense_adjacency(orc, case)
    CP.test_worked_example(orc)
    for case in CP._cases()[:6]:
        CP.test_against_brute_force_and_sklearn(orc, case)
    CP.test_identical_partitions(orc, 0)
    CP.test_degenerate_conventions(orc)
    WP.test_two_triangles_weighted(orc)
    for case in WP._cases()[2:4]:
        WP.test_unit_weights_equal_unweighted(orc, case)
    for seed in (1, 2):
        WP.test_against_dense_weighted_algebra(orc, seed)


def test_unmutated_oracle_passes_the_pin_set(orc):
    _pins(orc)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(tmp_path, name):
    orc = _build_mutant(str(tmp_path), name)
    with pytest.raises((AssertionError, oracle.OracleError)):
        _pins(orc)
