"""Pins for the oracle's ground-truth comparison (Section II-A: Eqs. 1-7).

The oracle is held against:
  * a hand-derived worked example (exact fractions / closed-form logs),
  * scikit-learn (NMI with arithmetic averaging = Eq. 2, rand_score = Eq. 5,
    adjusted_rand_score = Eq. 6, mutual_info_score for VI = H + H' - 2I),
  * explicit enumeration of all ordered node pairs i != j (the per-node loop of
    Alg. 4), halved, for a11, a10, a01, a00,
  * brute force over explicit node sets for F-measure and NVD (Eqs. 3, 4),
  * invariants: identical partitions, symmetry, relabelling.
"""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest
from sklearn.metrics import adjusted_rand_score, mutual_info_score, normalized_mutual_info_score, rand_score
from sklearn.metrics.cluster import contingency_matrix

REL = 1e-12


def close(a, b, rel=REL, abs_=1e-14):
    return abs(float(a) - float(b)) <= max(rel * abs(float(b)), abs_)


def test_worked_example(orc):
    # C = {0,1,2},{3,4,5}; C' = {0,1},{2,3},{4,5}.  Cells: (0,0)=2, (0,1)=1, (1,1)=1, (1,2)=2.
    # a11 = 1 + 0 + 0 + 1 = 2; sum C(|c|,2) = 6; sum C(|c'|,2) = 3; a10 = 4, a01 = 1,
    # A = 15, a00 = 8.  RI = 10/15; M = 6*3/15 = 6/5; ARI = (2 - 6/5) / (9/2 - 6/5) = 8/33;
    # JI = 2/7.  F: both rows reach 2*2/(3+2) = 4/5 -> F = 4/5.  NVD = 1 - (2+2 + 2+1+2)/12 = 1/4.
    # I = (2/3) ln 2, H = ln 2, H' = ln 3: NMI = (4/3) ln 2 / ln 6; VI = ln 3 - (1/3) ln 2.
    a = [0, 0, 0, 1, 1, 1]
    b = [0, 0, 1, 1, 2, 2]
    o = orc.compare(a, 2, b, 3)
    r = o.result
    assert (r["a11"], r["a10"], r["a01"], r["a00"], r["A"]) == (2, 4, 1, 8, 15)
    assert close(r["RI"], Fr(2, 3)) and close(r["ARI"], Fr(8, 33)) and close(r["JI"], Fr(2, 7))
    assert close(r["F"], Fr(4, 5)) and close(r["NVD"], Fr(1, 4))
    assert close(r["NMI"], (4.0 / 3.0) * math.log(2) / math.log(6))
    assert close(r["VI"], math.log(3) - math.log(2) / 3)
    assert o.cells.tolist() == [[0, 0, 2], [0, 1, 1], [1, 1, 1], [1, 2, 2]]
    assert r["nnz"] == 4 and r["Ka"] == 2 and r["Kb"] == 3


def _pairs_enumerated(a, b):
    """Visit every ordered pair of distinct nodes (as the node loop of Alg. 4 does), halve."""
    a = np.asarray(a)
    b = np.asarray(b)
    sa = a[:, None] == a[None, :]
    sb = b[:, None] == b[None, :]
    off = ~np.eye(len(a), dtype=bool)
    a11 = int((sa & sb & off).sum()) // 2
    a10 = int((sa & ~sb & off).sum()) // 2
    a01 = int((~sa & sb & off).sum()) // 2
    a00 = int((~sa & ~sb & off).sum()) // 2
    return a11, a10, a01, a00


def _pairs_loop(a, b):
    N = len(a)
    c = [0, 0, 0, 0]
    for i in range(N):
        for j in range(N):
            if i != j:
                c[(0 if a[i] == a[j] else 2) + (0 if b[i] == b[j] else 1)] += 1
    return tuple(x // 2 for x in c)


def _sets(lab):
    d = {}
    for u, c in enumerate(lab):
        d.setdefault(int(c), set()).add(u)
    return list(d.values())


def _f_brute(a, b):
    C, Cp = _sets(a), _sets(b)
    N = len(a)
    tot = Fr(0)
    for c in C:
        tot += len(c) * max(Fr(2 * len(c & cp), len(c) + len(cp)) for cp in Cp)
    return tot / N


def _nvd_brute(a, b):
    C, Cp = _sets(a), _sets(b)
    N = len(a)
    s = sum(max(len(c & cp) for cp in Cp) for c in C) + sum(max(len(cp & c) for c in C) for cp in Cp)
    return 1 - Fr(s, 2 * N)


def _cases():
    rng = np.random.default_rng(11)
    out = []
    for i in range(14):
        N = int(rng.integers(2, 160))
        La = int(rng.integers(1, 12))
        Lb = int(rng.integers(1, 15))
        a = rng.integers(0, La, N).astype(np.int32)
        if i % 3 == 0:  # perturbation of a (ground truth vs detected)
            b = a.copy() % Lb
            flip = rng.random(N) < 0.2
            b[flip] = rng.integers(0, Lb, int(flip.sum()))
        else:
            b = rng.integers(0, Lb, N).astype(np.int32)
        out.append((a, La, b.astype(np.int32), Lb))
    out.append((np.arange(30, dtype=np.int32), 30, np.zeros(30, np.int32), 1))
    out.append((np.zeros(25, np.int32), 1, np.arange(25, dtype=np.int32) % 5, 5))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"N{len(c[0])}_{c[1]}x{c[3]}")
def test_against_brute_force_and_sklearn(orc, case):
    a, La, b, Lb = case
    r = orc.compare(a, La, b, Lb).result
    assert (r["a11"], r["a10"], r["a01"], r["a00"]) == _pairs_enumerated(a, b)
    if len(a) <= 60:
        assert (r["a11"], r["a10"], r["a01"], r["a00"]) == _pairs_loop(a, b)
    assert close(r["F"], _f_brute(a, b))
    assert close(r["NVD"], _nvd_brute(a, b))
    assert close(r["RI"], rand_score(a, b), rel=1e-13)
    assert close(r["ARI"], adjusted_rand_score(a, b), rel=1e-10, abs_=1e-13)
    # sklearn returns 1.0 when both entropies are 0; so does the oracle.
    assert close(r["NMI"], normalized_mutual_info_score(a, b, average_method="arithmetic"), rel=1e-10, abs_=1e-13)
    pa = np.bincount(a) / len(a)
    pb = np.bincount(b) / len(b)
    ha = -sum(p * math.log(p) for p in pa if p > 0)
    hb = -sum(p * math.log(p) for p in pb if p > 0)
    assert close(r["VI"], ha + hb - 2 * mutual_info_score(a, b), rel=1e-10, abs_=1e-13)
    M = contingency_matrix(a, b)
    assert r["nnz"] == int((M > 0).sum())


def test_cells_match_contingency(orc):
    rng = np.random.default_rng(3)
    a = rng.integers(0, 7, 500).astype(np.int32)
    b = rng.integers(0, 9, 500).astype(np.int32)
    o = orc.compare(a, 7, b, 9)
    M = np.zeros((7, 9), np.int64)
    np.add.at(M, (a, b), 1)
    nz = np.argwhere(M > 0)
    assert np.array_equal(o.cells, np.concatenate([nz, M[M > 0][:, None]], axis=1))
    assert o.cells[:, 2].sum() == 500


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_identical_partitions(orc, seed):
    rng = np.random.default_rng(seed)
    a = rng.integers(0, 13, 400).astype(np.int32)
    r = orc.compare(a, 13, a, 13).result
    assert r["NMI"] == pytest.approx(1.0, abs=1e-15) and r["ARI"] == 1.0 and r["RI"] == 1.0
    assert r["JI"] == 1.0 and r["F"] == pytest.approx(1.0, abs=1e-15) and r["NVD"] == 0.0
    assert abs(r["VI"]) == 0.0
    # relabelled copy is the same partition
    perm = rng.permutation(20)[:13].astype(np.int32)
    r2 = orc.compare(a, 13, perm[a], 20).result
    assert r2["ARI"] == 1.0 and r2["NVD"] == 0.0 and abs(r2["NMI"] - 1.0) < 1e-15


def test_symmetry(orc):
    rng = np.random.default_rng(5)
    a = rng.integers(0, 10, 700).astype(np.int32)
    b = rng.integers(0, 6, 700).astype(np.int32)
    r1 = orc.compare(a, 10, b, 6).result
    r2 = orc.compare(b, 6, a, 10).result
    for k in ("NMI", "NVD", "RI", "ARI", "JI", "VI"):
        assert close(r1[k], r2[k], rel=1e-14), k
    assert (r1["a10"], r1["a01"]) == (r2["a01"], r2["a10"])


def test_degenerate_conventions(orc):
    one = np.zeros(10, np.int32)
    sing = np.arange(10, dtype=np.int32)
    r = orc.compare(one, 1, one, 1).result          # both one community: 0/0 -> 1
    assert r["NMI"] == 1.0 and r["ARI"] == 1.0 and r["JI"] == 1.0 and r["NVD"] == 0.0
    r = orc.compare(sing, 10, sing, 10).result      # both all singletons: ARI, JI 0/0 -> 1
    assert r["ARI"] == 1.0 and r["JI"] == 1.0 and r["RI"] == 1.0
    r = orc.compare(one, 1, sing, 10).result        # one community vs singletons
    assert r["a11"] == 0 and r["RI"] == 0.0 and r["JI"] == 0.0 and r["ARI"] == 0.0 and r["NMI"] == 0.0


def test_errors(orc):
    with pytest.raises(orc.OracleError) as e:
        orc.compare([0], 1, [0], 1)
    assert e.value.code == orc.ORC_E_ARG
    with pytest.raises(orc.OracleError) as e:
        orc.compare([0, 3], 2, [0, 0], 1)
    assert e.value.code == orc.ORC_E_LABEL
