"""Host code under sanitizers (CPU only, no GPU).

- The oracle, built with AddressSanitizer + UndefinedBehaviorSanitizer, on seeded LFR-style
  graphs and on the edge cases of its contract (isolated nodes, one community, all
  singletons, unused label ids, out-of-range labels, an odd entry count); every output
  array is allocated at exactly its stated length.  Each run's printout must equal the
  normally built oracle's results bit for bit.
- The pthreads CPU scorer under ThreadSanitizer and under ASan + UBSan at several
  thread counts, equal to the oracle.
- The scoring server's scheduler (the same header the library compiles) with a simulated
  executor: arena bounds and overlap, footprints, arrival order, grouping, injected
  failures, timeouts, one waiter per ticket, shutdown with waiters (tests/native/srv_sim.cpp),
  under ASan + UBSan and under ThreadSanitizer.

A sanitizer report makes the program exit non-zero, which fails the test.
"""
from __future__ import annotations

import os
import shutil
import struct
import subprocess

import functools

import numpy as np
import pytest
import torch

from cqgen import CONFIGS, csr_from_edges, edge_weights, lfr_graph, perturb_labels, random_labels
import oracle
from oracle.parity import score_mismatches

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_1507_05492_amd", "csrc")

ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-static-libasan", "-static-libubsan"]
TSAN = ["-fsanitize=thread"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", TSAN_OPTIONS="exitcode=66:halt_on_error=1")


def _have(tool: str) -> bool:
    return shutil.which(tool) is not None


pytestmark = pytest.mark.skipif(not (_have("gcc") and _have("g++")), reason="needs gcc and g++")


def _build(out: str, compiler: str, srcs: list[str], flags: list[str]) -> str:
    std = "-std=c++17" if compiler == "g++" else "-std=c11"
    cmd = [compiler, std, "-O1", "-g", "-Wall", "-Wextra", "-Werror", "-pthread", *flags, *srcs, "-o", out, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"build failed: {' '.join(cmd)}\n{r.stderr[-3000:]}"
    return out


def _run(args: list[str], timeout: int = 300) -> dict:
    r = subprocess.run(args, capture_output=True, text=True, env=ENV, timeout=timeout)
    assert r.returncode == 0, f"{' '.join(args)} exited {r.returncode}\n{r.stderr[-6000:]}"
    out = {}
    for line in r.stdout.splitlines():
        k, v = line.split()
        out[k] = v
    return out


@pytest.fixture(scope="module")
def bins(tmp_path_factory):
    d = tmp_path_factory.mktemp("sanitized")
    return {
        "oracle": _build(str(d / "oracle_run"), "gcc", [os.path.join(NATIVE, "oracle_run.c")],
                         ASAN + ["-I", os.path.join(ROOT, "oracle"), "-I", NATIVE]),
        "cpu_tsan": _build(str(d / "cpubase_tsan"), "gcc", [os.path.join(NATIVE, "cpubase_run.c")],
                           TSAN + ["-I", os.path.join(ROOT, "cpubase"), "-I", NATIVE]),
        "cpu_asan": _build(str(d / "cpubase_asan"), "gcc", [os.path.join(NATIVE, "cpubase_run.c")],
                           ASAN + ["-I", os.path.join(ROOT, "cpubase"), "-I", NATIVE]),
        "dir": d,
    }


# ---- expected printouts, from the normally built oracle -------------------------------

def _fnv(b: bytes) -> str:
    h = 1469598103934665603
    for x in b:
        h = ((h ^ x) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return f"{h:016x}"


def _dbits(x: float) -> str:
    return f"{struct.unpack('<Q', struct.pack('<d', float(x)))[0]:016x}"


def _put_result(res: dict, ints: tuple, dbls: tuple) -> dict:
    out = {k: str(int(res[k])) for k in ints}
    out.update({k: _dbits(res[k]) for k in dbls})
    return out


SCORE_I = ("n", "m", "K", "num_pairs", "sum_ein", "sum_eout")
SCORE_D = ("Q", "Qds", "split_penalty", "mean_intra_edges", "mean_intra_density", "mean_contraction",
           "mean_inter_edges", "mean_expansion", "mean_conductance")


def _expect_score(rp, ci, lab, L) -> dict:
    o = oracle.score(rp, ci, lab, L)
    e = {"rc": "0", **_put_result(o.result, SCORE_I, SCORE_D)}
    for k in ("size", "degsum", "ein", "eout"):
        e[k] = _fnv(np.ascontiguousarray(getattr(o, k), np.int64).tobytes())
    for k in ("intra_density", "contraction", "expansion", "conductance", "q_term", "qds_term"):
        e[k] = _fnv(np.ascontiguousarray(getattr(o, k), np.float64).tobytes())
    e["pair_i"] = _fnv(o.pairs[:, 0].astype(np.int32).tobytes())
    e["pair_j"] = _fnv(o.pairs[:, 1].astype(np.int32).tobytes())
    e["pair_cnt"] = _fnv(o.pairs[:, 2].astype(np.int64).tobytes())
    return e


def _expect_score_w(rp, ci, w, lab, L) -> dict:
    o = oracle.score_w(rp, ci, w, lab, L)
    e = {"rc": "0", **_put_result(o.result, SCORE_I, ("W", "sum_w_in", "sum_w_out") + SCORE_D)}
    for k in ("strength", "w_in", "w_out", "intra_density", "contraction", "expansion", "conductance",
              "q_term", "qds_term"):
        e[k] = _fnv(np.ascontiguousarray(getattr(o, k), np.float64).tobytes())
    e["pair_i"] = _fnv(o.pairs[:, 0].astype(np.int32).tobytes())
    e["pair_j"] = _fnv(o.pairs[:, 1].astype(np.int32).tobytes())
    e["pair_cnt"] = _fnv(o.pairs[:, 2].astype(np.int64).tobytes())
    e["pair_w"] = _fnv(np.ascontiguousarray(o.pair_w, np.float64).tobytes())
    return e


def _expect_compare(la, La, lb, Lb) -> dict:
    o = oracle.compare(la, La, lb, Lb)
    e = {"rc": "0", **_put_result(o.result, ("n", "Ka", "Kb", "nnz", "a11", "a10", "a01", "a00", "A"),
                                  ("VI", "NMI", "F", "NVD", "RI", "ARI", "JI"))}
    e["cell_i"] = _fnv(o.cells[:, 0].astype(np.int32).tobytes())
    e["cell_j"] = _fnv(o.cells[:, 1].astype(np.int32).tobytes())
    e["cell_n"] = _fnv(o.cells[:, 2].astype(np.int64).tobytes())
    return e


# ---- input files ------------------------------------------------------------------------

def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.int32)


def _write_score(path, rp, ci, lab, L, w=None):
    rp, ci, lab = _i32(rp), _i32(ci), _i32(lab)
    with open(path, "wb") as f:
        f.write(struct.pack("<iiiq", 1 if w is not None else 0, lab.shape[0], int(L), ci.shape[0]))
        f.write(rp.tobytes())
        f.write(ci.tobytes())
        if w is not None:
            f.write(np.ascontiguousarray(np.asarray(w), dtype=np.float32).tobytes())
        f.write(lab.tobytes())
    return str(path)


def _write_compare(path, la, La, lb, Lb):
    la, lb = _i32(la), _i32(lb)
    with open(path, "wb") as f:
        f.write(struct.pack("<iiii", 2, la.shape[0], int(La), int(Lb)))
        f.write(la.tobytes())
        f.write(lb.tobytes())
    return str(path)


def _perturb(lab, L, frac, seed):
    return perturb_labels(torch.as_tensor(np.asarray(lab, dtype=np.int32)), L, frac, seed).numpy()


@functools.lru_cache(maxsize=None)
def _lfr(name: str, seed: int = 21):
    g = lfr_graph(CONFIGS[name], seed)
    return g.row_ptr.numpy(), g.col_idx.numpy(), g.labels.numpy(), g.num_labels


def _score_cases():
    rp, ci, lab, L = _lfr("tiny_1k")
    n = lab.shape[0]
    yield "tiny_1k ground truth", rp, ci, lab, L
    yield "tiny_1k 30% reassigned", rp, ci, _perturb(lab, L, 0.30, 5), L
    yield "tiny_1k random labels, unused ids", rp, ci, random_labels(n, 3 * L, 6).numpy(), 3 * L
    yield "tiny_1k all singletons", rp, ci, np.arange(n), n
    yield "tiny_1k one community", rp, ci, np.zeros(n), 1
    # isolated nodes: a ring on the first half, the second half without edges
    half = 40
    rr, cc = csr_from_edges(2 * half, [(i, (i + 1) % half) for i in range(half)])
    yield "isolated nodes", rr, cc, np.arange(2 * half) % 7, 7
    yield "isolated nodes, own communities", rr, cc, np.where(np.arange(2 * half) < half, 0, 1 + np.arange(2 * half)), 2 * half + 1
    rp2, ci2, lab2, L2 = _lfr("m100k_mu0.3")
    yield "m100k ground truth", rp2, ci2, lab2, L2
    yield "m100k 15% reassigned", rp2, ci2, _perturb(lab2, L2, 0.15, 7), L2


@pytest.mark.parametrize("case", list(range(9)))
def test_oracle_score_sanitized(bins, case):
    name, rp, ci, lab, L = list(_score_cases())[case]
    path = _write_score(bins["dir"] / f"score{case}.bin", rp, ci, lab, L)
    got = _run([bins["oracle"], path])
    assert got == _expect_score(rp, ci, lab, L), name


def test_oracle_rejects_bad_inputs_sanitized(bins):
    rp, ci, lab, L = _lfr("tiny_1k")
    bad = lab.copy()
    bad[17] = L  # one label out of range
    got = _run([bins["oracle"], _write_score(bins["dir"] / "bad_label.bin", rp, ci, bad, L)])
    assert got == {"rc": str(oracle.ORC_E_LABEL)}
    # odd entry count: one entry dropped from the last row
    rp2 = rp.copy()
    rp2[-1] -= 1
    got = _run([bins["oracle"], _write_score(bins["dir"] / "odd.bin", rp2, ci[:-1], lab, L)])
    assert got == {"rc": str(oracle.ORC_E_GRAPH)}
    # no edges
    n = 10
    got = _run([bins["oracle"], _write_score(bins["dir"] / "empty.bin", np.zeros(n + 1), np.zeros(0), np.zeros(n), 1)])
    assert got == {"rc": str(oracle.ORC_E_NOEDGES)}


def test_oracle_weighted_sanitized(bins):
    rp, ci, lab, L = _lfr("tiny_1k")
    w = edge_weights(rp, ci, 3).numpy()
    for k, (lb, LL) in enumerate(((lab, L), (_perturb(lab, L, 0.3, 9), L), (np.zeros(lab.shape[0]), 1))):
        got = _run([bins["oracle"], _write_score_w(bins["dir"] / f"w{k}.bin", rp, ci, w, lb, LL)])
        assert got == _expect_score_w(rp, ci, w, lb, LL)


def _write_score_w(path, rp, ci, w, lab, L):
    return _write_score(path, rp, ci, lab, L, w=w)


def test_oracle_compare_sanitized(bins):
    _, _, lab, L = _lfr("m100k_mu0.3")
    n = lab.shape[0]
    cases = [
        (lab, L, _perturb(lab, L, 0.10, 11), L),
        (lab, L, lab, L),
        (np.zeros(n), 1, np.zeros(n), 1),
        (np.arange(n), n, np.zeros(n), 1),
        (lab, L, random_labels(n, 5 * L, 12).numpy(), 5 * L),
        (np.arange(7) % 2, 2, np.arange(7) % 3, 3),
    ]
    for k, (la, La, lb, Lb) in enumerate(cases):
        got = _run([bins["oracle"], _write_compare(bins["dir"] / f"c{k}.bin", la, La, lb, Lb)])
        assert got == _expect_compare(la, La, lb, Lb), k


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_pthreads_scorer_sanitized(bins, threads):
    rp, ci, lab, L = _lfr("m100k_mu0.3")
    cases = [(lab, L), (_perturb(lab, L, 0.3, 13), L), (random_labels(lab.shape[0], 2 * L, 14).numpy(), 2 * L)]
    for k, (lb, LL) in enumerate(cases):
        path = _write_score(bins["dir"] / f"p{threads}_{k}.bin", rp, ci, lb, LL)
        o = oracle.score(rp, ci, lb, LL, want_pairs=False).result
        for tool in ("cpu_tsan", "cpu_asan"):
            got = _run([bins[tool], path, str(threads)])
            assert got.pop("rc") == "0"
            res = {k: int(got[k]) for k in SCORE_I}
            res.update({k: struct.unpack("<d", struct.pack("<Q", int(got[k], 16)))[0] for k in SCORE_D})
            bad = score_mismatches(res, o)  # per-thread compensated sums are added in thread order
            assert not bad, (tool, k, bad)


@pytest.mark.parametrize("flags", ["asan", "tsan"])
def test_server_scheduler_sanitized(tmp_path, flags):
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    extra = ASAN if flags == "asan" else TSAN + ["-DSIM_TSAN_CLOCKWAIT"]
    exe = _build(str(tmp_path / f"srv_sim_{flags}"), "g++", [os.path.join(NATIVE, "srv_sim.cpp")], extra + inc)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "srv_sim: all passed" in r.stdout
