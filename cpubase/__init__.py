"""Multi-threaded CPU scoring (pthreads, C) -- BENCHMARK BASELINE ONLY.

``cq_cpu_pthreads.c`` scores a partition (Q, Qds and the six measures of Section II-B)
on all host cores, organised like the paper's shared-memory algorithm (communities
assigned to threads by id modulo the thread count, Section III-B).  The benchmark times
it at one thread and at all cores, next to the single-threaded oracle, to report the
host's speedup and efficiency as the paper defines them (Eqs. 10-11).  The GPU library
never calls it; the tests check it against the oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cq_cpu_pthreads.c")
_SO = os.path.join(_HERE, "libcqcpu.so")

FIELDS_I = ("n", "m", "K", "num_pairs", "sum_ein", "sum_eout")
FIELDS_D = ("Q", "Qds", "split_penalty", "mean_intra_edges", "mean_intra_density", "mean_contraction",
            "mean_inter_edges", "mean_expansion", "mean_conductance")


class _Result(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in FIELDS_I] + [(k, ctypes.c_double) for k in FIELDS_D]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c11", "-Wall", "-pthread", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.cpu_score.restype = ctypes.c_int
        L.cpu_score.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_Result)]
        _LIB = L
    return _LIB


def host_threads() -> int:
    """Threads to use for 'all host cores': the CPU share this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    if env and env.isdigit() and int(env) > 0:
        cores = min(cores, int(env))
    return max(1, cores)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def score(row_ptr, col_idx, labels, num_labels: int, threads: int) -> dict:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    res = _Result()
    P = ctypes.c_void_p
    rc = lib().cpu_score(lab.shape[0], rp.ctypes.data_as(P), ci.ctypes.data_as(P), lab.ctypes.data_as(P),
                         int(num_labels), int(threads), ctypes.byref(res))
    if rc != 0:
        raise RuntimeError(f"cpu_score failed with status {rc}")
    return {k: getattr(res, k) for k, _ in _Result._fields_}
