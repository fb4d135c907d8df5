"""ctypes binding of the C ABI in ``include/cq.h`` (argument marshalling only).

Every function named ``cq_*`` here calls the library function of the same name.
The helpers at the bottom (:class:`Context`, :class:`Graph`, :func:`score_partition`,
:func:`compare_partitions`) take torch tensors for device memory and the current
torch stream, size the workspace and convert results to dicts.  All computation
happens in ``libcq.so``; if it is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcq.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cq.h")

CQ_OK = 0
CQ_SCRATCH_BYTES = 64 << 20  # include/cq.h: the library's per-device scratch array
CQ_STAGING_ROWS_ONLY, CQ_STAGING_BLOCKS, CQ_STAGING_ROWS = 0, 1, 2
CQ_E_INVALID_ARG = -1
CQ_E_LABEL_RANGE = -2
CQ_E_GRAPH_FORMAT = -3
CQ_E_OVERFLOW = -4
CQ_E_WORKSPACE = -5
CQ_E_NO_EDGES = -6
CQ_E_DEVICE = -7
CQ_E_BUSY = -8
CQ_E_CANCELLED = -9
CQ_E_CAPACITY = -10
CQ_VALIDATE_GRAPH = 1
CQ_GRAPH_REORDER = 2
CQ_GRAPH_NO_BLOCKS = 4
CQ_GRAPH_BLOCKS = 8

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t


class CQError(RuntimeError):
    def __init__(self, status: int, message: str = ""):
        self.status = status
        super().__init__(f"{_name(status)}: {message}" if message else _name(status))


class ScoreResult(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "m", "K", "num_pairs", "sum_ein", "sum_eout")] + [
        ("sum_degsum_sq", ctypes.c_uint64)
    ] + [(k, ctypes.c_double) for k in (
        "Q", "Qds", "split_penalty", "mean_intra_edges", "mean_intra_density", "mean_contraction",
        "mean_inter_edges", "mean_expansion", "mean_conductance",
    )] + [("device_flags", ctypes.c_uint32), ("weighted", ctypes.c_uint32)] + [
        (k, ctypes.c_double) for k in ("total_weight", "sum_w_in", "sum_w_out")] + [
        ("staging", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class CompareResult(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("n", "Ka", "Kb", "nnz", "a11", "a10", "a01", "a00", "A")] + [
        (k, ctypes.c_double) for k in ("VI", "NMI", "F", "NVD", "RI", "ARI", "JI")
    ] + [("device_flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


PER_COMMUNITY_FIELDS = ("size", "degsum", "ein", "eout", "intra_density", "contraction", "expansion",
                        "conductance", "q_term", "qds_term", "w_in", "strength")


class PerCommunity(ctypes.Structure):
    _fields_ = [(k, _P) for k in PER_COMMUNITY_FIELDS]


class PairTable(ctypes.Structure):
    _fields_ = [("ci", _P), ("cj", _P), ("count", _P), ("capacity", _I64)]


CellTable = PairTable


class BatchTask(ctypes.Structure):
    _fields_ = [("graph", _P), ("d_labels", _P), ("num_labels", _I32)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("gather_rows", _I32), ("group_blocks_per_cu", _I32), ("tuned_ms", ctypes.c_double),
                ("from_cache", _I32), ("graph_nodes", _I32), ("num_groups", _I32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("num_slots", _I32), ("max_batch", _I32), ("memory_budget", _I64), ("small_nnz", _I64)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, _I64) for k in ("submitted", "completed", "failed", "rejected", "launches", "grouped_requests")] + [
        (k, ctypes.c_double) for k in ("p50_ms", "p99_ms", "mean_ms", "max_ms", "busy_s")] + [("peak_bytes", _I64)]


CQ_BATCH_AUTOTUNE = 1
CQ_BATCH_NO_GRAPH = 2


class GraphStats(ctypes.Structure):
    _fields_ = [("n", _I64), ("nnz", _I64), ("m", _I64), ("max_degree", _I64), ("validated", ctypes.c_uint32),
                ("reordered", ctypes.c_uint32), ("owned_bytes", _I64), ("weighted", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("total_weight", ctypes.c_double), ("clusters", _I64),
                ("largest_cluster", _I64), ("degree_bins", _I64 * 32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python paper_1507_05492_amd/build.py` (needs hipcc)")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "cq_status_string": (ctypes.c_char_p, [_I32]),
        "cq_context_create": (_I32, [ctypes.c_int, _P, ctypes.POINTER(_P)]),
        "cq_context_set_stream": (_I32, [_P, _P]),
        "cq_context_destroy": (None, [_P]),
        "cq_context_last_error": (ctypes.c_char_p, [_P]),
        "cq_graph_load": (_I32, [_P, _I32, _I64, _P, _P, ctypes.c_uint32, ctypes.POINTER(_P)]),
        "cq_graph_load_weighted": (_I32, [_P, _I32, _I64, _P, _P, _P, ctypes.c_uint32, ctypes.POINTER(_P)]),
        "cq_graph_get_stats": (_I32, [_P, ctypes.POINTER(GraphStats)]),
        "cq_graph_copy_order": (_I32, [_P, _P, _P]),
        "cq_graph_release": (None, [_P]),
        "cq_score_workspace_size": (_SZ, [_P, _I32]),
        "cq_score_partition": (_I32, [_P, _P, _P, _I32, _P, _SZ, ctypes.POINTER(ScoreResult), _P, _P]),
        "cq_score_partition_async": (_I32, [_P, _P, _P, _I32, _P, _SZ, _P, _P, _P]),
        "cq_score_partition_noalloc": (_I32, [_P, _P, _P, _I32, ctypes.POINTER(ScoreResult), _P, _P]),
        "cq_compare_workspace_size": (_SZ, [_I32, _I32, _I32]),
        "cq_compare_partitions": (_I32, [_P, _I32, _P, _I32, _P, _I32, _P, _SZ, ctypes.POINTER(CompareResult), _P]),
        "cq_compare_partitions_async": (_I32, [_P, _I32, _P, _I32, _P, _I32, _P, _SZ, _P, _P]),
        "cq_context_enable_timing": (_I32, [_P, ctypes.c_int]),
        "cq_context_set_row_staging": (_I32, [_P, ctypes.c_double]),
        "cq_context_time_stages": (_I32, [_P, ctypes.c_uint32]),
        "cq_context_stage_times": (_I32, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64), _I32]),
        "cq_stage_name": (ctypes.c_char_p, [_I32]),
        "cq_batch_plan_create": (_I32, [_P, ctypes.POINTER(BatchTask), _I32, ctypes.c_uint32, ctypes.POINTER(_P)]),
        "cq_batch_workspace_size": (_SZ, [_P]),
        "cq_batch_bind": (_I32, [_P, _P, _SZ, _P]),
        "cq_batch_run": (_I32, [_P]),
        "cq_batch_run_sync": (_I32, [_P, ctypes.POINTER(ScoreResult)]),
        "cq_batch_get_tuning": (_I32, [_P, ctypes.POINTER(BatchTuning)]),
        "cq_batch_plan_destroy": (None, [_P]),
        "cq_server_create": (_I32, [_P, ctypes.POINTER(ServerConfig), ctypes.POINTER(_P)]),
        "cq_server_submit_score": (_I32, [_P, _P, _P, _I32, ctypes.POINTER(ctypes.c_uint64)]),
        "cq_server_submit_compare": (_I32, [_P, _I32, _P, _I32, _P, _I32, ctypes.POINTER(ctypes.c_uint64)]),
        "cq_server_wait": (_I32, [_P, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(_I32), ctypes.POINTER(ScoreResult),
                                  ctypes.POINTER(CompareResult), ctypes.POINTER(ctypes.c_double)]),
        "cq_server_get_stats": (_I32, [_P, ctypes.POINTER(ServerStats)]),
        "cq_server_reset_stats": (_I32, [_P]),
        "cq_server_destroy": (None, [_P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


_lib = _load()


def header_functions() -> list[str]:
    """Names of the functions declared in include/cq.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\**\s+\**\s*(cq_[a-z_]+)\s*\(", txt, re.M)))


def _name(status: int) -> str:
    return _lib.cq_status_string(status).decode()


# ---- raw C ABI (same names) -------------------------------------------------
def cq_status_string(status: int) -> str:
    return _name(status)


def cq_context_create(device: int = 0, stream: int | None = None) -> int:
    out = _P()
    st = _lib.cq_context_create(device, stream, ctypes.byref(out))
    if st != CQ_OK:
        raise CQError(st, "cq_context_create")
    return out.value


def cq_context_set_stream(ctx: int, stream: int | None) -> None:
    st = _lib.cq_context_set_stream(ctx, stream)
    if st != CQ_OK:
        raise CQError(st)


def cq_context_destroy(ctx: int) -> None:
    _lib.cq_context_destroy(ctx)


def cq_context_last_error(ctx: int) -> str:
    return _lib.cq_context_last_error(ctx).decode()


CQ_MAX_STAGES = 12


def cq_context_enable_timing(ctx: int, enable: bool) -> None:
    st = _lib.cq_context_enable_timing(ctx, 1 if enable else 0)
    if st != CQ_OK:
        raise CQError(st)


def cq_context_time_stages(ctx: int, stage_mask: int) -> None:
    st = _lib.cq_context_time_stages(ctx, stage_mask)
    if st != CQ_OK:
        raise CQError(st)


def stage_id(name: str) -> int:
    """Stage id of a stage name (as cq_context_stage_times reports it)."""
    for i in range(32):
        if cq_stage_name(i) == name:
            return i
    raise KeyError(name)


def cq_stage_name(s: int) -> str:
    return _lib.cq_stage_name(s).decode()


def cq_context_stage_times(ctx: int) -> dict:
    """{stage name: (total ms, count)} for stages that ran while timing was on."""
    tot = (ctypes.c_double * CQ_MAX_STAGES)()
    cnt = (_I64 * CQ_MAX_STAGES)()
    st = _lib.cq_context_stage_times(ctx, tot, cnt, CQ_MAX_STAGES)
    if st != CQ_OK:
        raise CQError(st)
    return {cq_stage_name(i): (tot[i], cnt[i]) for i in range(CQ_MAX_STAGES) if cnt[i] > 0}


def _check(ctx: int, st: int, allow=(CQ_OK,)) -> int:
    if st not in allow:
        raise CQError(st, cq_context_last_error(ctx))
    return st


def cq_graph_load(ctx: int, n: int, nnz: int, d_row_ptr: int, d_col_idx: int, flags: int = 0) -> int:
    out = _P()
    _check(ctx, _lib.cq_graph_load(ctx, n, nnz, d_row_ptr, d_col_idx, flags, ctypes.byref(out)))
    return out.value


def cq_graph_load_weighted(ctx: int, n: int, nnz: int, d_row_ptr: int, d_col_idx: int, d_weights: int,
                           flags: int = 0) -> int:
    out = _P()
    _check(ctx, _lib.cq_graph_load_weighted(ctx, n, nnz, d_row_ptr, d_col_idx, d_weights, flags, ctypes.byref(out)))
    return out.value


def cq_graph_copy_order(ctx: int, g: int, d_order: int) -> None:
    _check(ctx, _lib.cq_graph_copy_order(ctx, g, d_order))


def cq_graph_get_stats(g: int) -> dict:
    s = GraphStats()
    st = _lib.cq_graph_get_stats(g, ctypes.byref(s))
    if st != CQ_OK:
        raise CQError(st)
    out = {k: getattr(s, k) for k, _ in GraphStats._fields_ if k != "pad"}
    out["degree_bins"] = list(out["degree_bins"])
    return out


def cq_graph_release(g: int) -> None:
    _lib.cq_graph_release(g)


def cq_score_workspace_size(g: int, num_labels: int) -> int:
    return _lib.cq_score_workspace_size(g, num_labels)


def cq_compare_workspace_size(n: int, num_labels_a: int, num_labels_b: int) -> int:
    return _lib.cq_compare_workspace_size(n, num_labels_a, num_labels_b)


def cq_score_partition(ctx, g, d_labels, num_labels, d_ws, ws_bytes, per_comm: PerCommunity | None = None,
                       pairs: PairTable | None = None, allow=(CQ_OK,)) -> tuple[int, ScoreResult]:
    res = ScoreResult()
    st = _lib.cq_score_partition(ctx, g, d_labels, num_labels, d_ws, ws_bytes, ctypes.byref(res),
                                 ctypes.byref(per_comm) if per_comm is not None else None,
                                 ctypes.byref(pairs) if pairs is not None else None)
    return _check(ctx, st, allow), res


def cq_context_set_row_staging(ctx, change_fraction: float) -> None:
    _check(ctx, _lib.cq_context_set_row_staging(ctx, float(change_fraction)))


def cq_score_partition_noalloc(ctx, g, d_labels, num_labels, per_comm: PerCommunity | None = None,
                               pairs: PairTable | None = None, allow=(CQ_OK,)) -> tuple[int, ScoreResult]:
    res = ScoreResult()
    st = _lib.cq_score_partition_noalloc(ctx, g, d_labels, num_labels, ctypes.byref(res),
                                         ctypes.byref(per_comm) if per_comm is not None else None,
                                         ctypes.byref(pairs) if pairs is not None else None)
    return _check(ctx, st, allow), res


def cq_score_partition_async(ctx, g, d_labels, num_labels, d_ws, ws_bytes, d_out, per_comm=None, pairs=None) -> None:
    _check(ctx, _lib.cq_score_partition_async(ctx, g, d_labels, num_labels, d_ws, ws_bytes, d_out,
                                              ctypes.byref(per_comm) if per_comm is not None else None,
                                              ctypes.byref(pairs) if pairs is not None else None))


def cq_compare_partitions(ctx, n, d_a, La, d_b, Lb, d_ws, ws_bytes, cells: CellTable | None = None,
                          allow=(CQ_OK,)) -> tuple[int, CompareResult]:
    res = CompareResult()
    st = _lib.cq_compare_partitions(ctx, n, d_a, La, d_b, Lb, d_ws, ws_bytes, ctypes.byref(res),
                                    ctypes.byref(cells) if cells is not None else None)
    return _check(ctx, st, allow), res


def cq_compare_partitions_async(ctx, n, d_a, La, d_b, Lb, d_ws, ws_bytes, d_out, cells=None) -> None:
    _check(ctx, _lib.cq_compare_partitions_async(ctx, n, d_a, La, d_b, Lb, d_ws, ws_bytes, d_out,
                                                 ctypes.byref(cells) if cells is not None else None))


def cq_batch_plan_create(ctx: int, tasks: list[tuple[int, int, int]], flags: int = 0) -> int:
    """tasks: (graph handle, device label pointer, num_labels)."""
    arr = (BatchTask * len(tasks))(*[BatchTask(g, lab, L) for g, lab, L in tasks])
    out = _P()
    _check(ctx, _lib.cq_batch_plan_create(ctx, arr, len(tasks), flags, ctypes.byref(out)))
    return out.value


def cq_batch_workspace_size(plan: int) -> int:
    return _lib.cq_batch_workspace_size(plan)


def cq_batch_bind(ctx: int, plan: int, d_ws: int, ws_bytes: int, d_results: int) -> None:
    _check(ctx, _lib.cq_batch_bind(plan, d_ws, ws_bytes, d_results))


def cq_batch_run(ctx: int, plan: int) -> None:
    _check(ctx, _lib.cq_batch_run(plan))


def cq_batch_run_sync(ctx: int, plan: int, num_tasks: int, allow=(CQ_OK,)) -> tuple[int, list[ScoreResult]]:
    res = (ScoreResult * num_tasks)()
    st = _lib.cq_batch_run_sync(plan, res)
    return _check(ctx, st, allow), list(res)


def cq_batch_get_tuning(plan: int) -> dict:
    t = BatchTuning()
    st = _lib.cq_batch_get_tuning(plan, ctypes.byref(t))
    if st != CQ_OK:
        raise CQError(st)
    return {k: getattr(t, k) for k, _ in BatchTuning._fields_}


def cq_batch_plan_destroy(plan: int) -> None:
    _lib.cq_batch_plan_destroy(plan)


def cq_server_create(ctx: int, num_slots: int, max_batch: int, memory_budget: int, small_nnz: int) -> int:
    cfg = ServerConfig(num_slots, max_batch, memory_budget, small_nnz)
    out = _P()
    _check(ctx, _lib.cq_server_create(ctx, ctypes.byref(cfg), ctypes.byref(out)))
    return out.value


def cq_server_submit_score(ctx: int, srv: int, g: int, h_labels: int, num_labels: int) -> int:
    t = ctypes.c_uint64()
    _check(ctx, _lib.cq_server_submit_score(srv, g, h_labels, num_labels, ctypes.byref(t)))
    return t.value


def cq_server_submit_compare(ctx: int, srv: int, n: int, h_a: int, La: int, h_b: int, Lb: int) -> int:
    t = ctypes.c_uint64()
    _check(ctx, _lib.cq_server_submit_compare(srv, n, h_a, La, h_b, Lb, ctypes.byref(t)))
    return t.value


def cq_server_wait(ctx: int, srv: int, ticket: int, timeout_ms: float = -1.0):
    """Returns (call status, request status, score dict | None, compare dict | None, latency ms)."""
    rs = _I32()
    sr = ScoreResult()
    cr = CompareResult()
    lat = ctypes.c_double()
    st = _lib.cq_server_wait(srv, ticket, timeout_ms, ctypes.byref(rs), ctypes.byref(sr), ctypes.byref(cr), ctypes.byref(lat))
    if st not in (CQ_OK, CQ_E_BUSY):
        raise CQError(st, cq_context_last_error(ctx))
    return st, rs.value, as_dict(sr), as_dict(cr), lat.value


def cq_server_get_stats(srv: int) -> dict:
    s = ServerStats()
    st = _lib.cq_server_get_stats(srv, ctypes.byref(s))
    if st != CQ_OK:
        raise CQError(st)
    return {k: getattr(s, k) for k, _ in ServerStats._fields_}


def cq_server_reset_stats(srv: int) -> None:
    _lib.cq_server_reset_stats(srv)


def cq_server_destroy(srv: int) -> None:
    _lib.cq_server_destroy(srv)


# ---- torch conveniences -------------------------------------------------------
def _torch():
    import torch

    return torch


def _dev_i32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.int32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous int32 CUDA tensor")
    return t


def _dev_f32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


# Fields that describe how a call ran rather than what it computed: left out of result
# dicts, so that results of the same inputs compare equal whatever path produced them.
_INFO_FIELDS = ("reserved", "staging")


def as_dict(res) -> dict:
    return {k: getattr(res, k) for k, _ in res._fields_ if k not in _INFO_FIELDS}


class Context:
    """A library context on a torch device, enqueueing on the current torch stream."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.device = device
        self.stream = torch.cuda.current_stream(device)
        self.handle = cq_context_create(device, self.stream.cuda_stream)
        self._ws = None

    def use_current_stream(self):
        torch = _torch()
        self.stream = torch.cuda.current_stream(self.device)
        cq_context_set_stream(self.handle, self.stream.cuda_stream)

    def workspace(self, nbytes: int):
        torch = _torch()
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{self.device}")
        return self._ws

    def close(self):
        if self.handle:
            cq_context_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A registered graph; keeps its CSR tensors alive while registered."""

    def __init__(self, ctx: Context, row_ptr, col_idx, validate: bool = False, reorder: bool = False,
                 blocks: bool | None = None, weights=None):
        """reorder: store in a locality order; blocks (with reorder): None = column blocks
        when the library's size rule says so, True = always (n <= 2^24), False = never.
        weights: float32 per stored entry (an edge-weighted graph), or None."""
        self.ctx = ctx
        self.row_ptr = _dev_i32(row_ptr, "row_ptr")
        self.col_idx = _dev_i32(col_idx, "col_idx")
        self.n = self.row_ptr.numel() - 1
        self.nnz = self.col_idx.numel()
        self.handle = 0
        self.last_staging = None  # CQ_STAGING_* of the last score_partition call on this graph
        flags = ((CQ_VALIDATE_GRAPH if validate else 0) | (CQ_GRAPH_REORDER if reorder else 0)
                 | (CQ_GRAPH_BLOCKS if reorder and blocks is True else 0)
                 | (CQ_GRAPH_NO_BLOCKS if reorder and blocks is False else 0))
        col = self.col_idx.data_ptr() if self.nnz else None
        if weights is None:
            self.weights = None
            self.handle = cq_graph_load(ctx.handle, self.n, self.nnz, self.row_ptr.data_ptr(), col, flags)
        else:
            self.weights = _dev_f32(weights, "weights")
            if self.weights.numel() != self.nnz:
                raise ValueError("weights must have one entry per stored CSR entry")
            self.handle = cq_graph_load_weighted(ctx.handle, self.n, self.nnz, self.row_ptr.data_ptr(), col,
                                                 self.weights.data_ptr() if self.nnz else None, flags)
        self.stats = cq_graph_get_stats(self.handle)

    def workspace_size(self, num_labels: int) -> int:
        return cq_score_workspace_size(self.handle, num_labels)

    def order(self):
        """int32 tensor: caller id of every stored node (graphs loaded with reorder=True)."""
        out = _torch().empty(self.n, dtype=_torch().int32, device=self.row_ptr.device)
        cq_graph_copy_order(self.ctx.handle, self.handle, out.data_ptr())
        return out

    def close(self):
        if self.handle:
            cq_graph_release(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def score_partition(graph: Graph, labels, num_labels: int, *, per_community: bool = False,
                    pairs_capacity: int = 0, workspace=None, noalloc: bool = False, allow=(CQ_OK,)):
    """Score a partition; returns (result dict, per-community dict | None, pairs tensor | None).
    noalloc=True calls cq_score_partition_noalloc (the library's scratch array, no workspace)."""
    torch = _torch()
    labels = _dev_i32(labels, "labels")
    if labels.numel() != graph.n:
        raise ValueError("labels must have one entry per node")
    ctx = graph.ctx
    ws = None
    if not noalloc:
        need = graph.workspace_size(num_labels)
        ws = workspace if workspace is not None else ctx.workspace(need)
    dev = labels.device
    pc = None
    pc_t = None
    if per_community:
        pc_t = {}
        for k in PER_COMMUNITY_FIELDS:
            dt = torch.int64 if k in ("size", "degsum", "ein", "eout") else torch.float64
            pc_t[k] = torch.empty(num_labels, dtype=dt, device=dev)
        pc = PerCommunity(*[pc_t[k].data_ptr() for k in PER_COMMUNITY_FIELDS])
    pt = None
    pairs = None
    if pairs_capacity > 0:
        pairs = (torch.empty(pairs_capacity, dtype=torch.int32, device=dev),
                 torch.empty(pairs_capacity, dtype=torch.int32, device=dev),
                 torch.empty(pairs_capacity, dtype=torch.int64, device=dev))
        pt = PairTable(pairs[0].data_ptr(), pairs[1].data_ptr(), pairs[2].data_ptr(), pairs_capacity)
    if noalloc:
        st, res = cq_score_partition_noalloc(ctx.handle, graph.handle, labels.data_ptr(), num_labels, pc, pt, allow=allow)
    else:
        st, res = cq_score_partition(ctx.handle, graph.handle, labels.data_ptr(), num_labels, ws.data_ptr(),
                                     ws.numel(), pc, pt, allow=allow)
    r = as_dict(res)
    r["status"] = st
    graph.last_staging = res.staging  # CQ_STAGING_*: how this call staged the neighbour labels
    pair_tensor = None
    if pairs is not None:
        k = min(r["num_pairs"], pairs_capacity)
        pair_tensor = torch.stack([pairs[0][:k].to(torch.int64), pairs[1][:k].to(torch.int64), pairs[2][:k]], dim=1)
    return r, pc_t, pair_tensor


def compare_partitions(ctx: Context, labels_a, num_labels_a: int, labels_b, num_labels_b: int, *,
                       cells_capacity: int = 0, workspace=None, allow=(CQ_OK,)):
    """Compare ground truth (labels_a) with a detected partition (labels_b); returns (dict, cells | None)."""
    torch = _torch()
    la = _dev_i32(labels_a, "labels_a")
    lb = _dev_i32(labels_b, "labels_b")
    n = la.numel()
    if lb.numel() != n:
        raise ValueError("label arrays differ in length")
    need = cq_compare_workspace_size(n, num_labels_a, num_labels_b)
    ws = workspace if workspace is not None else ctx.workspace(need)
    ct = None
    cells = None
    if cells_capacity > 0:
        cells = (torch.empty(cells_capacity, dtype=torch.int32, device=la.device),
                 torch.empty(cells_capacity, dtype=torch.int32, device=la.device),
                 torch.empty(cells_capacity, dtype=torch.int64, device=la.device))
        ct = CellTable(cells[0].data_ptr(), cells[1].data_ptr(), cells[2].data_ptr(), cells_capacity)
    st, res = cq_compare_partitions(ctx.handle, n, la.data_ptr(), num_labels_a, lb.data_ptr(), num_labels_b,
                                    ws.data_ptr(), ws.numel(), ct, allow=allow)
    r = as_dict(res)
    r["status"] = st
    cell_tensor = None
    if cells is not None:
        k = min(r["nnz"], cells_capacity)
        cell_tensor = torch.stack([cells[0][:k].to(torch.int64), cells[1][:k].to(torch.int64), cells[2][:k]], dim=1)
    return r, cell_tensor


class Batch:
    """Many (graph, labels, num_labels) scoring tasks run as one batch (one HIP graph replay)."""

    def __init__(self, ctx: Context, tasks, *, autotune: bool = True, use_graph: bool = True):
        torch = _torch()
        self.ctx = ctx
        self.tasks = [(g, _dev_i32(lab, "labels"), int(L)) for g, lab, L in tasks]
        for g, lab, _ in self.tasks:
            if lab.numel() != g.n:
                raise ValueError("labels must have one entry per node of their graph")
        flags = (CQ_BATCH_AUTOTUNE if autotune else 0) | (0 if use_graph else CQ_BATCH_NO_GRAPH)
        self.handle = cq_batch_plan_create(ctx.handle, [(g.handle, lab.data_ptr(), L) for g, lab, L in self.tasks], flags)
        nbytes = cq_batch_workspace_size(self.handle)
        self.ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=f"cuda:{ctx.device}")
        self.results = torch.empty(len(self.tasks) * ctypes.sizeof(ScoreResult), dtype=torch.uint8,
                                   device=f"cuda:{ctx.device}")
        cq_batch_bind(ctx.handle, self.handle, self.ws.data_ptr(), self.ws.numel(), self.results.data_ptr())
        self.tuning = cq_batch_get_tuning(self.handle)

    def run(self) -> None:
        cq_batch_run(self.ctx.handle, self.handle)

    def run_sync(self, allow=(CQ_OK,)) -> list[dict]:
        st, res = cq_batch_run_sync(self.ctx.handle, self.handle, len(self.tasks), allow=allow)
        out = [as_dict(r) for r in res]
        for r in out:
            r["status"] = st
        return out

    def close(self):
        if self.handle:
            cq_batch_plan_destroy(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server over resident graphs (labels in host memory)."""

    def __init__(self, ctx: Context, *, num_slots: int = 4, max_batch: int = 16, memory_budget: int = 8 << 30,
                 small_nnz: int = 4_000_000):
        self.ctx = ctx
        self.handle = cq_server_create(ctx.handle, num_slots, max_batch, memory_budget, small_nnz)
        self._keep = {}

    def submit_score(self, graph: Graph, h_labels, num_labels: int) -> int:
        """h_labels: host int32 tensor (pinned is fastest); kept alive until waited for."""
        torch = _torch()
        if not isinstance(h_labels, torch.Tensor) or h_labels.device.type != "cpu" or h_labels.dtype != torch.int32 \
                or not h_labels.is_contiguous() or h_labels.numel() != graph.n:
            raise TypeError("h_labels must be a contiguous int32 CPU tensor with one entry per node")
        t = cq_server_submit_score(self.ctx.handle, self.handle, graph.handle, h_labels.data_ptr(), num_labels)
        self._keep[t] = (h_labels,)
        return t

    def submit_compare(self, h_a, num_labels_a: int, h_b, num_labels_b: int) -> int:
        t = cq_server_submit_compare(self.ctx.handle, self.handle, h_a.numel(), h_a.data_ptr(), num_labels_a,
                                     h_b.data_ptr(), num_labels_b)
        self._keep[t] = (h_a, h_b)
        return t

    def wait(self, ticket: int, timeout_ms: float = -1.0):
        st, rs, sres, cres, lat = cq_server_wait(self.ctx.handle, self.handle, ticket, timeout_ms)
        if st == CQ_E_BUSY:
            return None
        self._keep.pop(ticket, None)
        return {"status": rs, "score": sres, "compare": cres, "latency_ms": lat}

    def stats(self) -> dict:
        return cq_server_get_stats(self.handle)

    def reset_stats(self) -> None:
        cq_server_reset_stats(self.handle)

    def close(self):
        if self.handle:
            cq_server_destroy(self.handle)
            self.handle = 0
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
