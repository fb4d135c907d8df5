"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
function include/cq.h declares, reports status names, sizes workspaces, and rejects
bad arguments before touching a device."""
import ctypes
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cq():
    from paper_1507_05492_amd import cq as mod

    return mod


def test_exports_every_declared_function(cq):
    names = cq.header_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(cq.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", cq.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    assert set(names) <= exported


def test_library_has_gfx950_code(cq):
    # the offload bundle of the library built here names its target
    assert b"gfx950" in open(cq.LIB_PATH, "rb").read()


def test_status_strings(cq):
    assert cq.cq_status_string(cq.CQ_OK) == "CQ_OK"
    assert cq.cq_status_string(cq.CQ_E_LABEL_RANGE) == "CQ_E_LABEL_RANGE"
    assert cq.cq_status_string(cq.CQ_E_CAPACITY) == "CQ_E_CAPACITY"
    assert cq.cq_status_string(-99) == "CQ_E_UNKNOWN"


def test_compare_workspace_size(cq):
    assert cq.cq_compare_workspace_size(1, 1, 1) == 0          # n < 2
    assert cq.cq_compare_workspace_size(10, 0, 1) == 0
    s1 = cq.cq_compare_workspace_size(100_000, 399, 399)
    s2 = cq.cq_compare_workspace_size(200_000, 399, 399)
    s3 = cq.cq_compare_workspace_size(100_000, 100_000, 399)   # global-atomic layout
    assert 0 < s1 < s2 and s3 > s1
    assert s1 % 256 == 0
    # at least one 32-bit word per node (the band words, or the staged labels and per-node offsets)
    assert s1 >= 4 * 100_000


def test_null_handles(cq):
    lib = cq._lib
    assert lib.cq_score_workspace_size(None, 5) == 0
    assert lib.cq_context_set_stream(None, None) == cq.CQ_E_INVALID_ARG
    assert lib.cq_graph_get_stats(None, None) == cq.CQ_E_INVALID_ARG
    assert lib.cq_score_partition(None, None, None, 1, None, 0, None, None, None) == cq.CQ_E_INVALID_ARG
    assert lib.cq_compare_partitions(None, 10, None, 1, None, 1, None, 0, None, None) == cq.CQ_E_INVALID_ARG
    out = ctypes.c_void_p()
    assert lib.cq_context_create(0, None, None) == cq.CQ_E_INVALID_ARG
    lib.cq_context_destroy(None)
    lib.cq_graph_release(None)
    assert cq.cq_context_last_error(None) == "null context"


def test_context_without_gpu_fails_cleanly(cq):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(cq.CQError) as e:
        cq.cq_context_create(0, None)
    assert e.value.status == cq.CQ_E_DEVICE


def test_header_compiles_as_c():
    src = os.path.join(ROOT, "include", "cq.h")
    res = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-fsyntax-only", "-x", "c", src], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
