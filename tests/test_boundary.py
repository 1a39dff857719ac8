"""CPU tests of the C ABI boundary: the library loads, exports every symbol the
header declares, and rejects bad arguments before any HIP call (so these run
without a GPU)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bsps.h")


@pytest.fixture(scope="module")
def bsps():
    import paper_1408_6729_amd as m
    return m


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bsps_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol(bsps):
    names = _declared()
    assert "bsps_sort" in names and "bsps_sort_kv" in names and "bsps_sort_segmented" in names
    missing = [n for n in names if not hasattr(bsps.lib, n)]
    assert not missing, f"declared in bsps.h but not exported: {missing}"


def test_status_strings(bsps):
    assert bsps.status_string(0) == "ok"
    assert "workspace" in bsps.status_string(2)
    assert bsps.status_string(99) == "unknown status"


def _call(bsps, n, dtype, prm, ws=None, ws_bytes=0, keys=1):
    return bsps.lib.bsps_sort(ct.c_void_p(keys) if keys else None, n, dtype, ct.byref(prm), ws, ws_bytes, None,
                              None)


@pytest.mark.parametrize("case", [
    dict(n=-1, p=1, s=1), dict(n=10, p=0, s=1), dict(n=10, p=11, s=1), dict(n=10, p=2, s=0),
    dict(n=10, p=2, s=6, variant=1), dict(n=10, p=2, s=1, variant=7), dict(n=10, p=2, s=1, route=5),
    dict(n=10, p=2, s=1, bucketing=3), dict(n=10, p=2, s=1, leaves=-1), dict(n=10, p=2, s=1, dtype=9),
    dict(n=10, p=2, s=6, variant=2), dict(n=10, p=2, s=1, variant=2, route=1), dict(n=10, p=2, s=1, variant=3),
    dict(n=10, p=2, s=1, local_sort=3),
    # iterative rounds: p must be k^m (k >= 2), DET, fused route, splitter search, tagged, m <= 10
    dict(n=100, p=12, s=1, rounds=2), dict(n=100, p=8, s=1, rounds=2), dict(n=100, p=16, s=1, rounds=2, variant=1),
    dict(n=100, p=16, s=1, rounds=2, route=1), dict(n=100, p=16, s=1, rounds=2, bucketing=1),
    dict(n=100, p=16, s=1, rounds=2, untagged=True), dict(n=5000, p=1024, s=1, rounds=11),
    dict(n=100, p=16, s=1, rounds=-1),
])
def test_invalid_arguments_rejected_on_host(bsps, case):
    case = dict(case)
    dtype = case.pop("dtype", 0)
    n = case.pop("n")
    prm = bsps.make_params(case.pop("p"), case.pop("s"), **case)
    assert bsps.workspace_bytes(n, dtype, False, prm) == 0
    assert _call(bsps, n, dtype, prm) == bsps.EINVAL


def test_untagged_flag_is_boolean(bsps):
    prm = bsps.make_params(2, 2)
    prm.untagged = 2
    assert bsps.workspace_bytes(10, 0, False, prm) == 0
    assert _call(bsps, 10, 0, prm) == bsps.EINVAL


def test_iterative_dry_run(bsps):
    """Every launch of the iterative rounds checked on the host for several
    shapes (k = 2 .. 32, m = 2 .. 10), dtypes and payloads."""
    for n, p, s, m, dt, kv in [(1 << 20, 16, 8, 2, 0, False), (1 << 20, 64, 4, 3, 1, True), (1000, 16, 2, 4, 2, False),
                               (100_000, 1024, 4, 2, 0, True), (1 << 26, 1024, 16, 2, 0, False),
                               (1 << 28, 256, 64, 2, 1, True), (70, 64, 1, 3, 0, False), (5000, 1024, 1, 10, 0, True)]:
        k, rep = bsps.check_sort(n, dt, kv, bsps.make_params(p, s, rounds=m))
        assert k == 0, rep
    # rounds = 1 and p = 1 take the one-round path
    assert bsps.workspace_bytes(1000, 0, False, bsps.make_params(12, 2, rounds=1)) > 0
    assert bsps.workspace_bytes(1000, 0, False, bsps.make_params(1, 2, rounds=3)) > 0


def test_reserved_fields_must_be_zero(bsps):
    prm = bsps.make_params(2, 2)
    prm.reserved[3] = 1
    assert _call(bsps, 100, 0, prm) == bsps.EINVAL


def test_limits(bsps):
    assert _call(bsps, 5000, 0, bsps.make_params(1025, 1)) == bsps.EUNSUPPORTED
    assert _call(bsps, 1 << 32, 0, bsps.make_params(4, 1)) == bsps.EUNSUPPORTED
    # a block of more than 1024 tiles of 16K keys: too many runs for the merge of
    # its tiles; AUTO (and Sort_Ran_BSP, which merges no tiles) take it, by LSD passes
    big = (1 << 24) * 2 + 10
    assert _call(bsps, big, 0, bsps.make_params(1, 1, local_sort=bsps.LOCAL_MERGE)) == bsps.EUNSUPPORTED
    assert bsps.workspace_bytes(big, 0, False, bsps.make_params(1, 1)) > 0
    assert bsps.workspace_bytes(big, 0, False, bsps.make_params(2, 1, variant=bsps.RAN_SR)) > 0
    for prm in (bsps.make_params(1, 1), bsps.make_params(8, 64), bsps.make_params(8, 64, variant=bsps.RAN_SR),
                bsps.make_params(4, 16, rounds=2)):
        k, rep = bsps.check_sort(big, 0, True, prm)
        assert k == 0, rep


def test_workspace_checked_before_device(bsps):
    prm = bsps.make_params(16, 8)
    need = bsps.workspace_bytes(1 << 20, 0, False, prm)
    assert need > 2 * 4 * (1 << 20)
    assert _call(bsps, 1 << 20, 0, prm, ws=None, ws_bytes=0) == bsps.EWORKSPACE
    assert _call(bsps, 1 << 20, 0, prm, ws=ct.c_void_p(4096), ws_bytes=need - 1) == bsps.EWORKSPACE
    assert _call(bsps, 1 << 20, 0, prm, ws=ct.c_void_p(4096 + 8), ws_bytes=need) == bsps.EWORKSPACE  # unaligned
    kv = bsps.workspace_bytes(1 << 20, 0, True, prm)
    assert kv > need
    assert bsps.workspace_bytes(1 << 20, 1, False, prm) > need  # int64 keys


def test_trivial_sizes_are_noops(bsps):
    assert _call(bsps, 0, 0, bsps.make_params(1, 1), keys=0) == bsps.OK
    assert _call(bsps, 1, 2, bsps.make_params(1, 3)) == bsps.OK


def test_null_keys_rejected(bsps):
    assert _call(bsps, 100, 0, bsps.make_params(2, 2), keys=0) == bsps.EINVAL


def test_segmented_validation(bsps):
    import numpy as np
    ok = np.array([0, 10, 10, 25], dtype=np.int64)
    assert bsps.segmented_workspace_bytes(ok, 0, False) > 0
    assert bsps.segmented_workspace_bytes(np.array([1, 10], dtype=np.int64), 0, False) == 0   # must start at 0
    assert bsps.segmented_workspace_bytes(np.array([0, 10, 5], dtype=np.int64), 0, False) == 0  # decreasing
    assert bsps.segmented_workspace_bytes(ok, 7, False) == 0  # dtype
    assert bsps.segmented_workspace_bytes(ok, 0, False, tuning='{"classes": []}') == 0
    assert bsps.segmented_workspace_bytes(ok, 0, False, tuning='{"classes": [{"max_log2": 8, "block": 0, "s": 1}]}') == 0
    good = '{"classes": [{"max_log2": 8, "block": 64, "s": 2}, {"max_log2": 30, "block": 4096, "s": 8}]}'
    assert bsps.segmented_workspace_bytes(ok, 0, True, tuning=good) > bsps.segmented_workspace_bytes(ok, 0, False, tuning=good)
    assert "max_log2" in bsps.tuning_format() and "learned_above_log2" in bsps.tuning_format()
    lt = '{"learned_above_log2": %d, "classes": [{"max_log2": 30, "block": 4096, "s": 8}]}'
    assert bsps.segmented_workspace_bytes(ok, 0, False, tuning=lt % 16) > 0
    assert bsps.segmented_workspace_bytes(ok, 0, False, tuning=lt % 41) == 0
    # a segment that needs more than 1024 blocks of one tile
    big = np.array([0, 16384 * 1024 + 1], dtype=np.int64)
    assert bsps.segmented_workspace_bytes(big, 0, False) == 0


def test_stream_copy_checked_before_device(bsps):
    """The reference copy rejects misaligned pointers and sizes on the host."""
    f = bsps.lib.bsps_stream_copy
    assert f(ct.c_void_p(4096), ct.c_void_p(8192), 4096 + 8, None) == bsps.EINVAL  # size not a multiple of 16
    assert f(ct.c_void_p(4096 + 4), ct.c_void_p(8192), 4096, None) == bsps.EINVAL  # source misaligned
    assert f(ct.c_void_p(4096), ct.c_void_p(8192 + 8), 4096, None) == bsps.EINVAL  # destination misaligned
    assert f(None, ct.c_void_p(8192), 4096, None) == bsps.EINVAL
    assert f(ct.c_void_p(4096), ct.c_void_p(8192), 0, None) == bsps.OK  # nothing to copy, no device call


# ----------------------------------------------------------------- host dry runs of the plans

@pytest.mark.parametrize("dtype", [0, 1, 2])
@pytest.mark.parametrize("kv", [False, True])
@pytest.mark.parametrize("route,bucketing", [(0, 0), (1, 0), (1, 1)])
@pytest.mark.parametrize("local_sort", [0, 1, 2])
def test_dry_run_sort_plans(bsps, dtype, kv, route, bucketing, local_sort):
    """Every kernel launch of the sort, planned with fake buffers and checked
    on the host: pointers inside the caller's buffers or the workspace, tables
    inside at their full extent, grids non-empty. Sizes from the workloads
    (2^28 keys, p up to 1024) down to ragged small ones, both variants."""
    cases = [(1 << 28, 256, 64), (1 << 28, 1024, 64), (1 << 20, 16, 8), (5_000_003, 61, 8), (123457, 7, 3),
             (2 * 16384 + 1, 2, 8), (1000, 1000, 1), (3, 1, 1)]
    for n, p, s in cases:
        for variant in (0, 1):
            if variant == 1 and s * p - 1 > n:
                continue
            prm = bsps.make_params(p, s, variant, 1, bucketing, route, 0, 0, local_sort)
            k, rep = bsps.check_sort(n, dtype, kv, prm)
            assert k == 0, (n, p, s, variant, rep)


@pytest.mark.parametrize("dtype", [0, 1, 2])
@pytest.mark.parametrize("kv", [False, True])
def test_dry_run_segmented_plans(bsps, dtype, kv):
    """The segmented planner: the 4096-segment batch, edge segments and the
    learned path on and off, all launches and host tables checked."""
    import json
    import numpy as np
    import workloads as W
    sizes = W.segment_sizes(4096, 8, 20)
    batches = [sizes, np.array([0, 1, 2, 16383, 16384, 16385, 70000, 0, 3 << 16]), np.array([5])]
    for lg in (16, 40):
        tj = json.dumps({"learned_above_log2": lg, "classes": [{"max_log2": 14, "block": 16384, "s": 1},
                                                               {"max_log2": 20, "block": 4096, "s": 16},
                                                               {"max_log2": 40, "block": 16384, "s": 8}]})
        for sz in batches:
            off = np.zeros(len(sz) + 1, dtype=np.int64)
            np.cumsum(sz, out=off[1:])
            k, rep = bsps.check_segmented(off, dtype, kv, tj)
            assert k == 0, rep


def test_dry_run_rejects_like_the_call(bsps):
    prm = bsps.make_params(0, 1)
    assert bsps.check_sort(10, 0, False, prm)[0] == -bsps.EINVAL
    assert bsps.check_segmented([0, 5, 3], 0, False)[0] == -bsps.EINVAL


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "1"], {"WORLD_SIZE": "2"})])
def test_bench_refuses_more_than_one_gpu(argv, env):
    """The benchmark measures one GPU: asked for more (by flag or by a
    launcher's WORLD_SIZE) it exits with status 2 and says so, before any
    GPU work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    e = dict(os.environ)
    e.pop("WORLD_SIZE", None)
    e.update(env)
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), *argv], capture_output=True, text=True,
                       timeout=120, env=e, cwd=root)
    assert r.returncode == 2
    assert "single GPU" in r.stderr
    assert r.stdout == ""


def test_import_fails_loudly_without_the_library(tmp_path):
    """The product path has no CPU fallback: with the HIP library missing,
    importing the package raises and names the build step."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    e = dict(os.environ)
    e["BSPS_LIB"] = str(tmp_path / "libbsps_missing.so")
    r = subprocess.run([sys.executable, "-c", "import paper_1408_6729_amd"], capture_output=True, text=True,
                       timeout=120, env=e, cwd=root)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "no CPU fallback" in r.stderr
