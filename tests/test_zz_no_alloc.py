"""GPU test of the allocation-free entry point bsps_sort_noalloc.

Two calls in a row through the C ABI, the second with a smaller input of
another dtype and variant, each compared bit for bit with the existing entry
point (bsps_sort / bsps_sort_kv with a caller workspace) on the same input.
Since both calls share the GPU's scratch array, the second also shows that the
first call's leftovers do not affect a later sort. A size whose workspace
exceeds the scratch is rejected on the host.
"""
import ctypes as ct

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    import paper_1408_6729_amd as bsps  # noqa: F401  (fails loudly without the library)
    return torch.device("cuda:0")


def _both(dev, keys, p, s, variant, kv):
    import torch
    import paper_1408_6729_amd as bsps
    vals = np.arange(keys.size, dtype=np.uint32).view(np.int32) if kv else None
    a = torch.from_numpy(keys.copy()).to(dev)
    b = a.clone()
    va = None if vals is None else torch.from_numpy(vals.copy()).to(dev)
    vb = None if va is None else va.clone()
    dt = {np.dtype(np.int32): bsps.I32, np.dtype(np.int64): bsps.I64, np.dtype(np.float32): bsps.F32}[keys.dtype]
    prm = bsps.make_params(p, s, variant)
    assert bsps.workspace_bytes(keys.size, dt, kv, prm) <= bsps.NOALLOC_SCRATCH_BYTES
    bsps.sort_noalloc_(a, p, s, variant, values=va)
    bsps.sort_(b, p, s, variant, values=vb)
    torch.cuda.synchronize()
    ka, kb = a.cpu().numpy(), b.cpu().numpy()
    assert np.array_equal(ka.view(np.uint8), kb.view(np.uint8)), "keys differ from bsps_sort"
    if kv:
        assert np.array_equal(va.cpu().numpy(), vb.cpu().numpy()), "payloads differ from bsps_sort_kv"
    # and the result is the stable sort
    ref = np.argsort(keys if keys.dtype != np.float32 else _f32_order(keys), kind="stable")
    assert np.array_equal(ka.view(np.uint8), keys[ref].view(np.uint8))
    if kv:
        assert np.array_equal(va.cpu().numpy().view(np.uint32), ref.astype(np.uint32))


def _f32_order(f):
    b = f.view(np.uint32).astype(np.uint64)
    return np.where(b >= (1 << 31), 0xFFFFFFFF - b, b + (1 << 31))


def test_two_calls_second_smaller(dev):
    print("noalloc: call 1, 2^21+12345 int32 key-value, p=64, s=16, DET", flush=True)
    n1 = (1 << 21) + 12345
    _both(dev, W.int32_keys(n1, 64, "uniform"), 64, 16, 0, kv=True)
    print("noalloc: call 2, 100003 int64 keys, p=16, s=8, RAN", flush=True)
    _both(dev, W.random_keys(100003, "int64", seed=5, distinct=5000), 16, 8, 1, kv=False)
    print("noalloc: call 3, 70001 float32 key-value, p=8, s=4, DET", flush=True)
    _both(dev, W.random_keys(70001, "float32", seed=6), 8, 4, 0, kv=True)


def test_too_large_rejected_on_host(dev):
    import paper_1408_6729_amd as bsps
    n = 1 << 26
    prm = bsps.make_params(256, 64)
    assert bsps.workspace_bytes(n, bsps.I32, False, prm) > bsps.NOALLOC_SCRATCH_BYTES
    # rejected before any device access: the keys pointer is never touched
    code = bsps.lib.bsps_sort_noalloc(ct.c_void_p(16), None, n, bsps.I32, ct.byref(prm), None)
    assert code == bsps.EUNSUPPORTED
