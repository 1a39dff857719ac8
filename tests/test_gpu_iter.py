"""GPU parity of the iterative Sort_Det_BSP (Section 5.1: m rounds of k-way
partitioning and merging, p = k^m) against the CPU oracle, element by element.

Every case checks, bit for bit: the sorted keys (and payloads), every round's
splitters (keys and tags) and count matrix (processor x bucket), the sorted
sample of round 1 and the final bucket sizes. Sizes span several tiles and
ragged tails, shapes span k = 2 .. 32 and m = 2 .. 10.
"""
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


def _bits(a):
    return a.view(np.uint32) if a.dtype == np.float32 else a


def _check_iter(ora, dev, keys, p, s, m, kv=False, chunk_cap=0, local_sort=0):
    import torch
    import paper_1408_6729_amd as bsps
    print(f"iterative n={keys.size} dtype={keys.dtype} p={p} s={s} m={m} kv={kv} cap={chunk_cap} "
          f"local={local_sort}", flush=True)
    vals = np.arange(keys.size, dtype=np.uint32) if kv else None
    ref = ora.sort_iter(keys, p, s, m, vals)
    t = torch.from_numpy(np.ascontiguousarray(keys)).to(dev)
    v = None if vals is None else torch.from_numpy(vals.view(np.int32)).to(dev)
    st = bsps.sort_(t, p, s, bsps.DET, values=v, chunk_cap=chunk_cap, stats=True, local_sort=local_sort, rounds=m)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(t.cpu().numpy()), _bits(ref["keys"])), "sorted keys differ"
    if kv:
        assert np.array_equal(v.cpu().numpy().view(np.uint32), ref["values"]), "payload order differs"
    if p > 1:
        assert np.array_equal(st["splitter_pos"], ref["spl_pos"]), "splitter tags differ"
        assert np.array_equal(ora.order_keys(st["splitter_keys"]), ref["spl_key"]), "splitter keys differ"
        assert np.array_equal(st["count_matrix"], ref["C"]), "count matrices differ"
        # round 1's sample is the regular sample of Sort_Det_BSP
        one = ora.sort(keys, p, s, ora.DET)
        assert np.array_equal(st["sample_pos"], one["sample_pos"]), "round-1 sample differs"
        # the final buckets: the last round's sub-buckets
        last = ref["C"][-1]
        k = ref["k"]
        want = np.array([last[(i // k) * k:(i // k + 1) * k, i % k].sum() for i in range(p)])
        assert np.array_equal(st["bucket_sizes"], want), "final bucket sizes differ"
    return st


@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
@pytest.mark.parametrize("p,m", [(16, 2), (64, 3), (27, 3), (256, 4)])
def test_iter_against_oracle(ora, dev, dtype, p, m):
    keys = W.random_keys(155_494, dtype, seed=p + m)
    _check_iter(ora, dev, keys, p, 8, m, kv=dtype != "float32")


@pytest.mark.parametrize("dist", W.DISTRIBUTIONS)
def test_iter_distributions(ora, dev, dist):
    """The seven synthetic distributions, 2^21 int32 keys, p = 64 in two
    rounds of 8 buckets, s = 32."""
    keys = W.int32_keys(1 << 21, 64, dist)
    _check_iter(ora, dev, keys, 64, 32, 2)


@pytest.mark.parametrize("p,m,s", [(1024, 2, 4), (1024, 5, 2), (1024, 10, 1), (256, 2, 64), (4, 2, 1)])
def test_iter_shapes(ora, dev, p, m, s):
    keys = W.random_keys((1 << 20) + 12_345, "int32", seed=m, distinct=5000)
    _check_iter(ora, dev, keys, p, s, m, kv=True)


@pytest.mark.parametrize("kind", ["zero", "dup3", "sorted", "reversed"])
def test_iter_duplicates_and_order(ora, dev, kind):
    n = 300_001
    if kind == "zero":
        keys = np.zeros(n, dtype=np.int64)
    elif kind == "dup3":
        keys = W.random_keys(n, "int64", seed=3, distinct=3)
    elif kind == "sorted":
        keys = np.sort(W.random_keys(n, "int32", seed=4))
    else:
        keys = np.sort(W.random_keys(n, "int32", seed=5))[::-1].copy()
    _check_iter(ora, dev, keys, 64, 4, 2, kv=True)


def test_iter_oversize_chunks(ora, dev):
    """A small merge chunk cap sends chunks of the rounds' merges through the
    global-memory path (the caller's buffer is its scratch in round 1, the
    other work array in the last round)."""
    # every block holds the same 6000 keys: the runs a share merges have their
    # samples at the same keys, so a chunk between two consecutive boundaries
    # spans about one sample gap of every run, well above the cap
    rng = np.random.default_rng(9)
    keys = np.concatenate([rng.permutation(6000) for _ in range(64)]).astype(np.int32)
    st = _check_iter(ora, dev, keys, 64, 8, 2, kv=True, chunk_cap=128)
    assert st["oversize_bucket"] > 0


def test_iter_lsd_local_sort(ora, dev):
    keys = W.random_keys(500_000, "int64", seed=10)
    _check_iter(ora, dev, keys, 64, 8, 3, kv=True, local_sort=2)


def test_iter_tiny(ora, dev):
    """n = p (one key per processor) and a few keys more."""
    for n in (64, 65, 100, 127):
        keys = W.random_keys(n, "int32", seed=n, distinct=4)
        _check_iter(ora, dev, keys, 64, 3, 2)
