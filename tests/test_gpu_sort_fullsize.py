"""Parity at the full workload sizes, in the launch configurations the
benchmark times.

Every full-size workload is compared with the oracle itself, element by
element: the output (and payload), the sample and splitter tags and the count
matrix, for both variants. The oracle runs with its per-processor steps on
the host cores (oracle.sort(threads=...), byte-identical to the single-thread
oracle). The invariants that fix a stable sort at any size (ordered, a
permutation, equal keys in increasing original position) are checked on the
GPU as well, together with the paper's DET bucket-size bound (Lemma balance)
and the all-equal closed form.
"""
import functools
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _threads():
    """Host threads of the oracle (the CPU share of one GPU)."""
    import oracle
    return oracle.default_threads()


@functools.lru_cache(maxsize=1)
def _c3_input():
    return W.zipf_int64_kv(1 << 28)


@functools.lru_cache(maxsize=1)
def _c4_input():
    return W.lognormal_f32(1 << 28)


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    import paper_1408_6729_amd  # noqa: F401
    return torch.device("cuda:0")


def _to_dev(a, dev):
    """Host array -> device tensor through a pinned (hipHostMalloc) buffer:
    large transfers never hand a pageable range to the runtime."""
    import torch
    h = torch.from_numpy(np.ascontiguousarray(a))
    pin = torch.empty(h.shape, dtype=h.dtype, pin_memory=True)
    pin.copy_(h)
    return pin.to(dev)


def _to_host(t):
    """Device tensor -> numpy array through a pinned buffer."""
    import torch
    pin = torch.empty(t.shape, dtype=t.dtype, pin_memory=True)
    pin.copy_(t)
    return pin.numpy()


def _order_np(a):
    """Order-preserving unsigned image (numpy, float32 by its bits)."""
    if a.dtype == np.float32:
        b = a.view(np.uint32)
        return np.where(b >> 31, ~b, b | np.uint32(0x80000000))
    return a


def _lemma_bound(n, p, s):
    m = -(-n // p)
    x = -(-m // s)
    return (s + p - 1) * x


@pytest.mark.timeout(600)
def test_headline_det_2e28_against_oracle(ora, dev):
    """2^28 uniform int32 keys, p = 256, s = 64, DET: keys, sample tags,
    splitter tags and count matrix equal the oracle's; buckets obey Lemma
    balance."""
    import torch
    import paper_1408_6729_amd as bsps
    n, p, s = 1 << 28, 256, 64
    keys = W.int32_keys(n, p, "uniform")
    t = _to_dev(keys, dev)
    st = bsps.sort_(t, p, s, bsps.DET, stats=True)
    out = _to_host(t)
    del t
    ref = ora.sort(keys, p, s, ora.DET, threads=_threads())
    assert np.array_equal(out, ref["keys"])
    assert np.array_equal(st["sample_pos"], ref["sample_pos"])
    assert np.array_equal(st["splitter_pos"], ref["spl_pos"])
    assert np.array_equal(st["count_matrix"], ref["C"])
    assert st["bucket_sizes"].max() <= _lemma_bound(n, p, s)


@pytest.mark.timeout(300)
def test_headline_ran_2e28(ora, dev):
    """The same input, RAN (seed 1): output, sample tags (the oracle's keyed
    permutation positions), splitter tags and count matrix equal the
    oracle's."""
    import paper_1408_6729_amd as bsps
    n, p, s = 1 << 28, 256, 64
    keys = W.int32_keys(n, p, "uniform")
    t = _to_dev(keys, dev)
    st = bsps.sort_(t, p, s, bsps.RAN, seed=1, stats=True)
    out = _to_host(t)
    del t
    ref = ora.sort(keys, p, s, ora.RAN, 1, threads=_threads())
    assert np.array_equal(out, ref["keys"])
    assert np.array_equal(st["sample_pos"], ref["sample_pos"])
    assert np.array_equal(st["splitter_pos"], ref["spl_pos"])
    assert np.array_equal(st["count_matrix"], ref["C"])


@pytest.mark.timeout(300)
@pytest.mark.parametrize("dist", W.DISTRIBUTIONS)
def test_c2_distributions_full(ora, dev, dist):
    """2^26 int32 keys, p = 128, s = 32, both variants, each of the seven
    distributions: output, splitter tags and count matrix equal the oracle's;
    DET buckets obey Lemma balance; all-equal keys give the diagonal count
    matrix."""
    import paper_1408_6729_amd as bsps
    n, p, s = 1 << 26, 128, 32
    keys = W.int32_keys(n, p, dist)
    base = _to_dev(keys, dev)
    for variant in (bsps.DET, bsps.RAN):
        t = base.clone()
        st = bsps.sort_(t, p, s, variant, seed=1, stats=True)
        ref = ora.sort(keys, p, s, variant, 1, threads=_threads())
        assert np.array_equal(_to_host(t), ref["keys"]), (dist, variant)
        assert np.array_equal(st["splitter_pos"], ref["spl_pos"]), (dist, variant)
        assert np.array_equal(st["count_matrix"], ref["C"]), (dist, variant)
        C = st["count_matrix"]
        assert C.sum() == n
        if variant == bsps.DET:
            assert st["bucket_sizes"].max() <= _lemma_bound(n, p, s)
            if dist == "zero":
                m = [((k + 1) * n) // p - (k * n) // p for k in range(p)]
                assert np.array_equal(C, np.diag(m))


@pytest.mark.timeout(300)
@pytest.mark.parametrize("variant", [0, 1])
def test_int64_kv_duplicates_2e28(ora, dev, variant):
    """2^28 int64 Zipf keys + 25% equal block, uint32 payload = original
    index, p = 256, s = 64, DET and RAN: keys, payloads, sample and splitter
    tags and count matrix equal the oracle's; on the GPU also: ordered,
    keys[payload] = output keys, and payload strictly increasing inside every
    run of equal keys (the paper's tie rule)."""
    import torch
    import paper_1408_6729_amd as bsps
    n, p, s = 1 << 28, 256, 64
    k, v = _c3_input()
    base = _to_dev(k, dev)
    t = base.clone()
    vt = _to_dev(v.view(np.int32), dev)
    st = bsps.sort_(t, p, s, variant, seed=1, values=vt, stats=True)
    torch.cuda.synchronize()
    pay = vt.to(torch.int64) & 0xFFFFFFFF
    assert bool(torch.all(t[1:] >= t[:-1]))
    assert bool(torch.equal(base[pay], t))
    tie = t[1:] == t[:-1]
    assert bool(torch.all(pay[1:][tie] > pay[:-1][tie]))
    assert int(tie.sum()) > n // 4  # the duplicate stress is real
    del tie, pay, base
    out, outv = _to_host(t), _to_host(vt).view(np.uint32)
    del t, vt
    ref = ora.sort(k, p, s, variant, 1, v, threads=_threads())
    assert np.array_equal(out, ref["keys"])
    assert np.array_equal(outv, ref["values"])
    assert np.array_equal(st["sample_pos"], ref["sample_pos"])
    assert np.array_equal(st["splitter_pos"], ref["spl_pos"])
    assert np.array_equal(st["count_matrix"], ref["C"])


@pytest.mark.timeout(300)
@pytest.mark.parametrize("variant", [0, 1])
def test_learned_2e28_float32(ora, dev, variant):
    """2^28 float32 lognormal-mixture keys with -0.0/+0.0, p = 1024, s = 64,
    4096 leaves, DET and RAN: the learned route's output, splitter tags and
    count matrix equal the oracle's; for DET the splitter and fused routes give
    the same output and count matrix; the model predicts most keys exactly."""
    import torch
    import paper_1408_6729_amd as bsps
    n, p, s, L = 1 << 28, 1024, 64, 4096
    keys = _c4_input()
    base = _to_dev(keys, dev)
    routes = ((bsps.LEARNED, bsps.ROUTE_SCATTER),)
    if variant == bsps.DET:
        routes += ((bsps.SPLITTER, bsps.ROUTE_SCATTER), (bsps.SPLITTER, bsps.ROUTE_FUSED))
    outs, cms = [], []
    for bucketing, route in routes:
        t = base.clone()
        st = bsps.sort_(t, p, s, variant, seed=1, bucketing=bucketing, route=route, leaves=L, stats=True)
        if bucketing == bsps.LEARNED:
            learned = st
        outs.append(_to_host(t.view(torch.int32)))
        cms.append(st["count_matrix"])
        del t
    for o, c in zip(outs[1:], cms[1:]):
        assert np.array_equal(outs[0], o) and np.array_equal(cms[0], c)
    del base
    ref = ora.sort(keys, p, s, variant, 1, threads=_threads())
    assert np.array_equal(outs[0], ref["keys"].view(np.int32))
    assert np.array_equal(learned["splitter_pos"], ref["spl_pos"])
    assert np.array_equal(learned["sample_pos"], ref["sample_pos"])
    assert np.array_equal(cms[0], ref["C"])
    assert learned["mispredict_rate"] < 0.25, learned["mispredict_rate"]


@pytest.mark.timeout(300)
def test_segmented_4096_full(dev):
    """4096 int32 segments, log-uniform sizes in [2^8, 2^20] (about 5e8
    keys), one graph launch: every segment equals its sorted input."""
    import torch
    import paper_1408_6729_amd as bsps
    sizes = W.segment_sizes(4096, 8, 20)
    keys, offs = W.segmented_int32(sizes)
    t = _to_dev(keys, dev)
    st = bsps.sort_segmented_(t, offs, stats=True)
    assert st["graph"]
    out = _to_host(t)
    for i in range(len(sizes)):
        a, b = int(offs[i]), int(offs[i + 1])
        assert np.array_equal(out[a:b], np.sort(keys[a:b])), f"segment {i} of size {b - a}"


@pytest.mark.timeout(300)
def test_sr_full(ora, dev):
    """Sort_Ran_BSP at the mid size (2^26 int32 uniform, p = 128, s = 32) against
    the oracle (output, splitter tags, count matrix), and at the headline size
    (2^28, p = 256, s = 64) against the sorted input with the splitters' sample
    drawn from the oracle's keyed permutation."""
    import paper_1408_6729_amd as bsps
    n, p, s = 1 << 26, 128, 32
    keys = W.int32_keys(n, p, "uniform")
    t = _to_dev(keys, dev)
    st = bsps.sort_(t, p, s, bsps.RAN_SR, seed=1, stats=True)
    ref = ora.sort_sr(keys, p, s, 1)
    assert np.array_equal(_to_host(t), ref["keys"])
    assert np.array_equal(st["splitter_pos"], ref["spl_pos"])
    assert np.array_equal(st["count_matrix"], ref["C"])
    del t
    n, p, s = 1 << 28, 256, 64
    keys = W.int32_keys(n, p, "uniform")
    t = _to_dev(keys, dev)
    st = bsps.sort_(t, p, s, bsps.RAN_SR, seed=1, stats=True)
    assert np.array_equal(_to_host(t), np.sort(keys))
    pos = np.array([ora.feistel(1, n, j) for j in range(0, s * p - 1, 97)], dtype=np.int64)
    assert np.isin(pos, st["sample_pos"]).all()
    assert st["count_matrix"].sum() == n


@pytest.mark.timeout(600)
def test_iter_full(ora, dev):
    """The iterative Sort_Det_BSP in the configurations the benchmark times.
    At 2^24 int32 keys, p = 256, s = 64, m = 2 and 4 rounds: everything equals
    the oracle (output, every round's splitters and count matrix). At the
    headline size (2^28, p = 256, s = 64, m = 2): the output equals the
    threaded oracle's stable sort, round 1's splitters are the regular sample's
    records at ranks i*q*s/k (the sample of Sort_Det_BSP, from the oracle), and
    every round's count matrix partitions the shares."""
    import paper_1408_6729_amd as bsps
    n, p, s = 1 << 24, 256, 64
    keys = W.int32_keys(n, p, "uniform")
    for m in (2, 4):
        t = _to_dev(keys, dev)
        st = bsps.sort_(t, p, s, bsps.DET, stats=True, rounds=m)
        ref = ora.sort_iter(keys, p, s, m)
        assert np.array_equal(_to_host(t), ref["keys"]), m
        assert np.array_equal(st["splitter_pos"], ref["spl_pos"]), m
        assert np.array_equal(st["count_matrix"], ref["C"]), m
        del t
    n = 1 << 28
    keys = W.int32_keys(n, p, "uniform")
    t = _to_dev(keys, dev)
    st = bsps.sort_(t, p, s, bsps.DET, stats=True, rounds=2)
    out = _to_host(t)
    del t
    ref = ora.sort(keys, p, s, ora.DET, threads=_threads())
    assert np.array_equal(out, ref["keys"])
    k = 16
    stride = p * s // k
    assert np.array_equal(st["splitter_pos"][:k - 1], ref["sample_pos"][stride - 1:(k - 1) * stride:stride])
    C = st["count_matrix"]
    assert C.shape == (2, p, k) and (C.sum(axis=(1, 2)) == n).all()
    assert np.array_equal(C[0].sum(axis=1), [ora.block_start(n, p, j + 1) - ora.block_start(n, p, j)
                                            for j in range(p)])


@pytest.mark.timeout(400)
def test_large_blocks_beyond_merge_limit(ora, dev):
    """p = 8 on 2^27 + 12345 int32 keys: blocks of 2^24 + 1543 keys have more tiles
    than a merge group takes, so AUTO sorts them by LSD passes; Sort_Det_BSP and
    Sort_IRan_BSP against the threaded oracle (output, splitter tags, count
    matrix), and Sort_Ran_BSP (which merges no tiles) against the oracle's output."""
    import paper_1408_6729_amd as bsps
    n, p, s = (1 << 27) + 12345, 8, 64
    keys = W.random_keys(n, "int32", seed=27)
    for variant in (bsps.DET, bsps.RAN):
        t = _to_dev(keys, dev)
        st = bsps.sort_(t, p, s, variant, seed=3, stats=True)
        out = _to_host(t)
        del t
        ref = ora.sort(keys, p, s, variant, seed=3, threads=_threads())
        assert np.array_equal(out, ref["keys"]), variant
        assert np.array_equal(st["splitter_pos"], ref["spl_pos"]), variant
        assert np.array_equal(st["count_matrix"], ref["C"]), variant
    t = _to_dev(keys, dev)
    bsps.sort_(t, p, s, bsps.RAN_SR, seed=3)
    assert np.array_equal(_to_host(t), np.sort(keys))
