"""GPU parity of the fused sort path against the CPU oracle, element by element.

Every case checks, bit for bit: the sorted keys (and payloads), the
block-sorted array (Figure SortD step 3), the sorted sample and the splitters
(steps 4-6), and the count matrix (step 9). Sizes span several tiles and
ragged tails; the all-equal and few-distinct inputs exercise the tie rule.
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


def _torch_keys(keys, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(keys)).to(dev)


def _run(dev, keys, p, s, variant, seed=1, values=None, chunk_cap=0, local_sort=0, untagged=False, route=0):
    import torch
    import paper_1408_6729_amd as bsps
    t = _torch_keys(keys, dev)
    v = None if values is None else torch.from_numpy(values.view(np.int32)).to(dev)
    st = bsps.sort_(t, p, s, variant, seed, values=v, chunk_cap=chunk_cap, stats=True, stats_arrays=True,
                    local_sort=local_sort, untagged=untagged, route=route)
    torch.cuda.synchronize()
    out = t.cpu().numpy()
    outv = None if v is None else v.cpu().numpy().view(np.uint32)
    return out, outv, st


def _bits(a):
    return a.view(np.uint32) if a.dtype == np.float32 else a


def _order(a):
    """Order keys (unsigned, same width) of int32 / int64 / float32 keys."""
    if a.dtype == np.float32:
        u = a.view(np.uint32)
        return np.where(u >> 31 == 1, ~u, u | np.uint32(0x80000000))
    if a.dtype == np.int32:
        return a.view(np.uint32) ^ np.uint32(0x80000000)
    return a.view(np.uint64) ^ np.uint64(1 << 63)


def _exact_blocks(B, Bv, p, D):
    """Blocks sorted on order key >> D only, equal keys in input order: checks
    that, then returns the blocks sorted stably by key (the exactly sorted
    blocks)."""
    B = B.copy()
    Bv = None if Bv is None else Bv.copy()
    n = B.size
    for k in range(p):
        lo, hi = k * n // p, (k + 1) * n // p
        o = _order(B[lo:hi])
        h = o >> o.dtype.type(D)
        assert np.all(h[1:] >= h[:-1]), f"block {k} not sorted on key >> {D}"
        idx = np.argsort(o, kind="stable")
        B[lo:hi] = B[lo:hi][idx]
        if Bv is not None:
            Bv[lo:hi] = Bv[lo:hi][idx]
    return B, Bv


def _check(ora, dev, keys, p, s, variant, seed=1, kv=False, chunk_cap=0, check_B=True, local_sort=0, untagged=False,
           route=0):
    vals = np.arange(keys.size, dtype=np.uint32) if kv else None
    ref = ora.sort(keys, p, s, variant, seed, vals, untagged=untagged)
    out, outv, st = _run(dev, keys, p, s, variant, seed, vals, chunk_cap, local_sort, untagged, route)
    assert np.array_equal(_bits(out), _bits(ref["keys"])), "sorted keys differ"
    if kv:
        assert np.array_equal(outv, ref["values"]), "payload order differs"
    if p > 1:
        assert np.array_equal(st["splitter_pos"], ref["spl_pos"]), "splitter tags differ"
        assert np.array_equal(_bits(st["splitter_keys"]), _bits(ref["B_keys"][ref["spl_pos"]])), "splitter keys differ"
        assert np.array_equal(st["sample_pos"], ref["sample_pos"]), "sample tags differ"
        assert np.array_equal(st["count_matrix"], ref["C"]), "count matrix differs"
        assert np.array_equal(st["bucket_sizes"], ref["bucket_sizes"])
    if check_B:
        B, Bv = st["block_sorted"], (st["block_sorted_values"][:keys.size] if kv else None)
        if st.get("block_shift", 0):
            B, Bv = _exact_blocks(B, Bv, p, st["block_shift"])
        assert np.array_equal(_bits(B), _bits(ref["B_keys"])), "block-sorted array differs"
        if kv:
            assert np.array_equal(Bv, ref["B_values"])
    return st


def test_c1_plain_det(ora, dev):
    """Plain DET: 2^20 int32 uniform keys, p = 16, s = 8."""
    keys = W.int32_keys(1 << 20, 16, "uniform")
    _check(ora, dev, keys, 16, 8, ora.DET)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("dist", W.DISTRIBUTIONS)
def test_c2_distributions_small(ora, dev, variant, dist):
    """The seven mid-size distributions at 2^21 keys, p = 128, s = 32."""
    keys = W.int32_keys(1 << 21, 128, dist)
    _check(ora, dev, keys, 128, 32, variant)


@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
@pytest.mark.parametrize("variant", [0, 1])
def test_ragged_random(ora, dev, dtype, variant):
    rng = np.random.default_rng(7)
    for trial in range(6):
        n = int(rng.integers(2, 300000))
        p = int(rng.integers(1, min(n, 300) + 1))
        s = int(rng.integers(1, 70))
        if variant == 1 and s * p - 1 > n:
            s = max(1, (n + 1) // p)
        distinct = None if trial % 2 else int(rng.integers(1, 50))
        keys = W.random_keys(n, dtype, seed=100 + trial, distinct=distinct)
        _check(ora, dev, keys, p, s, variant, seed=trial + 3, kv=(trial % 3 == 0))


@pytest.mark.parametrize("n", [2, 3, 17, 1000, 16383, 16384, 16385, 50001])
def test_edges(ora, dev, n):
    keys = W.random_keys(n, "int32", seed=n, distinct=max(1, n // 4))
    for p in sorted({1, 2, min(n, 7), min(n, 1024)}):
        _check(ora, dev, keys, p, 3, ora.DET)


@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
@pytest.mark.parametrize("n,p", [(2 * 16384 + 1, 2), (3 * 16384 + 2, 3), (5_000_003, 61)])
def test_tile_loop_edges(ora, dev, dtype, n, p):
    """Keys-only tile sorts run as a persistent grid that loads each next tile
    early: a block one tile long beside blocks one key longer leaves an empty
    tile inside the loop (first two cases), and 5*10^6 keys in 61 ragged blocks
    give more tiles than resident workgroups, with a partial tile per block."""
    keys = W.random_keys(n, dtype, seed=n + p, distinct=max(1, n // 3))
    _check(ora, dev, keys, p, 8, ora.DET)


@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
@pytest.mark.parametrize("span_bits", [1, 2, 3, 7, 13])
@pytest.mark.parametrize("kv", [False, True])
def test_narrow_ranges(ora, dev, dtype, span_bits, kv):
    """Keys spanning 2^span_bits consecutive order-key values. The rebased
    keys have 1-2 bits (a single pass of at most 2 bits, ranked without LDS
    counters), 3 bits (one 6-bit pass), 7 bits (6 + a 1-bit pass) or 13 bits
    (6 + 6 + 1), in the tile sorts and in every merge chunk."""
    rng = np.random.default_rng(span_bits * 7 + (1 if kv else 0))
    n = 3 * 16384 + 1234
    off = rng.integers(0, 1 << span_bits, size=n)
    if dtype == "int32":
        keys = (np.int64(-(1 << 20)) + off).astype(np.int32)
    elif dtype == "int64":
        keys = (np.int64(1 << 40) + off).astype(np.int64)
    else:
        # consecutive float32 bit patterns above 1.0
        keys = (np.uint32(0x3f800000) + off.astype(np.uint32)).view(np.float32)
    _check(ora, dev, keys, 5, 4, ora.DET, kv=kv)
    _check(ora, dev, keys, 5, 4, ora.RAN, kv=kv)


def test_p_limit(dev):
    import torch
    import paper_1408_6729_amd as bsps
    t = torch.zeros(5000, dtype=torch.int32, device=dev)
    with pytest.raises(bsps.BspsError) as e:
        bsps.sort_(t, 1025, 1, bsps.DET)
    assert e.value.code == bsps.EUNSUPPORTED


def test_all_equal_diagonal(ora, dev):
    keys = np.zeros(1 << 20, dtype=np.int32)
    st = _check(ora, dev, keys, 64, 16, ora.DET)
    m = (1 << 20) // 64
    assert np.array_equal(st["count_matrix"], np.diag(np.full(64, m)))


def test_oversize_chunk_path(ora, dev):
    """A small LDS chunk cap sends most merge chunks through the global path."""
    keys = W.random_keys(300000, "int32", seed=5, distinct=1000)
    st = _check(ora, dev, keys, 32, 16, ora.RAN, seed=9, kv=True, chunk_cap=600)
    assert st["oversize_chunks"] > 0
    keys64 = W.random_keys(200000, "int64", seed=6)
    st = _check(ora, dev, keys64, 16, 16, ora.DET, kv=True, chunk_cap=300)
    assert st["oversize_chunks"] > 0


def test_duplicate_stress_small(ora, dev):
    """Scaled-down duplicate stress: Zipf(1.2) int64 keys plus a 25% equal
    block, payload = original index, p = 256, s = 64."""
    keys, vals = W.zipf_int64_kv(1 << 21)
    ref = ora.sort(keys, 256, 64, ora.DET, 1, vals)
    out, outv, st = _run(dev, keys, 256, 64, ora.DET, 1, vals)
    assert np.array_equal(out, ref["keys"])
    assert np.array_equal(outv, ref["values"])
    eq = out[1:] == out[:-1]
    assert (outv[1:][eq] > outv[:-1][eq]).all()


@pytest.mark.parametrize("case", ["clusters", "spread_dups"])
@pytest.mark.parametrize("variant", [0, 1])
def test_int64_top_first_sort(ora, dev, case, variant):
    """Wide 64-bit keys are ranked on their top 30 bits first, and the lower
    passes run only where two different keys share those bits. "clusters":
    two clusters 2^63 apart of 2^16-wide offsets, so every tile and chunk has
    many different keys per top-bit class and always takes the full sort
    after the first; "spread_dups": 4096 values spread over the whole range,
    each repeated, so the first sort is the whole sort and the payloads must
    keep input order within equal keys. Key-value, against the oracle."""
    rng = np.random.Generator(np.random.PCG64(31 + variant))
    n = 1 << 20
    if case == "clusters":
        base = np.where(rng.random(n) < 0.5, np.int64(-(1 << 62)), np.int64(1 << 62))
        keys = base + rng.integers(0, 1 << 16, size=n, dtype=np.int64)
    else:
        vals = rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, size=4096, dtype=np.int64)
        keys = vals[rng.integers(0, vals.size, size=n)]
    _check(ora, dev, keys, 32, 16, variant, seed=3, kv=True)


def test_float_special_values(ora, dev):
    keys = W.lognormal_f32(1 << 20, zeros=1024)
    keys[:7] = np.array([np.inf, -np.inf, -0.0, 0.0, 1e-45, -1e-45, 3.4e38], dtype=np.float32)
    _check(ora, dev, keys, 64, 16, ora.RAN, seed=2)


def test_stream_copy_exact(dev):
    """The reference copy kernel behind the bench's attainable-bandwidth line
    copies every byte, including a tail shorter than one grid stride."""
    import torch
    import paper_1408_6729_amd as bsps
    for n in (4, 1 << 20, (1 << 22) + 12):
        src = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device=dev)
        dst = torch.zeros_like(src)
        bsps.stream_copy(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst), n


# ----------------------------------------------------------------- the two local sorts

LOCAL = [1, 2]  # tiles + multiway merge, LSD radix passes through HBM


@pytest.mark.parametrize("local_sort", LOCAL)
@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
@pytest.mark.parametrize("kv", [False, True])
def test_local_sorts_multi_tile_blocks(ora, dev, local_sort, dtype, kv):
    """Blocks of several tiles, ragged sizes (n not a multiple of p, block
    starts not 16-byte aligned, partial last tiles), many equal keys: the
    block-sorted array, sample, splitters, count matrix and output equal the
    oracle's with either local sort."""
    n = 7 * 16384 + 12345
    keys = W.random_keys(n, dtype, seed=31, distinct=3000)
    _check(ora, dev, keys, 3, 16, ora.DET, kv=kv, local_sort=local_sort)
    keys = W.random_keys(n, dtype, seed=32)
    _check(ora, dev, keys, 5, 8, ora.RAN, seed=4, kv=kv, local_sort=local_sort)


@pytest.mark.parametrize("dist", W.DISTRIBUTIONS)
def test_lsd_distributions(ora, dev, dist):
    """The seven distributions at 2^22 keys, p = 128 (two tiles per block),
    through the LSD local sort: positions where a block's keys share a digit
    are skipped (all-zero keys: one copying pass), so blocks run different
    numbers of passes."""
    keys = W.int32_keys(1 << 22, 128, dist)
    for variant in (0, 1):
        _check(ora, dev, keys, 128, 32, variant, local_sort=2)


@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
@pytest.mark.parametrize("span_bits", [0, 1, 8, 9, 20])
def test_lsd_digit_positions(ora, dev, dtype, span_bits):
    """Keys spanning 2^span_bits consecutive order-key values, key-value,
    through the LSD local sort: 0 to 3 digit positions differ inside a block."""
    rng = np.random.default_rng(span_bits + 100)
    n = 4 * 16384 + 999
    off = rng.integers(0, 1 << span_bits, size=n) if span_bits else np.zeros(n, dtype=np.int64)
    if dtype == "int32":
        keys = (np.int64(-(1 << 24)) + off).astype(np.int32)
    elif dtype == "int64":
        keys = (np.int64(1 << 44) + off).astype(np.int64)
    else:
        keys = (np.uint32(0x3f800000) + off.astype(np.uint32)).view(np.float32)
    _check(ora, dev, keys, 2, 4, ora.DET, kv=True, local_sort=2)


def test_lsd_many_blocks(ora, dev):
    """More blocks than resident workgroups (each workgroup walks several
    blocks), one tile per block plus a few keys."""
    n = 1100 * 16390
    keys = W.random_keys(n, "int32", seed=77, distinct=n // 2)
    _check(ora, dev, keys, 1024, 8, ora.DET, local_sort=2)


# ----------------------------------------------------------------- duplicate handling switched off

@pytest.mark.parametrize("route", [0, 1])
@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("case", ["distinct", "dict", "zero", "int64kv"])
def test_untagged_against_oracle(ora, dev, route, variant, case):
    """The ablation of Section 6.4: splitters compared by key alone. Output,
    payloads, splitters and count matrix equal the untagged oracle's; with
    distinct keys the count matrix also equals the tagged one, and with all-equal
    keys every key lands in bucket 0."""
    n = 3 * 16384 + 777
    if case == "distinct":
        keys = np.random.default_rng(3).permutation(n).astype(np.int32)
    elif case == "dict":
        keys = W.random_keys(n, "int32", seed=8, distinct=300)
    elif case == "zero":
        keys = np.zeros(n, dtype=np.int32)
    else:
        keys = W.random_keys(n, "int64", seed=9, distinct=500)
    st = _check(ora, dev, keys, 16, 8, variant, seed=2, kv=case != "distinct", untagged=True, route=route)
    if case == "distinct":
        tagged = ora.sort(keys, 16, 8, variant, 2)
        assert np.array_equal(st["count_matrix"], tagged["C"])
    if case == "zero":
        assert np.array_equal(st["count_matrix"][:, 1:], np.zeros((16, 15), dtype=np.int64))


# ----------------------------------------------------------------- Sort_Ran_BSP (Figure SortR)

def _check_sr(ora, dev, keys, p, s, seed=1, kv=False, bucketing=0, untagged=False):
    import torch
    import paper_1408_6729_amd as bsps
    vals = np.arange(keys.size, dtype=np.uint32) if kv else None
    ref = ora.sort_sr(keys, p, s, seed, vals)
    t = _torch_keys(keys, dev)
    v = None if vals is None else torch.from_numpy(vals.view(np.int32)).to(dev)
    st = bsps.sort_(t, p, s, bsps.RAN_SR, seed, values=v, bucketing=bucketing, leaves=256, stats=True,
                    stats_arrays=True, untagged=untagged)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(t.cpu().numpy()), _bits(ref["keys"])), "sorted keys differ"
    if kv:
        assert np.array_equal(v.cpu().numpy().view(np.uint32), ref["values"]), "payload order differs"
    if p > 1:
        assert np.array_equal(st["sample_pos"], ref["sample_pos"]), "sample tags (input positions) differ"
        assert np.array_equal(st["splitter_pos"], ref["spl_pos"]), "splitter tags differ"
        assert np.array_equal(_bits(st["splitter_keys"]), _bits(keys[ref["spl_pos"]]))
    assert np.array_equal(st["count_matrix"], ref["C"]), "count matrix differs"
    assert np.array_equal(_bits(st["routed"][:keys.size]), _bits(ref["Z_keys"])), "routed array differs"
    # the bucket of every input record: the bucket its routed position falls in
    want = np.empty(keys.size, np.uint32)
    want[ref["Z_perm"]] = np.repeat(np.arange(p, dtype=np.uint32), ref["bucket_sizes"])
    assert np.array_equal(st["buckets"][:keys.size], want), "per-record bucket ids differ"
    return st


@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
@pytest.mark.parametrize("kv", [False, True])
@pytest.mark.parametrize("bucketing", [0, 1])
def test_sr_against_oracle(ora, dev, dtype, kv, bucketing):
    """Sort_Ran_BSP: sample of the unsorted input, splitters, every input record
    ranked (splitter search or learned model with the exact check), routed in
    input order, buckets sorted. Output, payloads, sample and splitter tags,
    count matrix and routed array equal the oracle's; ragged sizes, buckets
    of several tiles, duplicates."""
    rng = np.random.default_rng(21 + bucketing)
    for trial in range(3):
        n = int(rng.integers(50000, 400000))
        p = int(rng.integers(2, 300))
        s = max(1, min(int(rng.integers(1, 40)), (n + 1) // p))
        keys = W.random_keys(n, dtype, seed=trial + 60, distinct=None if trial % 2 else 500)
        _check_sr(ora, dev, keys, p, s, seed=trial + 2, kv=kv, bucketing=bucketing)


@pytest.mark.parametrize("case", ["zero", "p1", "p1024", "untagged"])
def test_sr_edges(ora, dev, case):
    if case == "zero":
        st = _check_sr(ora, dev, np.zeros(100003, dtype=np.int32), 64, 8, kv=True)
        assert st["bucket_sizes"].max() < 4 * 100003 / 64  # ties split by position
    elif case == "p1":
        _check_sr(ora, dev, W.random_keys(70001, "int32", seed=3), 1, 1, kv=True)
    elif case == "p1024":
        _check_sr(ora, dev, W.random_keys(1 << 21, "float32", seed=4), 1024, 16, bucketing=1)
    else:
        keys = W.random_keys(200000, "int32", seed=5, distinct=100)
        vals = np.arange(keys.size, dtype=np.uint32)
        import torch
        import paper_1408_6729_amd as bsps
        t = _torch_keys(keys, dev)
        v = torch.from_numpy(vals.view(np.int32)).to(dev)
        bsps.sort_(t, 32, 8, bsps.RAN_SR, 3, values=v, untagged=True)
        assert np.array_equal(t.cpu().numpy(), keys[np.argsort(keys, kind="stable")])
        assert np.array_equal(v.cpu().numpy().view(np.uint32), np.argsort(keys, kind="stable").astype(np.uint32))


@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
def test_truncated_tile_sort(ora, dev, dtype):
    """Tiles of multi-tile blocks sorted on the key's high part only, the block
    merge cutting on that part, and the blocks themselves left sorted on a high
    part (the block shift): on spread-out keys both are on, on keys with a
    value of 1/64 of the input they are off, and in every case the block-sorted
    array (after a stable sort of every block), sample, splitters, counts and
    output equal the oracle's. Last, a value filling a quarter of every block but
    none of the 1024 positions the shift's probe samples (block k's sample i
    sits at start_k + floor(i m_k / 1024)): the truncation stays on, and the
    value's group, larger than a merge chunk, pushes chunks to the
    global-memory sort."""
    n, p = 1_300_001, 8  # blocks of about 10 tiles
    keys = W.random_keys(n, dtype, seed=61)
    st = _check(ora, dev, keys, p, 32, ora.DET, kv=True)
    assert st["trunc_shift"] > 0 and st["block_shift"] > 0
    # every value about three times: groups of equal high parts hold equal
    # keys on both sides of a splitter, which the tags must order
    few = keys[np.random.default_rng(64).integers(0, n // 3, n)]
    for variant, untagged in ((ora.DET, False), (ora.RAN, False), (ora.DET, True)):
        st = _check(ora, dev, few, p, 32, variant, kv=True, seed=7, untagged=untagged)
        assert st["block_shift"] > 0
    heavy = keys.copy()
    heavy[np.random.default_rng(62).choice(n, n // 64, replace=False)] = heavy[0]
    st = _check(ora, dev, heavy, p, 32, ora.RAN, kv=True, seed=5)
    assert st["trunc_shift"] == 0
    missed = keys.copy()
    rng = np.random.default_rng(63)
    for k in range(p):
        lo, hi = k * n // p, (k + 1) * n // p
        m = hi - lo
        free = np.setdiff1d(np.arange(lo, hi), lo + (np.arange(1024) * m) // 1024)
        missed[rng.choice(free, m // 4, replace=False)] = keys[n // 2]
    st = _check(ora, dev, missed, p, 32, ora.DET, kv=True)
    assert st["trunc_shift"] > 0 and st["oversize_block"] > 0 and st["block_shift"] > 0


def test_block_shift_limit(ora, dev):
    """The blocks stay exactly sorted above 256 virtual processors (the block
    shift is off), and below it on all-equal keys (the tile sort is full)."""
    keys = W.random_keys(10_240_001, "int32", seed=65)  # blocks of 2 tiles
    st = _check(ora, dev, keys, 512, 4, ora.DET)
    assert st["trunc_shift"] > 0 and st["block_shift"] == 0
    st = _check(ora, dev, np.full(1 << 21, 7, dtype=np.int32), 64, 8, ora.RAN, kv=True)
    assert st["trunc_shift"] == 0 and st["block_shift"] == 0


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_merge_plan_int64_no_oversize(ora, dev, dist):
    """The tiles of a block are alike, so every run's j-th sample sits near the
    same quantile; the boundary pick's subsample starts each run at a
    different phase, so that the subsamples do not line up across the runs
    near both ends of the key range. With one phase the block merge of int64
    key-value blocks of 128 tiles left ~10-15 chunks per block past the tile
    (a boundary took a whole row of aligned subsamples at once); now none."""
    n, p = 1 << 24, 16  # blocks of 2^20 int64 keys: 128 tiles of 8 Ki
    if dist == "uniform":
        keys = W.random_keys(n, "int64", seed=71)
    else:
        keys, _ = W.zipf_int64_kv(n, equal_frac=0.0, seed=72)
    st = _check(ora, dev, keys, p, 32, ora.DET, kv=True)
    assert st["oversize_block"] == 0
