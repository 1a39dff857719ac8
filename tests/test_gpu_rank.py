"""GPU parity of per-key bucket ranking (splitter search and learned model),
the scatter routing, and the learned model's gradient against the oracle."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    assert torch.cuda.is_available()
    import paper_1408_6729_amd  # noqa: F401
    return torch.device("cuda:0")


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _bits(a):
    return a.view(np.uint32) if a.dtype == np.float32 else a


@pytest.mark.parametrize("bucketing", [0, 1])
@pytest.mark.parametrize("dtype,variant", [("int32", 0), ("float32", 1), ("int64", 0)])
def test_scatter_route_parity(ora, dev, bucketing, dtype, variant):
    """Route by per-key ranking: buckets, count matrix, routed array and the
    sorted output all equal the oracle's (Figure SortD steps 9-12)."""
    import torch
    import paper_1408_6729_amd as bsps
    n, p, s = 300001, 64, 24
    keys = W.lognormal_f32(n, zeros=64) if dtype == "float32" else W.random_keys(n, dtype, seed=3, distinct=5000)
    vals = np.arange(n, dtype=np.uint32)
    ref = ora.sort(keys, p, s, variant, 5, vals)
    t = _t(keys, dev)
    v = _t(vals.view(np.int32), dev)
    st = bsps.sort_(t, p, s, variant, seed=5, values=v, bucketing=bucketing, route=bsps.ROUTE_SCATTER,
                    leaves=256, stats=True, stats_arrays=True)
    torch.cuda.synchronize()
    assert np.array_equal(_bits(t.cpu().numpy()), _bits(ref["keys"]))
    assert np.array_equal(v.cpu().numpy().view(np.uint32), ref["values"])
    assert np.array_equal(st["count_matrix"], ref["C"])
    assert np.array_equal(_bits(st["routed"]), _bits(ref["Z_keys"]))
    truth = ora.rank(ref["B_keys"], ref["spl_key"], ref["spl_pos"])
    assert np.array_equal(st["buckets"].astype(np.int64), truth)
    if bucketing == 1:
        assert 0.0 <= st["mispredict_rate"] < 0.5


@pytest.mark.parametrize("p", [3, 64, 1024])
@pytest.mark.parametrize("bucketing", [0, 1])
def test_scatter_route_without_diagnostics(ora, dev, p, bucketing):
    """Scatter route with no diagnostic arrays: no per-key bucket ids are kept,
    and the runs are routed from the count matrix alone (Figure SortD steps
    10-11); output keys and payloads equal the oracle's."""
    import torch
    import paper_1408_6729_amd as bsps
    n, s = 500003, 16
    keys = W.random_keys(n, "int32", seed=7, distinct=20000)
    vals = np.arange(n, dtype=np.uint32)
    ref = ora.sort(keys, p, s, ora.DET, 1, vals)
    t = _t(keys, dev)
    v = _t(vals.view(np.int32), dev)
    bsps.sort_(t, p, s, ora.DET, values=v, bucketing=bucketing, route=bsps.ROUTE_SCATTER, leaves=64)
    torch.cuda.synchronize()
    assert np.array_equal(t.cpu().numpy(), ref["keys"])
    assert np.array_equal(v.cpu().numpy().view(np.uint32), ref["values"])


@pytest.mark.parametrize("dtype", ["int32", "int64", "float32"])
@pytest.mark.parametrize("bucketing", [0, 1])
def test_scatter_route_random(ora, dev, dtype, bucketing):
    """Seeded sweep of the scatter route: random n, p (odd and even, up to
    1024), s, leaf count, variant and payload; sorted keys, payloads and the
    count matrix equal the oracle's (Figure SortD steps 9-12)."""
    import torch
    import paper_1408_6729_amd as bsps
    rng = np.random.default_rng(11 + 7 * bucketing + {"int32": 0, "int64": 1, "float32": 2}[dtype])
    for trial in range(4):
        n = int(rng.integers(2, 300000))
        p = int(rng.integers(2, min(n, 1024) + 1))
        s = int(rng.integers(1, 40))
        variant = trial % 2
        if variant == 1 and s * p - 1 > n:
            s = max(1, (n + 1) // p)
        leaves = int(rng.integers(1, 4097))
        if dtype == "float32":
            keys = W.lognormal_f32(n, seed=200 + trial, zeros=min(64, n // 4))
        else:
            keys = W.random_keys(n, dtype, seed=200 + trial, distinct=None if trial % 2 else int(rng.integers(1, 5000)))
        kv = trial % 2 == 0
        vals = np.arange(n, dtype=np.uint32) if kv else None
        ref = ora.sort(keys, p, s, variant, trial + 1, vals)
        t = _t(keys, dev)
        v = _t(vals.view(np.int32), dev) if kv else None
        st = bsps.sort_(t, p, s, variant, seed=trial + 1, values=v, bucketing=bucketing, route=bsps.ROUTE_SCATTER,
                        leaves=leaves, stats=True)
        torch.cuda.synchronize()
        case = f"n={n} p={p} s={s} variant={variant} leaves={leaves} kv={kv}"
        assert np.array_equal(_bits(t.cpu().numpy()), _bits(ref["keys"])), case
        if kv:
            assert np.array_equal(v.cpu().numpy().view(np.uint32), ref["values"]), case
        assert np.array_equal(st["count_matrix"], ref["C"]), case


@pytest.mark.parametrize("p", [2, 100, 1024])
@pytest.mark.parametrize("bucketing", [0, 1])
def test_rank_entry_point(ora, dev, p, bucketing):
    """bsps_rank on the oracle's block-sorted array and splitters."""
    import torch
    import paper_1408_6729_amd as bsps
    n, s = 1 << 19, 32
    keys = W.lognormal_f32(n, zeros=16)
    ref = ora.sort(keys, p, s, ora.RAN, 11)
    B = _t(ref["B_keys"], dev)
    sk = _t(ref["B_keys"][ref["spl_pos"]], dev)
    sp = _t(ref["spl_pos"].astype(np.int32), dev)
    buckets = torch.empty(n, dtype=torch.int32, device=dev)
    counts = torch.empty(p * p, dtype=torch.int32, device=dev)
    model = None
    if bucketing == 1:
        sorted_sample = _t(ref["B_keys"][ref["sample_pos"]], dev)
        model = bsps.fit_model(sorted_sample, p, s, leaves=1024)
    st = bsps.rank(B, p, sk, sp, bucketing, model, buckets, counts, stats=True)
    torch.cuda.synchronize()
    truth = ora.rank(ref["B_keys"], ref["spl_key"], ref["spl_pos"])
    assert np.array_equal(buckets.cpu().numpy().astype(np.int64), truth)
    assert np.array_equal(counts.cpu().numpy().reshape(p, p), ref["C"])
    if bucketing == 1:
        assert st["mispredict_rate"] < 0.3, st


# ----------------------------------------------------------------- learned model vs the oracle
#
# Training and inference take one integer decision in floating point: the leaf
# floor(L r(x)) of every sample. The GPU takes it in FP32, the oracle in FP64.
# The test samples are therefore built so that every sample's L r(x) lies far
# (about 0.15 leaf widths or more) from a leaf boundary, while each leaf's own
# data is not a straight line: leaf l holds k keys at design positions
# w = (l + z_j) / L, with z_j in [0.15, 0.85] drawn per leaf and mirrored about
# 1/2 (z_j + z_{k-1-j} = 1). The targets are y = (l + (j + 1/2)/k) / L, so
# y - w depends on j only through a pattern that averages to zero in every leaf;
# the least-squares root then predicts L r = l + z_j up to terms of order
# 1/L^2, and both sides put every sample in leaf l. The FP32 root and x differ
# from FP64 by a few 1e-4 leaf widths at L = 4096.


def _f32_from_order(ok):
    """float32 values whose totalOrder keys are `ok` (inverse of the order map)."""
    ok = ok.astype(np.uint32)
    bits = np.where(ok & np.uint32(0x80000000), ok & np.uint32(0x7FFFFFFF), ~ok)
    return bits.astype(np.uint32).view(np.float32)


def _leaf_pos(root, lohi, okeys, L):
    """L r(x) of each order key in FP64 (the value the leaf decision floors)."""
    lo, hi = lohi
    x = (okeys.astype(np.float64) - lo) / (hi - lo)
    return (root[0] * (x - root[2]) + root[1]) * L


def _leafy_sample(L, k, seed):
    """Order keys (uint64, sorted, distinct) of L*k positive float32 keys laid
    out as described above, spanning 2^16 order-key units per leaf."""
    rng = np.random.default_rng(seed)
    half = np.stack([0.15 + np.sort(rng.choice(22000, size=k // 2, replace=False)) / 65536.0 for _ in range(L)])
    z = np.concatenate([half, 1.0 - half[:, ::-1]], axis=1)
    w = (np.arange(L)[:, None] + z).reshape(-1)
    ok = (0x80000000 + (1 << 20) + np.round(w * (1 << 16))).astype(np.uint64)
    assert np.all(np.diff(ok) > 0)
    return ok


def _check_margins(ora, ok, m, L, root=None):
    v = _leaf_pos(m["root"] if root is None else root, m["lohi"], ok, L)
    lid = np.clip(np.floor(v), 0, L - 1).astype(np.int64)
    fr = v - np.floor(v)
    assert np.min(np.minimum(fr, 1 - fr)) > 0.1, "a sample lies near a leaf boundary"
    return lid


@pytest.mark.parametrize("iters", [1, 2])
def test_model_fit_matches_oracle(ora, dev, iters):
    """Fit kernels (init, centres, forward, backward, Newton update; root then
    leaves) against the oracle's FP64 fit of the same sorted sample: the range,
    the root line and every leaf's centre, slope and intercept, for one and two
    Newton iterations. p = 1024, s = 64, L = 4096 as in the learned workload."""
    import paper_1408_6729_amd as bsps
    p, s, L = 1024, 64, 4096
    ok = _leafy_sample(L, 16, seed=11)
    m = ora.rmi_fit(ok, p, s, L, iters)
    model = bsps.fit_model(_t(_f32_from_order(ok), dev), p, s, leaves=L, iters=iters)
    hdr, leaf = bsps.model_fields(model)
    assert (hdr["lo"], hdr["hi"]) == tuple(m["lohi"])
    assert hdr["L"] == L and hdr["p"] == p and hdr["s"] == s
    # root: sums of N = 2^16 terms by FP32 tree reductions, error about lg N * 2^-24 of the sum of magnitudes
    assert np.allclose([hdr["a"], hdr["b"], hdr["mur"]], m["root"], rtol=1e-4, atol=1e-6)
    c, d, mu = (leaf[:, i].astype(np.float64) for i in range(3))
    # leaf membership by the oracle's root; the margin makes it the GPU's too
    lid = _check_margins(ora, ok, m, L)
    x = (ok.astype(np.float64) - m["lohi"][0]) / (m["lohi"][1] - m["lohi"][0])
    cnt = np.bincount(lid, minlength=L)
    sx = np.bincount(lid, weights=x, minlength=L)
    sxx = np.bincount(lid, weights=x * x, minlength=L)
    sig = np.sqrt(np.maximum(sxx / np.maximum(cnt, 1) - (sx / np.maximum(cnt, 1)) ** 2, 0))
    empty = cnt == 0
    # empty leaves: c = 0, d = (samples below) / (p s), exactly in FP32
    assert np.array_equal(c[empty], np.zeros(empty.sum()))
    below = np.concatenate([[0], np.cumsum(cnt)[:-1]])
    assert np.array_equal(leaf[empty, 1], (below[empty] / (p * s)).astype(np.float32))
    used = ~empty
    eps = 2.0 ** -23  # bound of the FP32 error of x (rounding of u - lo and of 1/(hi - lo))
    assert np.all(np.abs(mu[used] - m["mu"][used]) <= 4 * eps + 1e-5 * np.abs(m["mu"][used]))
    assert np.all(np.abs(d[used] - m["d"][used]) <= 2e-5)
    # slope: relative error about 2 eps / sigma_x of the leaf (centred x); leaves
    # whose x spread is below FP32 resolution are singular on either side
    ok_c = used & (sig > 2.0 ** -16) & (cnt >= 2)
    tol = np.abs(m["c"][ok_c]) * (1e-4 + 8 * eps / sig[ok_c]) + 1e-6
    err = np.abs(c[ok_c] - m["c"][ok_c])
    assert np.all(err <= tol), (err / tol).max()
    assert ok_c.sum() > 0.8 * used.sum()
    # the leaves' data are not lines: the fit leaves a residual
    assert np.abs(m["c"][used] - 1).max() > 1e-3


@pytest.mark.parametrize("L", [2, 8])
@pytest.mark.parametrize("iters", [1, 2])
def test_model_fit_hand_worked(dev, L, iters):
    """The GPU fit of the 8-key example worked by hand (tests/golden/rmi_worked_n8.json):
    root, leaf lines, centres and the empty-leaf intercepts of L = 8, in FP32."""
    import json
    import os
    from fractions import Fraction
    import paper_1408_6729_amd as bsps
    with open(os.path.join(os.path.dirname(__file__), "golden", "rmi_worked_n8.json")) as f:
        g = json.load(f)
    u = np.array(g["sample_okeys"], dtype=np.int64)
    keys = (u - (1 << 31)).astype(np.int32)  # int32 keys whose order keys are u
    model = bsps.fit_model(_t(keys, dev), g["p"], g["s"], leaves=L, iters=iters)
    hdr, leaf = bsps.model_fields(model)
    assert (hdr["lo"], hdr["hi"]) == tuple(float(v) for v in g["lohi"])
    fr = lambda v: float(Fraction(v))  # noqa: E731
    assert np.allclose([hdr["a"], hdr["b"], hdr["mur"]], [fr(g["root"][k]) for k in ("a", "b", "mu_r")],
                       rtol=0, atol=2e-6)
    e = g["models"][str(L)]
    for i, name in enumerate(("c", "d", "mu")):
        assert np.allclose(leaf[:, i], [fr(v) for v in e[name]], rtol=0, atol=4e-6), name


@pytest.mark.parametrize("k", [1, 16])
def test_model_fit_equally_spaced(dev, k):
    """Equally spaced sample keys, the closed form of the CPU pin: root a = (N-1)/N,
    b = mu_r = 1/2, leaf l: c = (N-1)/N (0 for one-record leaves),
    mu = (l k + (k-1)/2)/(N-1), d = (l k + k/2)/N, at L = 4096."""
    import paper_1408_6729_amd as bsps
    L = 4096
    N = L * k
    p = 1024 if N >= 1024 else N
    s = N // p
    t = np.arange(N)
    keys = (1000 + 7 * t - (1 << 31)).astype(np.int32)
    model = bsps.fit_model(_t(keys, dev), p, s, leaves=L, iters=1)
    hdr, leaf = bsps.model_fields(model)
    a = (N - 1) / N
    assert np.allclose([hdr["a"], hdr["b"], hdr["mur"]], [a, 0.5, 0.5], rtol=0, atol=1e-5)
    lidx = np.arange(L)
    # slope: relative error about 8 eps / sigma_x of a leaf (eps = 2^-23, sigma_x =
    # sqrt((k^2 - 1)/12) / (N - 1) for k equally spaced records)
    sig = np.sqrt((k * k - 1) / 12) / (N - 1)
    tol = a * 8 * 2.0 ** -23 / sig if k > 1 else 0.0
    assert np.allclose(leaf[:, 0], np.full(L, a if k > 1 else 0.0), rtol=0, atol=tol + 1e-7)
    assert np.allclose(leaf[:, 2], (lidx * k + (k - 1) / 2) / (N - 1), rtol=0, atol=1e-6)
    assert np.allclose(leaf[:, 1], (lidx * k + k / 2) / N, rtol=0, atol=1e-6)


def test_model_gradient_matches_fp64(ora, dev):
    """Forward and backward kernels at given parameters: the oracle's FP64 fit
    rounded to FP32 and perturbed (seeded), written into the model buffer. The
    FP32 gradient, Gram sums and loss equal the oracle's FP64 ones at the same
    parameters, with the leaf of every sample decided alike on both sides."""
    import torch
    import paper_1408_6729_amd as bsps
    p, s, L = 256, 64, 512
    ok = _leafy_sample(L, 32, seed=12)
    m = ora.rmi_fit(ok, p, s, L, 2)
    rng = np.random.default_rng(1)
    c = (m["c"] * (1 + 0.1 * rng.standard_normal(L))).astype(np.float32)
    d = (m["d"] + 0.01 * rng.standard_normal(L)).astype(np.float32)
    mu = m["mu"].astype(np.float32)
    root = m["root"].astype(np.float32)
    lo, hi = m["lohi"]
    hdr = np.zeros(48, dtype=np.uint8)
    hdr[0:16] = np.frombuffer(np.array([lo, hi], dtype=np.float64).tobytes(), dtype=np.uint8)
    inv = np.float32(1.0 / (hi - lo))
    hdr[16:32] = np.frombuffer(np.array([root[0], root[1], root[2], inv], dtype=np.float32).tobytes(), np.uint8)
    hdr[32:48] = np.frombuffer(np.array([L, p, s, 0], dtype=np.int32).tobytes(), dtype=np.uint8)
    tab = np.stack([c, d, mu], axis=1).astype(np.float32)
    raw = np.concatenate([hdr, np.frombuffer(tab.tobytes(), dtype=np.uint8)])
    model = torch.from_numpy(raw).to(dev)
    smp_t = _t(_f32_from_order(ok), dev)
    lid, grad, gram, loss = bsps.model_grad(smp_t, p, s, L, model)
    torch.cuda.synchronize()
    lid_ref = _check_margins(ora, ok, m, L, root.astype(np.float64)).astype(np.int32)
    assert np.array_equal(lid.cpu().numpy(), lid_ref)
    x = (ok.astype(np.float64) - lo) / (hi - lo)
    y = (np.arange(ok.size) + 0.5) / (p * s)
    l64, g64, h64 = ora.rmi_grad(x, y, lid_ref, c.astype(np.float64), d.astype(np.float64), mu.astype(np.float64))
    g = grad.cpu().numpy().astype(np.float64)
    h = gram.cpu().numpy().astype(np.float64)
    scale = np.abs(g64).max()
    assert np.abs(g - g64).max() <= 1e-4 * scale, (np.abs(g - g64).max(), scale)
    assert np.allclose(h, h64, rtol=1e-4, atol=1e-6 * np.abs(h64).max())
    assert abs(loss.item() - l64) <= 1e-4 * l64


def test_model_training_reduces_loss_and_predicts_buckets(ora, dev):
    """Forward/backward/update: after training, the loss is far below the
    untrained one and most keys are predicted in their exact bucket."""
    import torch
    import paper_1408_6729_amd as bsps
    n, p, s, L = 1 << 20, 1024, 16, 4096
    keys = W.lognormal_f32(n, zeros=64)
    ref = ora.sort(keys, p, s, ora.DET)
    smp_t = _t(ref["B_keys"][ref["sample_pos"]], dev)
    m0 = bsps.fit_model(smp_t, p, s, leaves=L, iters=1)
    m2 = bsps.fit_model(smp_t, p, s, leaves=L, iters=2)
    zero = m2.clone()
    zero[48:] = 0
    _, _, _, loss0 = bsps.model_grad(smp_t, p, s, L, zero)
    _, g1, _, loss1 = bsps.model_grad(smp_t, p, s, L, m0)
    _, g2, _, loss2 = bsps.model_grad(smp_t, p, s, L, m2)
    torch.cuda.synchronize()
    assert loss1.item() < 1e-3 * loss0.item()
    assert loss2.item() <= loss1.item() * 1.01
    B = _t(ref["B_keys"], dev)
    sk = _t(ref["B_keys"][ref["spl_pos"]], dev)
    sp = _t(ref["spl_pos"].astype(np.int32), dev)
    buckets = torch.empty(n, dtype=torch.int32, device=dev)
    st = bsps.rank(B, p, sk, sp, 1, m2, buckets, None, stats=True)
    truth = ora.rank(ref["B_keys"], ref["spl_key"], ref["spl_pos"])
    assert np.array_equal(buckets.cpu().numpy().astype(np.int64), truth)
    assert st["mispredict_rate"] < 0.25 and st["mean_fix_dist"] < 0.5, st
