"""Seeded synthetic inputs for the BSP sample sort (host numpy, PCG64).

This module only draws input data. It holds none of the sorting method's
arithmetic, and both the CPU oracle and the GPU library are fed from it.

Workload definitions follow the paper's benchmark section (Section 6.3,
"Sorting Benchmarks"): processor i draws its share of [U] with seed
21 + 1001*i, and INT_MAX there means 2^31. Each generator returns a numpy
array (and, for key-value workloads, a uint32 payload array).

Distributions of the mid-size DET/RAN workload (2^26 int32 keys, p = 128):
  uniform   [U]  uniform in [0, 2^31)
  gauss     [G]  mean of four uniform draws, rounded down
  zero           every key 0 (all duplicates)
  bucket    [B]  each share split into p runs of n/p^2 keys; run i uniform in
                 [i*M/p, (i+1)*M/p)
  staggered [S]  share i < p/2 uniform in [(2i+1)M/p, (2i+2)M/p); share
                 i >= p/2 uniform in [(i-p/2)M/p, (i-p/2+1)M/p)
  ggroup    [g-G] g = 8: group j = i // g; run r of the share uniform in
                 [c*M/p, (c+1)*M/p) with c = (j*g + p/2 + r) mod p (the upper
                 end wraps together with the lower one)
  dict1024       2^10 distinct values drawn once, keys drawn from them
The paper's [DD] definition is garbled and [WR] is defined only in a cited
report that is not available; the all-zero and 2^10-distinct inputs stand in
for the duplicate-heavy cases.
"""
from __future__ import annotations

import numpy as np

M31 = 1 << 31  # the paper's INT_MAX: 2^31
SEED_BASE = 21
SEED_STRIDE = 1001

DISTRIBUTIONS = ("uniform", "gauss", "zero", "bucket", "staggered", "ggroup", "dict1024")


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _shares(n: int, p: int):
    """Yield (i, lo, hi): the contiguous share of processor i, sizes differ by <= 1."""
    for i in range(p):
        yield i, (i * n) // p, ((i + 1) * n) // p


def _uniform_range(rng, lo: int, hi: int, size: int) -> np.ndarray:
    return rng.integers(lo, hi, size=size, dtype=np.int64).astype(np.int32)


def int32_keys(n: int, p: int, dist: str = "uniform", g: int = 8) -> np.ndarray:
    """int32 keys in [0, 2^31) of the named distribution, one seed per share."""
    out = np.empty(n, dtype=np.int32)
    if dist == "zero":
        out[:] = 0
        return out
    if dist == "dict1024":
        d = _uniform_range(_rng(SEED_BASE), 0, M31, 1 << 10)
        while np.unique(d).size != d.size:  # keep exactly 2^10 distinct values
            d = np.unique(np.concatenate([d, _uniform_range(_rng(d.size), 0, M31, 1 << 10)]))[: 1 << 10]
        for i, lo, hi in _shares(n, p):
            idx = _rng(SEED_BASE + SEED_STRIDE * i).integers(0, d.size, size=hi - lo)
            out[lo:hi] = d[idx]
        return out
    step = M31 // p
    for i, lo, hi in _shares(n, p):
        rng = _rng(SEED_BASE + SEED_STRIDE * i)
        m = hi - lo
        if dist == "uniform":
            out[lo:hi] = _uniform_range(rng, 0, M31, m)
        elif dist == "gauss":
            s = rng.integers(0, M31, size=(4, m), dtype=np.int64).sum(axis=0)
            out[lo:hi] = (s // 4).astype(np.int32)
        elif dist == "bucket":
            for r, (a, b) in enumerate(_runs(m, p)):
                out[lo + a:lo + b] = _uniform_range(rng, r * step, (r + 1) * step, b - a)
        elif dist == "staggered":
            c = 2 * i + 1 if i < p // 2 else i - p // 2
            out[lo:hi] = _uniform_range(rng, c * step, (c + 1) * step, m)
        elif dist == "ggroup":
            j = i // g
            for r, (a, b) in enumerate(_runs(m, g)):
                c = (j * g + p // 2 + r) % p
                out[lo + a:lo + b] = _uniform_range(rng, c * step, (c + 1) * step, b - a)
        else:
            raise ValueError(f"unknown distribution {dist!r}")
    return out


def _runs(m: int, parts: int):
    return [((r * m) // parts, ((r + 1) * m) // parts) for r in range(parts)]


def zipf_int64_kv(n: int, distinct: int = 1 << 16, alpha: float = 1.2,
                  equal_frac: float = 0.25, seed: int = SEED_BASE):
    """Duplicate-stress keys: Zipf(alpha) ranks over `distinct` int64 values,
    plus an unaligned block of equal_frac*n copies of the most frequent value.
    Payload = original index (uint32)."""
    rng = _rng(seed)
    vals = rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, size=distinct,
                        dtype=np.int64, endpoint=True)
    while np.unique(vals).size != distinct:
        vals = rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, size=distinct,
                            dtype=np.int64, endpoint=True)
    w = np.arange(1, distinct + 1, dtype=np.float64) ** (-alpha)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    keys = np.empty(n, dtype=np.int64)
    chunk = 1 << 24
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        r = np.searchsorted(cdf, rng.random(b - a), side="right")
        keys[a:b] = vals[np.minimum(r, distinct - 1)]
    lo = int(0.3 * n)
    keys[lo:lo + int(equal_frac * n)] = vals[0]
    payload = np.arange(n, dtype=np.uint32)
    return keys, payload


def lognormal_f32(n: int, seed: int = SEED_BASE, zeros: int = 1024) -> np.ndarray:
    """float32 keys from a mixture of three lognormals (weights .5/.3/.2,
    ln-space (mu, sigma) = (0,1), (3,.5), (-3,.25)), drawn in float64 and
    rounded; `zeros` copies each of -0.0 and +0.0 at seeded positions. No NaN/Inf."""
    rng = _rng(seed)
    out = np.empty(n, dtype=np.float32)
    mu = np.array([0.0, 3.0, -3.0])
    sg = np.array([1.0, 0.5, 0.25])
    chunk = 1 << 24
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        comp = np.searchsorted(np.array([0.5, 0.8]), rng.random(b - a), side="right")
        z = rng.standard_normal(b - a)
        out[a:b] = np.exp(mu[comp] + sg[comp] * z).astype(np.float32)
    if zeros and n >= 2 * zeros:
        pos = rng.choice(n, size=2 * zeros, replace=False)
        out[pos[:zeros]] = np.float32(-0.0)
        out[pos[zeros:]] = np.float32(0.0)
    assert np.isfinite(out).all()
    return out


def segment_sizes(nseg: int = 4096, lo_log2: int = 8, hi_log2: int = 20,
                  seed: int = SEED_BASE) -> np.ndarray:
    """Segment sizes floor(2^(lo + (hi-lo)*U)), log-uniform in [2^lo, 2^hi]."""
    u = _rng(seed).random(nseg)
    return np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)).astype(np.int64)


def segmented_int32(sizes: np.ndarray, seed: int = SEED_BASE):
    """Concatenated int32 segments: even segments uniform in [0, 2^31), odd
    segments drawn from a per-segment dictionary of 2^8 distinct values.
    Returns (keys, offsets[nseg+1])."""
    offs = np.zeros(len(sizes) + 1, dtype=np.int64)
    np.cumsum(sizes, out=offs[1:])
    keys = np.empty(int(offs[-1]), dtype=np.int32)
    for i, m in enumerate(sizes):
        rng = _rng(seed + SEED_STRIDE * (i + 1))
        a, b = int(offs[i]), int(offs[i + 1])
        if i % 2 == 0:
            keys[a:b] = _uniform_range(rng, 0, M31, int(m))
        else:
            d = _uniform_range(rng, 0, M31, 1 << 8)
            keys[a:b] = d[rng.integers(0, d.size, size=int(m))]
    return keys, offs


def random_keys(n: int, dtype: str, seed: int, distinct: int | None = None) -> np.ndarray:
    """Small generic inputs for tests: full-range random keys of dtype
    ('int32', 'int64', 'float32'); `distinct` limits the number of values."""
    rng = _rng(seed)
    if dtype == "int32":
        base = rng.integers(-(1 << 31), 1 << 31, size=distinct or n, dtype=np.int64).astype(np.int32)
    elif dtype == "int64":
        base = rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, size=distinct or n,
                            dtype=np.int64, endpoint=True)
    elif dtype == "float32":
        bits = rng.integers(0, 1 << 32, size=distinct or n, dtype=np.uint64).astype(np.uint32)
        f = bits.view(np.float32)
        bad = ~np.isfinite(f)
        bits[bad] &= np.uint32(0x807FFFFF)  # clear the exponent: finite (denormal or zero)
        base = bits.view(np.float32)
    else:
        raise ValueError(dtype)
    if distinct is None:
        return base
    return base[rng.integers(0, base.size, size=n)]
