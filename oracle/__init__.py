"""CPU oracle for the BSP sample sort -- TEST INFRASTRUCTURE ONLY.

Plain single-thread C (``bsp_oracle.c``) behind ctypes. Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it;
the GPU library never imports it and shares no code with it.

``sort()`` simulates Sort_Det_BSP (paper Section 5.1, Figure SortD) or
Sort_IRan_BSP (Section 5.2, Figure SortRI) with the duplicate-key handling of
Section 5.1.1, and returns the sorted keys, the payload and every intermediate
(block-sorted array, sorted sample, splitters, count matrix, routed array).
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bsp_oracle.c")
_SRC_MT = os.path.join(_HERE, "bsp_oracle_mt.c")
LIB_PATH = os.path.join(_HERE, "liboracle.so")

DET, RAN = 0, 1
KIND = {"int32": 0, "int64": 1, "float32": 2}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, no SIMD intrinsics): the
    single-thread oracle and its threaded driver."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-Wno-unused-parameter", "-pthread", _SRC, _SRC_MT, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=True)
        L = ct.CDLL(LIB_PATH)
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        L.ora_order_keys.argtypes = [ct.c_int, ct.c_void_p, ct.c_int64, u64p]
        L.ora_mix64.restype = ct.c_uint64
        L.ora_mix64.argtypes = [ct.c_uint64]
        L.ora_feistel.restype = ct.c_int64
        L.ora_feistel.argtypes = [ct.c_uint64, ct.c_int64, ct.c_int64]
        L.ora_block_start.restype = ct.c_int64
        L.ora_block_start.argtypes = [ct.c_int64, ct.c_int, ct.c_int]
        L.ora_validate.argtypes = [ct.c_int64, ct.c_int, ct.c_int, ct.c_int]
        L.ora_sample_size.restype = ct.c_int64
        L.ora_sample_size.argtypes = [ct.c_int, ct.c_int, ct.c_int]
        L.ora_sort.argtypes = [u64p, ct.c_int64, ct.c_int, ct.c_int, ct.c_int, ct.c_uint64,
                               i64p, ct.c_void_p, ct.c_void_p, ct.c_void_p,
                               ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.ora_sort_mt.argtypes = L.ora_sort.argtypes + [ct.c_int]
        L.ora_sort_untagged.argtypes = L.ora_sort.argtypes
        L.ora_sort_sr.argtypes = [u64p, ct.c_int64, ct.c_int, ct.c_int, ct.c_uint64, i64p, ct.c_void_p,
                                  ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.ora_iter_k.argtypes = [ct.c_int, ct.c_int]
        L.ora_iter_k.restype = ct.c_int
        L.ora_sort_iter.argtypes = [u64p, ct.c_int64, ct.c_int, ct.c_int, ct.c_int, i64p, ct.c_void_p,
                                    ct.c_void_p, ct.c_void_p, ct.c_void_p]
        L.ora_rank.argtypes = [u64p, ct.c_int64, u64p, i64p, ct.c_int, i64p]
        L.ora_rmi_grad.restype = ct.c_double
        L.ora_rmi_grad.argtypes = [f64p, f64p, i32p, ct.c_int64, ct.c_int, f64p, f64p, f64p, f64p, f64p]
        L.ora_rmi_newton.argtypes = [ct.c_int, f64p, f64p, f64p, f64p]
        L.ora_rmi_fit.argtypes = [u64p, ct.c_int64, ct.c_int, ct.c_int, ct.c_int, ct.c_int,
                                  f64p, f64p, f64p, f64p, f64p]
        L.ora_rmi_predict.restype = ct.c_int64
        L.ora_rmi_predict.argtypes = [ct.c_uint64, ct.c_int, ct.c_int, f64p, f64p, f64p, f64p, f64p]
        _lib = L
    return _lib


def _kind(keys: np.ndarray) -> int:
    if keys.dtype == np.int32:
        return 0
    if keys.dtype == np.int64:
        return 1
    if keys.dtype == np.float32:
        return 2
    raise TypeError(f"unsupported key dtype {keys.dtype}")


def order_keys(keys: np.ndarray) -> np.ndarray:
    """Unsigned 64-bit order keys: their unsigned order is the key order."""
    keys = np.ascontiguousarray(keys)
    out = np.empty(keys.size, dtype=np.uint64)
    lib().ora_order_keys(_kind(keys), keys.ctypes.data, keys.size, out)
    return out


def mix64(z: int) -> int:
    return int(lib().ora_mix64(z & 0xFFFFFFFFFFFFFFFF))


def feistel(seed: int, n: int, t: int) -> int:
    return int(lib().ora_feistel(seed & 0xFFFFFFFFFFFFFFFF, n, t))


def block_start(n: int, p: int, k: int) -> int:
    return int(lib().ora_block_start(n, p, k))


def validate(n: int, p: int, s: int, variant: int) -> int:
    return int(lib().ora_validate(n, p, s, variant))


def sample_size(p: int, s: int, variant: int) -> int:
    return int(lib().ora_sample_size(p, s, variant))


class OracleError(ValueError):
    pass


def default_threads() -> int:
    """Host threads for the threaded driver: the cores this process may use,
    at most 16 (a host's CPU share per GPU on an 8-GPU node of 128 cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def sort(keys: np.ndarray, p: int, s: int, variant: int = DET, seed: int = 1,
         values: np.ndarray | None = None, intermediates: bool = True, threads: int = 1,
         untagged: bool = False) -> dict:
    """Run the simulated BSP sort (threads > 1: the same per-processor steps
    spread over that many host threads, byte-identical result; untagged: the
    duplicate handling switched off, splitters compared by key alone). Returns a dict with
    keys, values (if given), perm, and when `intermediates`:
    B_keys/B_perm (block-sorted), sample_key/sample_pos (sorted sample, order keys
    and positions in the block-sorted array), spl_key/spl_pos (p-1 splitters),
    C (p x p), bucket_sizes (p), Z_keys/Z_perm (routed)."""
    keys = np.ascontiguousarray(keys)
    n = keys.size
    ok = order_keys(keys)
    rc = validate(n, p, s, variant)
    if rc:
        raise OracleError(f"invalid arguments n={n} p={p} s={s} variant={variant} (rc={rc})")
    perm = np.empty(max(n, 1), dtype=np.int64)
    res = {}
    args = [None] * 7
    if intermediates:
        ns = sample_size(p, s, variant) if n >= 1 else 0
        B = np.empty(max(n, 1), dtype=np.int64)
        sk = np.empty(max(ns, 1), dtype=np.uint64)
        sp = np.empty(max(ns, 1), dtype=np.int64)
        pk = np.empty(max(p - 1, 1), dtype=np.uint64)
        pp = np.empty(max(p - 1, 1), dtype=np.int64)
        C = np.zeros(p * p, dtype=np.int64)
        Z = np.empty(max(n, 1), dtype=np.int64)
        args = [B.ctypes.data, sk.ctypes.data, sp.ctypes.data, pk.ctypes.data, pp.ctypes.data,
                C.ctypes.data, Z.ctypes.data]
    if untagged:
        rc = lib().ora_sort_untagged(ok, n, p, s, variant, seed & 0xFFFFFFFFFFFFFFFF, perm, *args)
    elif threads > 1:
        rc = lib().ora_sort_mt(ok, n, p, s, variant, seed & 0xFFFFFFFFFFFFFFFF, perm, *args, int(threads))
    else:
        rc = lib().ora_sort(ok, n, p, s, variant, seed & 0xFFFFFFFFFFFFFFFF, perm, *args)
    if rc:
        raise OracleError(f"oracle failed rc={rc}")
    perm = perm[:n]
    res["perm"] = perm
    res["keys"] = keys[perm]
    if values is not None:
        res["values"] = np.ascontiguousarray(values)[perm]
    if intermediates:
        B, Z = B[:n], Z[:n]
        res["B_perm"] = B
        res["B_keys"] = keys[B]
        if values is not None:
            res["B_values"] = values[B]
        res["sample_key"] = sk[:ns]
        res["sample_pos"] = sp[:ns]
        res["spl_key"] = pk[:p - 1]
        res["spl_pos"] = pp[:p - 1]
        res["C"] = C.reshape(p, p)
        res["bucket_sizes"] = res["C"].sum(axis=0)
        res["Z_perm"] = Z
        res["Z_keys"] = keys[Z]
    return res


def sort_sr(keys: np.ndarray, p: int, s: int, seed: int = 1, values: np.ndarray | None = None) -> dict:
    """Sort_Ran_BSP (Figure SortR): sample of the unsorted input, route, then
    sort every bucket. Returns keys, values (if given), perm, sample_key /
    sample_pos (sorted sample, order keys and INPUT positions), spl_key /
    spl_pos, C (p x p, row = input block), bucket_sizes, Z_perm (routed)."""
    keys = np.ascontiguousarray(keys)
    n = keys.size
    ok = order_keys(keys)
    if validate(n, p, s, RAN):
        raise OracleError(f"invalid arguments n={n} p={p} s={s}")
    ns = max(s * p - 1, 1)
    perm = np.empty(max(n, 1), dtype=np.int64)
    sk = np.empty(ns, dtype=np.uint64)
    sp = np.empty(ns, dtype=np.int64)
    pk = np.empty(max(p - 1, 1), dtype=np.uint64)
    pp = np.empty(max(p - 1, 1), dtype=np.int64)
    C = np.zeros(p * p, dtype=np.int64)
    Z = np.empty(max(n, 1), dtype=np.int64)
    rc = lib().ora_sort_sr(ok, n, p, s, seed & 0xFFFFFFFFFFFFFFFF, perm, sk.ctypes.data, sp.ctypes.data,
                           pk.ctypes.data, pp.ctypes.data, C.ctypes.data, Z.ctypes.data)
    if rc:
        raise OracleError(f"oracle failed rc={rc}")
    perm, Z = perm[:n], Z[:n]
    res = {"perm": perm, "keys": keys[perm], "sample_key": sk[:s * p - 1], "sample_pos": sp[:s * p - 1],
           "spl_key": pk[:p - 1], "spl_pos": pp[:p - 1], "C": C.reshape(p, p), "Z_perm": Z, "Z_keys": keys[Z]}
    res["bucket_sizes"] = res["C"].sum(axis=0)
    if values is not None:
        res["values"] = np.ascontiguousarray(values)[perm]
    return res


def iter_k(p: int, m: int) -> int:
    """k with k^m = p (0 when p is not an m-th power)."""
    return int(lib().ora_iter_k(p, m))


def sort_iter(keys: np.ndarray, p: int, s: int, m: int, values: np.ndarray | None = None,
              rounds: bool = False) -> dict:
    """Iterative Sort_Det_BSP (Section 5.1): local sort, then m rounds of
    k-way partitioning and merging, p = k^m. Returns keys, values (if
    given), perm, k, spl_key / spl_pos (p-1: round 1's k-1 splitters, then
    round 2's, group by group ...; order keys, positions in the round's input
    array), C (m x p x k: round, processor, bucket); with
    rounds=True also A_perm (m x n: original index of every element after
    each round)."""
    keys = np.ascontiguousarray(keys)
    n = keys.size
    ok = order_keys(keys)
    k = iter_k(p, m)
    if validate(n, p, s, DET) or k == 0:
        raise OracleError(f"invalid arguments n={n} p={p} s={s} m={m}")
    perm = np.empty(max(n, 1), dtype=np.int64)
    pk = np.empty(max(p - 1, 1), dtype=np.uint64)
    pp = np.empty(max(p - 1, 1), dtype=np.int64)
    C = np.zeros(m * p * k, dtype=np.int64)
    A = np.empty(max(m * n, 1), dtype=np.int64) if rounds else None
    rc = lib().ora_sort_iter(ok, n, p, s, m, perm, pk.ctypes.data, pp.ctypes.data, C.ctypes.data,
                             None if A is None else A.ctypes.data)
    if rc:
        raise OracleError(f"oracle failed rc={rc}")
    perm = perm[:n]
    res = {"perm": perm, "keys": keys[perm], "k": k, "spl_key": pk[:p - 1], "spl_pos": pp[:p - 1],
           "C": C.reshape(m, p, k)}
    if A is not None:
        res["A_perm"] = A[:m * n].reshape(m, n)
    if values is not None:
        res["values"] = np.ascontiguousarray(values)[perm]
    return res


def rank(B_keys: np.ndarray, spl_key: np.ndarray, spl_pos: np.ndarray) -> np.ndarray:
    """Bucket of every record (B[g], g) against the splitter records."""
    ok = order_keys(B_keys)
    out = np.empty(max(ok.size, 1), dtype=np.int64)
    lib().ora_rank(ok, ok.size, np.ascontiguousarray(spl_key, dtype=np.uint64),
                   np.ascontiguousarray(spl_pos, dtype=np.int64), int(spl_key.size), out)
    return out[:ok.size]


def sort_segmented(keys: np.ndarray, offsets: np.ndarray, params, values=None) -> dict:
    """Sort each segment [offsets[i], offsets[i+1]) on its own; params(i, n_i)
    returns (p, s, variant, seed) for segment i."""
    out_k = np.empty_like(keys)
    out_v = None if values is None else np.empty_like(values)
    for i in range(len(offsets) - 1):
        a, b = int(offsets[i]), int(offsets[i + 1])
        p, s, variant, seed = params(i, b - a)
        r = sort(keys[a:b], p, s, variant, seed, None if values is None else values[a:b],
                 intermediates=False)
        out_k[a:b] = r["keys"]
        if values is not None:
            out_v[a:b] = r["values"]
    return {"keys": out_k, "values": out_v}


# ---------------------------------------------------------------- learned model

def rmi_grad(x, y, leaf, c, d, mu):
    """Loss, gradient (2L) and Gram sums (3L) of the leaf models, float64."""
    L = len(c)
    g = np.empty(2 * L)
    h = np.empty(3 * L)
    loss = lib().ora_rmi_grad(np.ascontiguousarray(x, np.float64), np.ascontiguousarray(y, np.float64),
                              np.ascontiguousarray(leaf, np.int32), len(x), L,
                              np.ascontiguousarray(c, np.float64), np.ascontiguousarray(d, np.float64),
                              np.ascontiguousarray(mu, np.float64), g, h)
    return loss, g, h


def rmi_newton(g, h, c, d):
    c = np.array(c, dtype=np.float64)
    d = np.array(d, dtype=np.float64)
    lib().ora_rmi_newton(len(c), np.ascontiguousarray(g, np.float64), np.ascontiguousarray(h, np.float64), c, d)
    return c, d


def rmi_fit(sample_okeys: np.ndarray, p: int, s: int, L: int, iters: int = 2) -> dict:
    root = np.zeros(3)
    c = np.zeros(L)
    d = np.zeros(L)
    mu = np.zeros(L)
    lohi = np.zeros(2)
    sk = np.ascontiguousarray(sample_okeys, dtype=np.uint64)
    lib().ora_rmi_fit(sk, sk.size, p, s, L, iters, root, c, d, mu, lohi)
    return {"root": root, "c": c, "d": d, "mu": mu, "lohi": lohi, "p": p, "L": L}


def rmi_predict(model: dict, okeys: np.ndarray) -> np.ndarray:
    L_ = lib()
    out = np.empty(len(okeys), dtype=np.int64)
    for i, u in enumerate(okeys):
        out[i] = L_.ora_rmi_predict(int(u), model["p"], model["L"], model["root"], model["c"],
                                    model["d"], model["mu"], model["lohi"])
    return out
