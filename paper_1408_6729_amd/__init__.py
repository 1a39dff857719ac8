"""MI355X BSP sample sort: Python binding of libbsps.so (ctypes).

Argument marshalling only: every step of the sort runs in the library's HIP
kernels on the tensor's GPU. Device memory (keys, payload, workspace) comes
from torch on the tensor's device; the work is enqueued on
torch.cuda.current_stream(). The library must have been built
(`python -m paper_1408_6729_amd.build` or `__graft_entry__.build()`);
importing this package fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np
# torch first: the library must bind to the HIP runtime torch has loaded
# (loading it before torch can leave the process with two runtimes).
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("BSPS_LIB") or os.path.join(_HERE, "libbsps.so")

OK, EINVAL, EWORKSPACE, EDEVICE, EUNSUPPORTED = 0, 1, 2, 3, 4
DET, RAN, RAN_SR = 0, 1, 2
I32, I64, F32 = 0, 1, 2
SPLITTER, LEARNED = 0, 1
ROUTE_FUSED, ROUTE_SCATTER = 0, 1
LOCAL_AUTO, LOCAL_MERGE, LOCAL_LSD = 0, 1, 2


class BspsError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} (status {code})")
        self.code = code


class Params(ct.Structure):
    _fields_ = [("p", ct.c_int32), ("s", ct.c_int32), ("variant", ct.c_int32), ("bucketing", ct.c_int32),
                ("route", ct.c_int32), ("leaves", ct.c_int32), ("seed", ct.c_uint64),
                ("chunk_cap", ct.c_int32), ("local_sort", ct.c_int32), ("untagged", ct.c_int32),
                ("rounds", ct.c_int32), ("reserved", ct.c_int32 * 4)]


class Stats(ct.Structure):
    _fields_ = [("splitter_keys", ct.c_void_p), ("splitter_pos", ct.c_void_p), ("sample_keys", ct.c_void_p),
                ("sample_pos", ct.c_void_p), ("bucket_sizes", ct.c_void_p), ("count_matrix", ct.c_void_p),
                ("block_sorted", ct.c_void_p), ("block_sorted_values", ct.c_void_p), ("routed", ct.c_void_p),
                ("buckets", ct.c_void_p), ("max_bucket_ratio", ct.c_double), ("mispredict_rate", ct.c_double),
                ("mean_fix_dist", ct.c_double), ("oversize_chunks", ct.c_int64), ("reserved_i", ct.c_int64 * 4),
                ("seg_models", ct.c_void_p), ("seg_grad", ct.c_void_p), ("seg_gram", ct.c_void_p),
                ("seg_capacity", ct.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    L = ct.CDLL(LIB_PATH)
    vp, sz, i32, i64 = ct.c_void_p, ct.c_size_t, ct.c_int32, ct.c_int64
    PP = ct.POINTER(Params)
    SP = ct.POINTER(Stats)
    L.bsps_workspace_bytes.restype = sz
    L.bsps_workspace_bytes.argtypes = [i64, i32, i32, PP]
    L.bsps_sort.restype = i32
    L.bsps_sort.argtypes = [vp, i64, i32, PP, vp, sz, vp, SP]
    L.bsps_sort_kv.restype = i32
    L.bsps_sort_kv.argtypes = [vp, vp, i64, i32, PP, vp, sz, vp, SP]
    L.bsps_sort_noalloc.restype = i32
    L.bsps_sort_noalloc.argtypes = [vp, vp, i64, i32, PP, vp]
    L.bsps_status_string.restype = ct.c_char_p
    L.bsps_status_string.argtypes = [i32]
    L.bsps_rank.restype = i32
    L.bsps_rank.argtypes = [vp, i64, i32, i32, vp, vp, i32, vp, vp, vp, vp, sz, vp, SP]
    L.bsps_rank_workspace_bytes.restype = sz
    L.bsps_rank_workspace_bytes.argtypes = [i64, i32]
    L.bsps_model_bytes.restype = sz
    L.bsps_model_bytes.argtypes = [i32]
    L.bsps_fit_workspace_bytes.restype = sz
    L.bsps_fit_workspace_bytes.argtypes = [i64, i32]
    L.bsps_fit_model.restype = i32
    L.bsps_fit_model.argtypes = [vp, i64, i32, i32, i32, i32, i32, vp, vp, sz, vp]
    L.bsps_model_grad.restype = i32
    L.bsps_model_grad.argtypes = [vp, i64, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, sz, vp]
    L.bsps_sort_segmented.restype = i32
    L.bsps_sort_segmented.argtypes = [vp, vp, vp, i32, i32, ct.c_char_p, vp, sz, vp, SP]
    L.bsps_segmented_workspace_bytes.restype = sz
    L.bsps_segmented_workspace_bytes.argtypes = [vp, i32, i32, i32, ct.c_char_p]
    L.bsps_tuning_format.restype = ct.c_char_p
    L.bsps_tuning_format.argtypes = []
    L.bsps_stream_copy.restype = i32
    L.bsps_stream_copy.argtypes = [vp, vp, sz, vp]
    L.bsps_release_cache.restype = None
    L.bsps_release_cache.argtypes = []
    L.bsps_check_sort.restype = i64
    L.bsps_check_sort.argtypes = [i64, i32, i32, PP, ct.c_char_p, sz]
    L.bsps_check_segmented.restype = i64
    L.bsps_check_segmented.argtypes = [vp, i32, i32, i32, ct.c_char_p, ct.c_char_p, sz]
    L.bsps_timing.argtypes = [ct.c_int]
    L.bsps_timing_read.argtypes = [vp, vp, ct.c_int, ct.c_int]
    return L


_lib = _load()
lib = _lib

EXPORTS = ("bsps_workspace_bytes", "bsps_sort", "bsps_sort_kv", "bsps_sort_segmented",
           "bsps_segmented_workspace_bytes", "bsps_rank", "bsps_rank_workspace_bytes", "bsps_model_bytes",
           "bsps_fit_model", "bsps_fit_workspace_bytes", "bsps_model_grad", "bsps_status_string",
           "bsps_tuning_format", "bsps_release_cache")


def status_string(code: int) -> str:
    return _lib.bsps_status_string(int(code)).decode()


def make_params(p: int, s: int, variant: int = DET, seed: int = 1, bucketing: int = SPLITTER,
                route: int = ROUTE_FUSED, leaves: int = 0, chunk_cap: int = 0, local_sort: int = LOCAL_AUTO,
                untagged: bool = False, rounds: int = 1) -> Params:
    prm = Params()
    prm.p, prm.s, prm.variant, prm.bucketing = p, s, variant, bucketing
    prm.route, prm.leaves, prm.seed, prm.chunk_cap = route, leaves, seed & 0xFFFFFFFFFFFFFFFF, chunk_cap
    prm.local_sort = local_sort
    prm.untagged = int(bool(untagged))
    prm.rounds = rounds
    return prm


def _dtype_code(t) -> int:
    import torch
    if t.dtype == torch.int32:
        return I32
    if t.dtype == torch.int64:
        return I64
    if t.dtype == torch.float32:
        return F32
    raise TypeError(f"unsupported key dtype {t.dtype}")


def workspace_bytes(n: int, dtype: int, with_values: bool, prm: Params) -> int:
    return int(_lib.bsps_workspace_bytes(n, dtype, int(with_values), ct.byref(prm)))


def _stream(t) -> int:
    import torch
    return torch.cuda.current_stream(t.device).cuda_stream


def sort_(keys, p: int, s: int, variant: int = DET, seed: int = 1, values=None, bucketing: int = SPLITTER,
          route: int = ROUTE_FUSED, leaves: int = 0, chunk_cap: int = 0, stats: bool = False, workspace=None,
          stats_arrays: bool = False, local_sort: int = LOCAL_AUTO, untagged: bool = False, rounds: int = 1):
    """Sorts `keys` (a contiguous int32/int64/float32 CUDA tensor) in place; with
    `values` (uint32 payload as an int32 tensor of the same length) a key-value
    sort. With stats=True the call synchronizes and returns the diagnostic
    statistics (splitters, sample, counts, bucket sizes ...); stats_arrays=True
    adds the n-element arrays (block-sorted keys and payloads, and for the
    scatter route the routed keys and bucket ids; Sort_Ran_BSP the routed keys).
    rounds=m >= 2 runs the iterative Sort_Det_BSP (p = k^m); its count matrix
    comes back as m x p x k (round, processor, bucket) and its p-1 splitters
    are round 1's, then round 2's group by group, ..."""
    import torch
    assert keys.is_cuda and keys.is_contiguous() and keys.dim() == 1
    n = keys.numel()
    dt = _dtype_code(keys)
    prm = make_params(p, s, variant, seed, bucketing, route, leaves, chunk_cap, local_sort, untagged, rounds)
    hasv = values is not None
    if hasv:
        assert values.is_cuda and values.is_contiguous() and values.numel() == n and values.element_size() == 4
    need = workspace_bytes(n, dt, hasv, prm)
    if need == 0:
        code = _lib.bsps_sort(None, n, dt, ct.byref(prm), None, 0, None, None)
        raise BspsError(code if code else EINVAL, "bsps_workspace_bytes")
    ws = workspace if workspace is not None else torch.empty(need, dtype=torch.uint8, device=keys.device)
    st = None
    host = {}
    if stats:
        st = Stats()
        kd = {I32: np.int32, I64: np.int64, F32: np.float32}[dt]
        ns = p * s if variant == DET else p * s - 1
        host = {
            "splitter_keys": np.zeros(max(p - 1, 1), kd), "splitter_pos": np.zeros(max(p - 1, 1), np.int64),
            "sample_keys": np.zeros(max(ns, 1), kd), "sample_pos": np.zeros(max(ns, 1), np.int64),
            "bucket_sizes": np.zeros(p, np.int64), "count_matrix": np.zeros(p * p, np.int64),
        }
        if stats_arrays:
            host["block_sorted"] = np.zeros(max(n, 1), kd)
        if hasv and stats_arrays:
            host["block_sorted_values"] = np.zeros(max(n, 1), np.uint32)
        if (route == ROUTE_SCATTER or variant == RAN_SR) and stats_arrays:
            host["routed"] = np.zeros(max(n, 1), kd)
            host["buckets"] = np.zeros(max(n, 1), np.uint32)
        for k, arr in host.items():
            setattr(st, k, arr.ctypes.data)
    args = (ct.byref(prm), ct.c_void_p(ws.data_ptr()), ws.numel(), ct.c_void_p(_stream(keys)),
            ct.byref(st) if st is not None else None)
    if hasv:
        code = _lib.bsps_sort_kv(ct.c_void_p(keys.data_ptr()), ct.c_void_p(values.data_ptr()), n, dt, *args)
    else:
        code = _lib.bsps_sort(ct.c_void_p(keys.data_ptr()), n, dt, *args)
    if code != OK:
        raise BspsError(code, "bsps_sort")
    if not stats:
        return None
    out = {k: v for k, v in host.items()}
    out["splitter_keys"] = out["splitter_keys"][:p - 1]
    out["splitter_pos"] = out["splitter_pos"][:p - 1]
    ns = p * s if variant == DET else p * s - 1
    out["sample_keys"] = out["sample_keys"][:ns]
    out["sample_pos"] = out["sample_pos"][:ns]
    if rounds >= 2 and p > 1:
        k = round(p ** (1.0 / rounds))
        out["count_matrix"] = out["count_matrix"][:rounds * p * k].reshape(rounds, p, k)
    else:
        out["count_matrix"] = out["count_matrix"].reshape(p, p)
    if stats_arrays:
        out["block_sorted"] = out["block_sorted"][:n]
    out["max_bucket_ratio"] = st.max_bucket_ratio
    out["mispredict_rate"] = st.mispredict_rate
    out["mean_fix_dist"] = st.mean_fix_dist
    out["oversize_chunks"] = st.oversize_chunks
    out["oversize_block"], out["oversize_bucket"], out["oversize_max"] = (int(x) for x in st.reserved_i[:3])
    # low key bits the tile sort left to the block merge, and the block merge to the bucket merge
    out["trunc_shift"] = int(st.reserved_i[3]) & 0xFF
    out["block_shift"] = (int(st.reserved_i[3]) >> 8) & 0xFF
    return out


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


NOALLOC_SCRATCH_BYTES = 64 << 20  # BSPS_NOALLOC_SCRATCH_BYTES of bsps.h


def sort_noalloc_(keys, p: int, s: int, variant: int = DET, seed: int = 1, values=None, bucketing: int = SPLITTER,
                  route: int = ROUTE_FUSED, leaves: int = 0, chunk_cap: int = 0, local_sort: int = LOCAL_AUTO) -> None:
    """As sort_(), through bsps_sort_noalloc: no workspace is allocated, the
    library's per-GPU scratch array is used (sizes whose workspace exceeds
    NOALLOC_SCRATCH_BYTES are rejected with EUNSUPPORTED)."""
    assert keys.is_cuda and keys.is_contiguous() and keys.dim() == 1
    n = keys.numel()
    if values is not None:
        assert values.is_cuda and values.is_contiguous() and values.numel() == n and values.element_size() == 4
    prm = make_params(p, s, variant, seed, bucketing, route, leaves, chunk_cap, local_sort)
    code = _lib.bsps_sort_noalloc(ct.c_void_p(keys.data_ptr()), _ptr(values), n, _dtype_code(keys), ct.byref(prm),
                                  ct.c_void_p(_stream(keys)))
    if code != OK:
        raise BspsError(code, "bsps_sort_noalloc")


def rank(keys, p: int, spl_keys, spl_pos, bucketing: int = SPLITTER, model=None, buckets=None, counts=None,
         stats: bool = False):
    """Bucket of every key of a block-sorted array (dtype of `keys`) against the
    p-1 splitter records (spl_keys same dtype, spl_pos uint32 as int32 tensor).
    Fills `buckets` (n, int32 view of uint32) and `counts` (p*p) when given."""
    import torch
    n = keys.numel()
    dt = _dtype_code(keys)
    ws = torch.empty(_lib.bsps_rank_workspace_bytes(n, p), dtype=torch.uint8, device=keys.device)
    st = Stats() if stats else None
    code = _lib.bsps_rank(_ptr(keys), n, dt, p, _ptr(spl_keys), _ptr(spl_pos), bucketing, _ptr(model),
                          _ptr(buckets), _ptr(counts), _ptr(ws), ws.numel(), ct.c_void_p(_stream(keys)),
                          ct.byref(st) if st is not None else None)
    if code != OK:
        raise BspsError(code, "bsps_rank")
    if stats:
        return {"mispredict_rate": st.mispredict_rate, "mean_fix_dist": st.mean_fix_dist}
    return None


def model_bytes(leaves: int) -> int:
    return int(_lib.bsps_model_bytes(leaves))


def fit_model(sample_keys, p: int, s: int, leaves: int = 4096, iters: int = 2):
    """Trains the learned bucketing model on a sorted sample (dtype of the
    tensor) with the library's forward / backward / Newton-update kernels.
    Returns the device model buffer (uint8 tensor)."""
    import torch
    N = sample_keys.numel()
    model = torch.zeros(model_bytes(leaves), dtype=torch.uint8, device=sample_keys.device)
    ws = torch.empty(_lib.bsps_fit_workspace_bytes(N, leaves), dtype=torch.uint8, device=sample_keys.device)
    code = _lib.bsps_fit_model(_ptr(sample_keys), N, _dtype_code(sample_keys), p, s, leaves, iters, _ptr(model),
                               _ptr(ws), ws.numel(), ct.c_void_p(_stream(sample_keys)))
    if code != OK:
        raise BspsError(code, "bsps_fit_model")
    return model


def model_grad(sample_keys, p: int, s: int, leaves: int, model):
    """Forward + backward of the leaf stage at the model's parameters:
    returns (leaf ids, gradient [2L], Gram sums [3L], loss) as tensors."""
    import torch
    N = sample_keys.numel()
    d = sample_keys.device
    leaf = torch.empty(N, dtype=torch.int32, device=d)
    grad = torch.empty(2 * leaves, dtype=torch.float32, device=d)
    gram = torch.empty(3 * leaves, dtype=torch.float32, device=d)
    loss = torch.empty(1, dtype=torch.float32, device=d)
    ws = torch.empty(_lib.bsps_fit_workspace_bytes(N, leaves), dtype=torch.uint8, device=d)
    code = _lib.bsps_model_grad(_ptr(sample_keys), N, _dtype_code(sample_keys), p, s, leaves, _ptr(model),
                                _ptr(leaf), _ptr(grad), _ptr(gram), _ptr(loss), _ptr(ws), ws.numel(),
                                ct.c_void_p(_stream(sample_keys)))
    if code != OK:
        raise BspsError(code, "bsps_model_grad")
    return leaf, grad, gram, loss


def model_fields(model):
    """Host view of a model buffer (device tensor or host uint8 array): header
    dict and (L, 3) float32 leaf table."""
    raw = model if isinstance(model, np.ndarray) else model.cpu().numpy()
    lo, hi = np.frombuffer(raw[:16].tobytes(), dtype=np.float64)
    a, b, mur, inv = np.frombuffer(raw[16:32].tobytes(), dtype=np.float32)
    L, p, s, _ = np.frombuffer(raw[32:48].tobytes(), dtype=np.int32)
    leaf = np.frombuffer(raw[48:48 + 12 * int(L)].tobytes(), dtype=np.float32).reshape(int(L), 3)
    return {"lo": lo, "hi": hi, "a": a, "b": b, "mur": mur, "inv": inv, "L": int(L), "p": int(p), "s": int(s)}, leaf


TUNING_PATH = os.path.join(_HERE, "tuning_mi355x.json")
_tuning_cache: list = []


def default_tuning() -> str | None:
    """The size-class table the segmented sort uses when none is given: the
    autotuner's output beside this file if present (else the library's
    built-in table, returned here as None)."""
    if not _tuning_cache:
        txt = None
        if os.path.exists(TUNING_PATH):
            with open(TUNING_PATH) as f:
                txt = f.read()
        _tuning_cache.append(txt)
    return _tuning_cache[0]


def _tuning_arg(tuning):
    t = tuning if tuning is not None else default_tuning()
    return t.encode() if t else None


def segmented_workspace_bytes(offsets, dtype: int, with_values: bool, tuning: str | None = None) -> int:
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    return int(_lib.bsps_segmented_workspace_bytes(off.ctypes.data, len(off) - 1, dtype, int(with_values),
                                                   _tuning_arg(tuning)))


SEG_LEAVES = 64  # leaves of a large segment's model


def sort_segmented_(keys, offsets, values=None, tuning: str | None = None, stats: bool = False, workspace=None,
                    models: int = 0):
    """Sorts every segment [offsets[i], offsets[i+1]) of `keys` (and `values`)
    in place, all segments in one captured graph launch. `offsets`: host array
    of nseg + 1 non-decreasing int64 starting at 0. `tuning`: a size-class
    table (JSON, `tuning_format()`); default `default_tuning()`. With stats and
    models = capacity > 0, the result also holds the learned models of the
    large segments and their leaf-stage gradient and Gram sums."""
    import torch
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nseg = len(off) - 1
    dt = _dtype_code(keys)
    tj = _tuning_arg(tuning)
    need = _lib.bsps_segmented_workspace_bytes(off.ctypes.data, nseg, dt, int(values is not None), tj)
    if need == 0 and nseg > 0 and off[-1] > 0:
        code = _lib.bsps_sort_segmented(None, None, off.ctypes.data, nseg, dt, tj, None, 0, None, None)
        raise BspsError(code if code else EINVAL, "bsps_segmented_workspace_bytes")
    ws = workspace if workspace is not None else torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
    st = Stats() if stats else None
    mbuf = gbuf = hbuf = None
    if stats and models > 0:
        mbuf = np.zeros(models * model_bytes(SEG_LEAVES), dtype=np.uint8)
        gbuf = np.zeros(models * SEG_LEAVES * 2, dtype=np.float32)
        hbuf = np.zeros(models * SEG_LEAVES * 3, dtype=np.float32)
        st.seg_models, st.seg_grad, st.seg_gram = mbuf.ctypes.data, gbuf.ctypes.data, hbuf.ctypes.data
        st.seg_capacity = models
    code = _lib.bsps_sort_segmented(_ptr(keys), _ptr(values), off.ctypes.data, nseg, dt, tj, _ptr(ws), ws.numel(),
                                    ct.c_void_p(_stream(keys)), ct.byref(st) if st is not None else None)
    if code != OK:
        raise BspsError(code, "bsps_sort_segmented")
    if stats:
        return {"oversize_chunks": st.oversize_chunks, "blocks": st.reserved_i[0], "merged_segments": st.reserved_i[1],
                "graph": bool(st.reserved_i[2]), "graph_cached": st.reserved_i[2] == 2, "learned_segments": st.reserved_i[3],
                "mispredict_rate": st.mispredict_rate, "mean_fix_dist": st.mean_fix_dist,
                "models": mbuf, "grad": gbuf, "gram": hbuf}
    return None


def tuning_format() -> str:
    return _lib.bsps_tuning_format().decode()


def stream_copy(src, dst) -> None:
    """Copies the contiguous CUDA tensor src into dst (same number of bytes, a
    multiple of 16, 16-byte aligned) with the library's reference copy kernel,
    on the current stream: the attainable-bandwidth yardstick of the bench."""
    import torch
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("stream_copy: sizes differ")
    code = _lib.bsps_stream_copy(ct.c_void_p(src.data_ptr()), ct.c_void_p(dst.data_ptr()), nbytes,
                                 ct.c_void_p(torch.cuda.current_stream().cuda_stream))
    if code:
        raise BspsError(code, "bsps_stream_copy")


def check_sort(n: int, dtype: int, with_values: bool, prm: Params) -> tuple[int, str]:
    """Host dry run of a sort's plan (no GPU): (findings, report)."""
    buf = ct.create_string_buffer(1 << 16)
    k = int(_lib.bsps_check_sort(n, dtype, int(with_values), ct.byref(prm), buf, len(buf)))
    return k, buf.value.decode()


def check_segmented(offsets, dtype: int, with_values: bool, tuning: str | None = None) -> tuple[int, str]:
    """Host dry run of a segmented sort's plan (no GPU): (findings, report)."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    buf = ct.create_string_buffer(1 << 16)
    k = int(_lib.bsps_check_segmented(off.ctypes.data, len(off) - 1, dtype, int(with_values), _tuning_arg(tuning),
                                      buf, len(buf)))
    return k, buf.value.decode()


def release_cache() -> None:
    _lib.bsps_release_cache()
