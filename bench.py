#!/usr/bin/env python3
"""Benchmark of the BSP sample sort on one MI355X.

Headline workload: 2^28 int32 keys uniform in [0, 2^31), drawn per virtual
processor with the paper's seeding (Section 6.3), p = 256 virtual processors,
oversampling s = 64, the deterministic variant Sort_Det_BSP (Figure SortD),
keys only. One step = one complete sort of one staged copy of the input
(local block sort, sample, splitters, bucket boundaries, prefix sums,
per-bucket merge), with the input already resident in HBM. The randomized
variant (Figure SortRI) is timed on the same input.

Beside it (in "detail"), each timed the same way:
  learned    2^28 float32 keys (mixture of three lognormals), p = 1024, s = 64:
             per-key ranking by the learned CDF model against plain splitter
             search, the scatter routing, identical outputs required
  int64_kv   2^28 int64 keys, Zipf(1.2) over 2^16 values + 25% equal block,
             uint32 payload, p = 256, s = 64
  segmented  4096 int32 segments, log-uniform sizes in [2^8, 2^20], one
             graph launch per step

Prints one JSON line: throughput in keys/s, the roofline of the dominant
kernel (algorithmic bytes over its HIP-event-timed duration against the
8 TB/s HBM peak, and against the rate the library's reference copy kernel
attains on the same array), and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only c0,learned,int64_kv,segmented]
"""
from __future__ import annotations

import argparse
import ctypes as ct
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STAGES = ["tile_sort", "block_merge", "sample_splitters", "bucket_ranking", "prefix_routing",
          "bucket_merge", "k_mwm_merge(block)", "k_mwm_merge(bucket)", "k_rank"]
ALL = ("c0", "learned", "int64_kv", "segmented")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_1408_6729_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel: str, workload: str):
    """HBM bytes per launch measured with rocprofv3 counters for this exact
    kernel source, if a committed measurement exists (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(workload, {}).get(kernel)
    if not e or e.get("source_hash") != source_hash():
        return None
    return e.get("bytes_per_launch")


def cpu_baseline(log2n: int, p: int, s: int):
    """The oracle (plain single-thread C) on a bounded sample of the workload."""
    import oracle
    import workloads as W
    n = 1 << log2n
    keys = W.int32_keys(n, p, "uniform")
    t0 = time.perf_counter()
    oracle.sort(keys, p, s, oracle.DET, intermediates=False)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "keys/s", "cores": 1, "kind": "oracle",
            "sample": f"2^{log2n} int32 uniform keys of the same distribution, p={p}, s={s}, DET, "
                      f"one thread, {dt:.1f} s"}


def to_dev(torch, a):
    """Host array -> cuda:0 through a pinned (hipHostMalloc) buffer."""
    h = torch.from_numpy(a)
    pin = torch.empty(h.shape, dtype=h.dtype, pin_memory=True)
    pin.copy_(h)
    return pin.to("cuda:0")


class Timer:
    """The library's per-stage HIP-event timing (events on the stream the
    kernels run on)."""

    def __init__(self, bsps):
        self.lib = bsps.lib

    def start(self):
        ms = (ct.c_double * len(STAGES))()
        cnt = (ct.c_int64 * len(STAGES))()
        self.lib.bsps_timing_read(ms, cnt, len(STAGES), 1)
        self.lib.bsps_timing(1)

    def stop(self, steps: int):
        self.lib.bsps_timing(0)
        ms = (ct.c_double * len(STAGES))()
        cnt = (ct.c_int64 * len(STAGES))()
        self.lib.bsps_timing_read(ms, cnt, len(STAGES), 1)
        return {STAGES[i]: {"ms_per_launch": ms[i] / cnt[i], "launches_per_step": cnt[i] / steps}
                for i in range(len(STAGES)) if cnt[i]}


def time_sort(bsps, torch, base, K, Wm, p, s, variant=0, bucketing=0, route=0, leaves=0, vbase=None,
              timer=None):
    """K timed sorts (after Wm untimed) of fresh device copies of `base`;
    returns (ms per step, stage timings, last output keys, last output values)."""
    dev = base.device
    n = base.numel()
    copies = torch.empty((K + Wm, n), dtype=base.dtype, device=dev)
    vcopies = None if vbase is None else torch.empty((K + Wm, n), dtype=vbase.dtype, device=dev)
    for i in range(K + Wm):
        copies[i].copy_(base)
        if vcopies is not None:
            vcopies[i].copy_(vbase)
    dt = {torch.int32: bsps.I32, torch.int64: bsps.I64, torch.float32: bsps.F32}[base.dtype]
    prm = bsps.make_params(p, s, variant, 1, bucketing, route, leaves)
    ws = torch.empty(bsps.workspace_bytes(n, dt, vbase is not None, prm), dtype=torch.uint8, device=dev)

    def run(i):
        bsps.sort_(copies[i], p, s, variant, values=None if vcopies is None else vcopies[i], bucketing=bucketing,
                   route=route, leaves=leaves, workspace=ws)

    for i in range(Wm):
        run(i)
    torch.cuda.synchronize()
    if timer:
        timer.start()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        run(Wm + i)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stages = timer.stop(K) if timer else {}
    out = copies[Wm + K - 1].clone()
    vout = None if vcopies is None else vcopies[Wm + K - 1].clone()
    del copies, vcopies, ws
    torch.cuda.empty_cache()
    return (t1 - t0) * 1e3 / K, stages, out, vout


def order_u32(torch, t):
    """Order-preserving unsigned image of int32 / float32 keys (int64 for
    comparison on the device), used only to check that outputs are sorted."""
    if t.dtype == torch.float32:
        b = t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        neg = b >= (1 << 31)
        return torch.where(neg, 0xFFFFFFFF - b, b + (1 << 31))
    return t.to(torch.int64)


def is_sorted(torch, t):
    u = order_u32(torch, t)
    return bool(torch.all(u[1:] >= u[:-1]).item())


def bench_c0(bsps, torch, W, args, timer):
    n, p, s = 1 << args.log2n, 256, 64
    log(f"c0: generating 2^{args.log2n} int32 keys")
    base = to_dev(torch, W.int32_keys(n, p, "uniform"))
    res = {}
    for variant, name in ((bsps.DET, "det"), (bsps.RAN, "ran")):
        ms, stages, out, _ = time_sort(bsps, torch, base, args.steps, args.warmup, p, s, variant, timer=timer)
        ok = is_sorted(torch, out)
        res[name] = {"ms": ms, "keys_per_s": n / (ms / 1e3), "sorted": ok, "stages": stages}
        log(f"c0 {name}: {ms:.3f} ms/step, {n / ms / 1e6:.2f} Gkeys/s, sorted={ok}")
    # attainable bandwidth: the library's reference copy kernel on the same
    # 2^28-key array, HIP events on the stream it runs on
    dst = torch.empty_like(base)
    for _ in range(3):
        bsps.stream_copy(base, dst)
    reps = 10
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        bsps.stream_copy(base, dst)
    e1.record()
    e1.synchronize()
    cms = e0.elapsed_time(e1) / reps
    cbytes = 2 * base.numel() * base.element_size()
    ok = bool(torch.equal(dst, base))
    res["stream_copy"] = {"ms": cms, "gbs": cbytes / (cms / 1e3) / 1e9, "bytes_moved": cbytes, "exact": ok}
    log(f"c0 stream copy: {cms:.3f} ms, {cbytes / cms / 1e6:.0f} GB/s, exact={ok}")
    del dst
    return n, p, s, res


def bench_learned(bsps, torch, W, args, timer):
    n, p, s, L = 1 << args.log2n, 1024, 64, 4096
    log(f"learned: generating 2^{args.log2n} float32 lognormal-mixture keys")
    base = to_dev(torch, W.lognormal_f32(n))
    K, Wm = max(1, min(args.steps, 5)), max(1, min(args.warmup, 2))
    out = {"workload": f"2^{args.log2n} float32, mixture of 3 lognormals with 1024 -0.0 and 1024 +0.0, "
                       f"p={p}, s={s}, Sort_Det_BSP, leaves={L}", "steps": K}
    ref = None
    for name, bucketing, route in (("fused", bsps.SPLITTER, bsps.ROUTE_FUSED),
                                   ("scatter_splitter", bsps.SPLITTER, bsps.ROUTE_SCATTER),
                                   ("scatter_learned", bsps.LEARNED, bsps.ROUTE_SCATTER)):
        ms, stages, o, _ = time_sort(bsps, torch, base, K, Wm, p, s, bsps.DET, bucketing, route, L, timer=timer)
        same = True if ref is None else bool(torch.equal(o.view(torch.int32), ref.view(torch.int32)))
        if ref is None:
            ref = o
        e = {"ms": ms, "keys_per_s": n / (ms / 1e3), "sorted": is_sorted(torch, o), "identical_output": same,
             "stages": stages}
        if "k_rank" in stages:
            e["rank_kernel_keys_per_s"] = n / (stages["k_rank"]["ms_per_launch"] / 1e3)
        out[name] = e
        log(f"learned/{name}: {ms:.3f} ms, rank {e.get('rank_kernel_keys_per_s', 0) / 1e9:.1f} Gkeys/s, "
            f"identical={same}")
    # misprediction statistics of one diagnostic run (outside the timed region)
    t = base.clone()
    st = bsps.sort_(t, p, s, bsps.DET, bucketing=bsps.LEARNED, route=bsps.ROUTE_SCATTER, leaves=L, stats=True)
    out["mispredict_rate"] = st["mispredict_rate"]
    out["mean_fix_dist"] = st["mean_fix_dist"]
    out["max_bucket_ratio"] = st["max_bucket_ratio"]
    sl, ss = out["scatter_learned"], out["scatter_splitter"]
    out["learned_speedup_rank_kernel"] = sl.get("rank_kernel_keys_per_s", 0) / max(ss.get("rank_kernel_keys_per_s", 1), 1)
    out["learned_speedup_end_to_end"] = sl["keys_per_s"] / ss["keys_per_s"]
    return out


def bench_int64_kv(bsps, torch, W, args, timer):
    n, p, s = 1 << args.log2n, 256, 64
    log(f"int64_kv: generating 2^{args.log2n} Zipf int64 keys with payload")
    k, v = W.zipf_int64_kv(n)
    base = to_dev(torch, k)
    vbase = to_dev(torch, v.view("int32"))
    K, Wm = max(1, min(args.steps, 5)), max(1, min(args.warmup, 2))
    ms, stages, o, vo = time_sort(bsps, torch, base, K, Wm, p, s, bsps.DET, vbase=vbase, timer=timer)
    ok = is_sorted(torch, o) and bool(torch.equal(base[vo.to(torch.int64) & 0xFFFFFFFF], o))
    log(f"int64_kv: {ms:.3f} ms, {n / ms / 1e6:.2f} Gkeys/s, ok={ok}")
    return {"workload": f"2^{args.log2n} int64 Zipf(1.2) over 2^16 values + 25% equal block, uint32 payload, "
                        f"p={p}, s={s}, Sort_Det_BSP", "ms": ms, "keys_per_s": n / (ms / 1e3),
            "sorted_and_payload_consistent": ok, "steps": K, "stages": stages,
            "floor_fraction_6w": 6 * 12 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}


def bench_segmented(bsps, torch, W, args):
    """The batch with the package's size-class table, learned bucketing on the
    segments above 2^16 keys (as the table says) and, for comparison, with
    splitter search everywhere."""
    import numpy as np
    log("segmented: generating 4096 segments")
    sizes = W.segment_sizes(4096, 8, 20)
    keys, offs = W.segmented_int32(sizes)
    n = keys.size
    base = to_dev(torch, keys)
    K, Wm = max(1, min(args.steps, 5)), max(1, min(args.warmup, 2))
    copies = torch.empty((K + Wm, n), dtype=torch.int32, device="cuda:0")
    table = json.loads(bsps.default_tuning() or json.dumps(
        {"classes": [{"max_log2": 14, "block": 16384, "s": 1}, {"max_log2": 17, "block": 16384, "s": 32},
                     {"max_log2": 20, "block": 16384, "s": 16}, {"max_log2": 40, "block": 16384, "s": 8}]}))
    inner = torch.from_numpy(np.asarray(offs[1:-1], dtype=np.int64)).to("cuda:0")
    cut = torch.zeros(n, dtype=torch.bool, device="cuda:0")
    cut[inner[(inner > 0) & (inner < n)]] = True
    res = {"workload": f"4096 int32 segments, log-uniform sizes in [2^8, 2^20], {n} keys; even segments "
                       "uniform, odd 2^8-distinct", "steps": K, "tuning": table}
    for name, lg in (("learned", 16), ("splitter", 40)):
        tj = json.dumps(dict(table, learned_above_log2=lg))
        for i in range(K + Wm):
            copies[i].copy_(base)
        ws = torch.empty(bsps.segmented_workspace_bytes(offs, bsps.I32, False, tj), dtype=torch.uint8,
                         device="cuda:0")
        for i in range(Wm):
            bsps.sort_segmented_(copies[i], offs, tuning=tj, workspace=ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(K):
            bsps.sort_segmented_(copies[Wm + i], offs, tuning=tj, workspace=ws)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / K
        out = copies[Wm + K - 1]
        ok = not bool(((out[1:] < out[:-1]) & ~cut[1:]).any().item())
        st = bsps.sort_segmented_(copies[0].copy_(base), offs, tuning=tj, workspace=ws, stats=True)
        e = {"ms": ms, "keys_per_s": n / (ms / 1e3), "segments_sorted": ok, "graph": st["graph"],
             "blocks": st["blocks"], "merged_segments": st["merged_segments"],
             "learned_segments": st["learned_segments"], "mispredict_rate": st["mispredict_rate"],
             "floor_fraction_6w": 6 * 4 * n / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
        res[name] = e
        log(f"segmented/{name}: {ms:.3f} ms, {n / ms / 1e6:.2f} Gkeys/s, sorted={ok}, "
            f"learned segments {e['learned_segments']}, mispredict {e['mispredict_rate']:.4f}")
        del ws
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--cpu-log2n", type=int, default=25)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", default=",".join(ALL))
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures a single GPU: the library has no multi-GPU path (the p virtual "
              "processors live on one GPU); run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    only = set(args.only.split(","))
    if not only <= set(ALL) or "c0" not in only:
        print(f"--only takes a subset of {ALL} that includes c0", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1408_6729_amd as bsps
    import workloads as W

    timer = Timer(bsps)
    n, p, s, c0 = bench_c0(bsps, torch, W, args, timer)
    det = c0["det"]
    detail = {"det": det, "ran": c0["ran"], "stream_copy": c0["stream_copy"]}
    if "learned" in only:
        detail["learned_vs_splitter"] = bench_learned(bsps, torch, W, args, timer)
    if "int64_kv" in only:
        detail["int64_kv"] = bench_int64_kv(bsps, torch, W, args, timer)
    if "segmented" in only:
        detail["segmented"] = bench_segmented(bsps, torch, W, args)

    # dominant kernel of the timed DET steps: a permuting pass reads and writes
    # every key once, 2 * 4 bytes per int32 key
    cand = {k: v for k, v in det["stages"].items() if k in ("tile_sort", "k_mwm_merge(block)", "k_mwm_merge(bucket)")}
    dom = max(cand, key=lambda k: cand[k]["ms_per_launch"] * cand[k]["launches_per_step"])
    alg_bytes = 2 * 4 * n
    achieved = alg_bytes / (cand[dom]["ms_per_launch"] / 1e3) / 1e9
    workload = "C0"
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(dom, workload), "kernel": dom,
                "alg_bytes_per_launch": alg_bytes, "attainable_copy_gbs": c0["stream_copy"]["gbs"],
                "frac_of_attainable": achieved / c0["stream_copy"]["gbs"]}
    detail["floor_fraction_6w"] = (6 * 4 * n) / (det["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS
    detail["floor_note"] = "6 * 4 bytes per key (three permuting passes) / time / 8 TB/s"
    cpu = None
    if not args.no_cpu:
        log(f"timing the CPU oracle on 2^{args.cpu_log2n} keys")
        cpu = cpu_baseline(args.cpu_log2n, p, s)
    line = {
        "metric": "keys/s and % HBM roofline, 2^28 int32; learned vs splitter bucketing",
        "value": det["keys_per_s"], "unit": "keys/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": det["ms"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{workload}: 2^{args.log2n} int32 keys uniform in [0,2^31), p={p}, s={s}, "
                               "Sort_Det_BSP, keys only, fused routing",
                   "n": n, "p": p, "s": s, "variant": "DET", "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
