#!/usr/bin/env python3
"""Benchmark of the BSP sample sort on one MI355X.

Headline workload: 2^28 int32 keys uniform in [0, 2^31), drawn per virtual
processor with the paper's seeding (Section 6.3), p = 256 virtual processors,
oversampling s = 64, the deterministic variant Sort_Det_BSP (Figure SortD),
keys only. One step = one complete sort of one staged copy of the input
(local block sort, sample, splitters, bucket boundaries, prefix sums,
per-bucket merge), with the input already resident in HBM: before every step
the pristine input is copied into the work buffer outside the timed region,
and the step itself is timed with HIP events on the stream the sort runs on.
The reported time is the median over the timed steps (min and max beside it).
The randomized variant (Figure SortRI) is timed on the same input.

Beside it (in "detail"), each timed the same way:
  configs      2^20 int32 uniform keys at p = 16, s = 8, and the seven
               synthetic distributions at 2^26 int32 keys, p = 128, s = 32,
               both variants
  variants     the same input sorted by Sort_Ran_BSP (Figure SortR), by the
               iterative Sort_Det_BSP (m = 2, 4, 8 rounds, Section 5.1), and
               with the duplicate handling switched off (Section 6.4), the
               latter also on 2^28 keys over 2^10 distinct values
  learned      2^28 float32 keys (mixture of three lognormals), p = 1024,
               s = 64: per-key ranking by the learned CDF model against plain
               splitter search on the scatter route and in Sort_Ran_BSP's
               ranking of the unsorted input, and the fused route; identical
               outputs required
  int64_kv     2^28 int64 keys, Zipf(1.2) over 2^16 values + 25% equal block,
               uint32 payload, p = 256, s = 64, DET and RAN
  segmented    4096 int32 segments, log-uniform sizes in [2^8, 2^20], one
               graph launch per step (the cached graph of one fixed buffer)
  operating    the paper's own oversampling (Section 6.1) on the mid-size
               workload: 2^26 int32 keys, p = 128, DET s = ceil(lg lg n) p and
               RAN s = 2 ceil(lg n)^2, with the largest bucket over n/p
Per-stage times come from one extra, separately run sort with the library's
stage timer on (HIP events between the stages), never from the timed steps.

Prints one JSON line: throughput in keys/s, the roofline of the dominant
kernel (algorithmic bytes of one launch over its HIP-event-timed duration,
against the 8 TB/s HBM peak and against the rate the library's reference copy
kernel attains on the same array), and the CPU oracle timed on the host cores.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--only c0,configs,variants,learned,int64_kv,segmented,operating]
"""
from __future__ import annotations

import argparse
import ctypes as ct
import glob
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STAGES = ["tile_sort", "block_merge", "sample_splitters", "bucket_ranking", "prefix_routing",
          "bucket_merge", "k_mwm_merge(block)", "k_mwm_merge(bucket)", "k_rank", "k_lsd_sweep"]
# kernels that move every record once per launch (a permuting pass: 2 w bytes per key)
PERMUTING = ("tile_sort", "k_lsd_sweep", "k_mwm_merge(block)", "k_mwm_merge(bucket)")
ALL = ("c0", "configs", "variants", "learned", "int64_kv", "segmented", "operating")


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


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return "unknown"


def cpu_baseline(keys, p: int, s: int, log2_one: int):
    """The oracle (plain C) on the host cores: its per-processor steps on all
    the cores this process may use (at most 16, the CPU share of one GPU) for
    the full headline input, and on one core for a bounded prefix sample."""
    import oracle
    import workloads as W
    threads = oracle.default_threads()
    n = keys.size
    t0 = time.perf_counter()
    oracle.sort(keys, p, s, oracle.DET, intermediates=False, threads=threads)
    dt_all = time.perf_counter() - t0
    n1 = 1 << log2_one
    k1 = W.int32_keys(n1, p, "uniform")
    t0 = time.perf_counter()
    oracle.sort(k1, p, s, oracle.DET, intermediates=False)
    dt_one = time.perf_counter() - t0
    return {"value": n / dt_all, "unit": "keys/s", "cores": threads, "kind": "oracle",
            "sample": f"the full headline input (2^{int(math.log2(n))} int32 keys, p={p}, s={s}, DET) with the "
                      f"oracle's per-processor steps on {threads} host threads: {dt_all:.1f} s",
            "one_core": {"value": n1 / dt_one, "unit": "keys/s", "cores": 1,
                         "sample": f"2^{log2_one} int32 uniform keys, p={p}, s={s}, DET, one thread: {dt_one:.1f} s"},
            "host_cpu": cpu_model(), "host_cpu_count": os.cpu_count()}


def cpu_configs(W, threads):
    """The oracle (threaded per-processor steps, as in cpu_baseline) on the
    parity configurations, for the comparison table: 2^20 int32 (p = 16, s =
    8), 2^26 int32 uniform (p = 128, s = 32), 2^28 int64 Zipf key-value (p =
    256, s = 64) and 2^28 float32 lognormal mixture (p = 1024, s = 64), DET.
    Seconds of the sort call only (inputs generated before)."""
    import oracle
    out = {}
    cases = [("C1", lambda: (W.int32_keys(1 << 20, 16, "uniform"), None), 16, 8),
             ("C2_uniform", lambda: (W.int32_keys(1 << 26, 128, "uniform"), None), 128, 32),
             ("C3", lambda: W.zipf_int64_kv(1 << 28), 256, 64),
             ("C4", lambda: (W.lognormal_f32(1 << 28), None), 1024, 64)]
    for name, gen, p, s in cases:
        keys, vals = gen()
        t0 = time.perf_counter()
        oracle.sort(keys, p, s, oracle.DET, values=vals, intermediates=False, threads=threads)
        dt = time.perf_counter() - t0
        out[name] = {"keys_per_s": keys.size / dt, "seconds": dt, "threads": threads, "n": int(keys.size)}
        log(f"cpu oracle {name}: {dt:.2f} s, {keys.size / dt / 1e6:.1f} Mkeys/s on {threads} threads")
        del keys, vals
    return out


def to_dev(torch, a):
    """Host array -> cuda:0 through a pinned (hipHostMalloc) buffer."""
    h = torch.from_numpy(a)
    pin = torch.empty(h.shape, dtype=h.dtype, pin_memory=True)
    pin.copy_(h)
    return pin.to("cuda:0")


def stage_times(bsps, run, restage, torch):
    """One extra run with the library's stage timer on (HIP events recorded
    between the stages on the sort's stream): per-stage ms and launches."""
    ms = (ct.c_double * len(STAGES))()
    cnt = (ct.c_int64 * len(STAGES))()
    restage()
    torch.cuda.synchronize()
    bsps.lib.bsps_timing_read(ms, cnt, len(STAGES), 1)
    bsps.lib.bsps_timing(1)
    run()
    torch.cuda.synchronize()
    bsps.lib.bsps_timing(0)
    bsps.lib.bsps_timing_read(ms, cnt, len(STAGES), 1)
    return {STAGES[i]: {"ms_per_launch": ms[i] / cnt[i], "launches_per_step": int(cnt[i])}
            for i in range(len(STAGES)) if cnt[i]}


def time_steps(torch, run, restage, K, Wm):
    """Wm untimed steps, then K timed ones; before each step the input is
    restaged (untimed), and the step is bracketed by synchronizations and
    timed with HIP events on the current stream. Returns per-step ms."""
    for _ in range(Wm):
        restage()
        run()
    torch.cuda.synchronize()
    out = []
    for _ in range(K):
        restage()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1))
    return out


def summary(ts, n):
    ts = sorted(ts)
    med = ts[len(ts) // 2] if len(ts) % 2 else 0.5 * (ts[len(ts) // 2 - 1] + ts[len(ts) // 2])
    return {"ms": med, "ms_min": ts[0], "ms_max": ts[-1], "steps": len(ts), "keys_per_s": n / (med / 1e3)}


def bench_sort(bsps, torch, base, K, Wm, p, s, variant=0, bucketing=0, route=0, leaves=0, vbase=None, untagged=False,
               rounds=1, local_sort=0):
    """K timed sorts of the staged input (median); then one stage-timed run."""
    n = base.numel()
    work = torch.empty_like(base)
    vwork = None if vbase is None else torch.empty_like(vbase)
    dt = {torch.int32: bsps.I32, torch.int64: bsps.I64, torch.float32: bsps.F32}[base.dtype]
    prm = bsps.make_params(p, s, variant, 1, bucketing, route, leaves, local_sort=local_sort, untagged=untagged,
                           rounds=rounds)
    ws = torch.empty(bsps.workspace_bytes(n, dt, vbase is not None, prm), dtype=torch.uint8, device=base.device)

    def restage():
        work.copy_(base)
        if vwork is not None:
            vwork.copy_(vbase)

    def run():
        bsps.sort_(work, p, s, variant, values=vwork, bucketing=bucketing, route=route, leaves=leaves, workspace=ws,
                   untagged=untagged, rounds=rounds, local_sort=local_sort)

    ts = time_steps(torch, run, restage, K, Wm)
    res = summary(ts, n)
    res["stages"] = stage_times(bsps, run, restage, torch)
    del ws
    return res, work, vwork


def order_u32(torch, t):
    """Order-preserving image of int32 / float32 keys as int64 (device), used
    only to check that outputs are sorted."""
    if t.dtype == torch.float32:
        b = t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        neg = b >= (1 << 31)
        return torch.where(neg, 0xFFFFFFFF - b, b + (1 << 31))
    return t.to(torch.int64)


def is_sorted(torch, t):
    u = order_u32(torch, t)
    return bool(torch.all(u[1:] >= u[:-1]).item())


def bench_c0(bsps, torch, W, args, keys):
    n, p, s = keys.size, 256, 64
    base = to_dev(torch, keys)
    res = {}
    for variant, name in ((bsps.DET, "det"), (bsps.RAN, "ran")):
        r, out, _ = bench_sort(bsps, torch, base, args.steps, args.warmup, p, s, variant)
        r["sorted"] = is_sorted(torch, out)
        res[name] = r
        del out
        log(f"c0 {name}: median {r['ms']:.3f} ms (min {r['ms_min']:.3f}, max {r['ms_max']:.3f}), "
            f"{r['keys_per_s'] / 1e9:.2f} Gkeys/s, sorted={r['sorted']}")
    # attainable bandwidth: the library's reference copy kernel on the same
    # array, HIP events on the stream it runs on
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
    del dst, base
    torch.cuda.empty_cache()
    return n, p, s, res


def bench_configs(bsps, torch, W, args):
    """The small and mid-size parity configurations, timed the same way: 2^20
    int32 uniform keys at p = 16, s = 8 (DET), and the seven distributions at
    2^26 int32 keys, p = 128, s = 32, DET and RAN."""
    out = {}
    K, Wm = max(5, min(args.steps, 10)), max(1, min(args.warmup, 2))
    base = to_dev(torch, W.int32_keys(1 << 20, 16, "uniform"))
    r, o, _ = bench_sort(bsps, torch, base, K, Wm, 16, 8, bsps.DET)
    r["sorted"] = is_sorted(torch, o)
    del r["stages"]
    out["C1_det"] = r
    log(f"configs/C1 det: median {r['ms']:.3f} ms, {r['keys_per_s'] / 1e9:.2f} Gkeys/s, sorted={r['sorted']}")
    del base, o
    for dist in W.DISTRIBUTIONS:
        base = to_dev(torch, W.int32_keys(1 << 26, 128, dist))
        for variant, vname in ((bsps.DET, "det"), (bsps.RAN, "ran")):
            r, o, _ = bench_sort(bsps, torch, base, K, Wm, 128, 32, variant)
            r["sorted"] = is_sorted(torch, o)
            del r["stages"]
            out[f"C2_{dist}_{vname}"] = r
            log(f"configs/C2 {dist} {vname}: median {r['ms']:.3f} ms, {r['keys_per_s'] / 1e9:.2f} Gkeys/s, "
                f"sorted={r['sorted']}")
            del o
        del base
    torch.cuda.empty_cache()
    return out


def bench_variants(bsps, torch, W, args, keys):
    """On the headline input (2^28 int32 uniform, p = 256, s = 64): the
    Sort_Ran_BSP ordering (Figure SortR), the iterative Sort_Det_BSP with m =
    2, 4 and 8 rounds (k = 16, 4, 2 buckets per round, Section 5.1), the
    duplicate handling switched off (Section 6.4's ablation) next to it on
    the headline input and on 2^28 keys over 2^10 distinct values, and the
    LSD local sort in place of tiles + merge."""
    n, p, s = keys.size, 256, 64
    base = to_dev(torch, keys)
    K, Wm = max(5, min(args.steps, 10)), max(1, min(args.warmup, 2))
    out = {"workload": f"2^{int(math.log2(n))} int32 uniform, p={p}, s={s}"}
    runs = [("sr", dict(variant=bsps.RAN_SR)), ("iter_m2", dict(rounds=2)), ("iter_m4", dict(rounds=4)),
            ("iter_m8", dict(rounds=8)), ("untagged", dict(untagged=True)),
            ("lsd_local_sort", dict(local_sort=bsps.LOCAL_LSD))]
    for name, kw in runs:
        r, o, _ = bench_sort(bsps, torch, base, K, Wm, p, s, **kw)
        r["sorted"] = is_sorted(torch, o)
        out[name] = r
        del o
        log(f"variants/{name}: median {r['ms']:.3f} ms [{r['ms_min']:.3f}, {r['ms_max']:.3f}], "
            f"{n / r['ms'] / 1e6:.2f} Gkeys/s, sorted={r['sorted']}")
    del base
    dk = to_dev(torch, W.int32_keys(n, p, "dict1024"))
    for name, kw in (("dict1024_tagged", {}), ("dict1024_untagged", dict(untagged=True))):
        r, o, _ = bench_sort(bsps, torch, dk, K, Wm, p, s, **kw)
        r["sorted"] = is_sorted(torch, o)
        t = dk.clone()
        r["max_bucket_ratio"] = bsps.sort_(t, p, s, stats=True, untagged=kw.get("untagged", False))["max_bucket_ratio"]
        out[name] = r
        del o, t
        log(f"variants/{name}: median {r['ms']:.3f} ms, largest bucket {r['max_bucket_ratio']:.3f} n/p")
    del dk
    torch.cuda.empty_cache()
    return out


def bench_learned(bsps, torch, W, args):
    n, p, s, L = 1 << args.log2n, 1024, 64, 4096
    log(f"learned: generating 2^{args.log2n} float32 lognormal-mixture keys")
    base = to_dev(torch, W.lognormal_f32(n))
    K, Wm = max(20, args.steps), max(2, args.warmup)
    out = {"workload": f"2^{args.log2n} float32, mixture of 3 lognormals with 1024 -0.0 and 1024 +0.0, "
                       f"p={p}, s={s}, leaves={L}"}
    for variant, vname in ((bsps.DET, "det"), (bsps.RAN, "ran"), (bsps.RAN_SR, "sr")):
        ref = None
        e_all = {}
        for name, bucketing, route in (("fused", bsps.SPLITTER, bsps.ROUTE_FUSED),
                                       ("scatter_splitter", bsps.SPLITTER, bsps.ROUTE_SCATTER),
                                       ("scatter_learned", bsps.LEARNED, bsps.ROUTE_SCATTER),
                                       ("sr_splitter", bsps.SPLITTER, bsps.ROUTE_FUSED),
                                       ("sr_learned", bsps.LEARNED, bsps.ROUTE_FUSED)):
            if (variant == bsps.RAN_SR) != name.startswith("sr_"):
                continue
            if variant == bsps.RAN and name == "scatter_splitter":
                continue
            r, o, _ = bench_sort(bsps, torch, base, K, Wm, p, s, variant, bucketing, route, L)
            same = True if ref is None else bool(torch.equal(o.view(torch.int32), ref.view(torch.int32)))
            if ref is None:
                ref = o.clone()
            r["sorted"] = is_sorted(torch, o)
            r["identical_output"] = same
            if "k_rank" in r["stages"]:
                r["rank_kernel_keys_per_s"] = n / (r["stages"]["k_rank"]["ms_per_launch"] / 1e3)
            e_all[name] = r
            del o
            log(f"learned/{vname}/{name}: median {r['ms']:.3f} ms [{r['ms_min']:.3f}, {r['ms_max']:.3f}], "
                f"rank {r.get('rank_kernel_keys_per_s', 0) / 1e9:.1f} Gkeys/s, identical={same}")
        # misprediction statistics of one diagnostic run (outside the timed region)
        t = base.clone()
        st = bsps.sort_(t, p, s, variant, bucketing=bsps.LEARNED,
                        route=bsps.ROUTE_FUSED if variant == bsps.RAN_SR else bsps.ROUTE_SCATTER, leaves=L, stats=True)
        e_all["mispredict_rate"] = st["mispredict_rate"]
        e_all["mean_fix_dist"] = st["mean_fix_dist"]
        e_all["max_bucket_ratio"] = st["max_bucket_ratio"]
        del t, ref
        pair = (("scatter_learned", "scatter_splitter") if "scatter_splitter" in e_all else
                ("sr_learned", "sr_splitter") if "sr_splitter" in e_all else None)
        if pair:
            sl, ss = e_all[pair[0]], e_all[pair[1]]
            e_all["learned_speedup_rank_kernel"] = (sl.get("rank_kernel_keys_per_s", 0) /
                                                    max(ss.get("rank_kernel_keys_per_s", 1), 1))
            e_all["learned_speedup_end_to_end"] = ss["ms"] / sl["ms"]
            # the spread of the timed steps: learned wins beyond it when its
            # slowest step beats the splitter route's fastest
            e_all["learned_faster_than_spread"] = sl["ms_max"] < ss["ms_min"]
        out[vname] = e_all
    torch.cuda.empty_cache()
    return out


def bench_int64_kv(bsps, torch, W, args):
    n, p, s = 1 << args.log2n, 256, 64
    log(f"int64_kv: generating 2^{args.log2n} Zipf int64 keys with payload")
    k, v = W.zipf_int64_kv(n)
    base = to_dev(torch, k)
    vbase = to_dev(torch, v.view("int32"))
    K, Wm = max(5, min(args.steps, 10)), max(1, min(args.warmup, 2))
    out = {"workload": f"2^{args.log2n} int64 Zipf(1.2) over 2^16 values + 25% equal block, uint32 payload, "
                       f"p={p}, s={s}"}
    for variant, vname in ((bsps.DET, "det"), (bsps.RAN, "ran")):
        r, o, vo = bench_sort(bsps, torch, base, K, Wm, p, s, variant, vbase=vbase)
        ok = is_sorted(torch, o) and bool(torch.equal(base[vo.to(torch.int64) & 0xFFFFFFFF], o))
        r["sorted_and_payload_consistent"] = ok
        r["floor_fraction_6w"] = 6 * 12 * n / (r["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS
        out[vname] = r
        del o, vo
        log(f"int64_kv/{vname}: median {r['ms']:.3f} ms, {n / r['ms'] / 1e6:.2f} Gkeys/s, ok={ok}")
    del base, vbase
    torch.cuda.empty_cache()
    return out


def bench_segmented(bsps, torch, W, args):
    """The batch with the package's size-class table, timed as repeated sorts
    of one fixed buffer (its graph is captured once and then replayed from the
    cache), learned bucketing on the large segments as the table says and,
    for comparison, with splitter search everywhere."""
    import numpy as np
    log("segmented: generating 4096 segments")
    sizes = W.segment_sizes(4096, 8, 20)
    keys, offs = W.segmented_int32(sizes)
    n = keys.size
    base = to_dev(torch, keys)
    work = torch.empty_like(base)
    K, Wm = max(10, args.steps), max(2, args.warmup)
    table = json.loads(bsps.default_tuning() or json.dumps(
        {"classes": [{"max_log2": 14, "block": 16384, "s": 1}, {"max_log2": 17, "block": 16384, "s": 32},
                     {"max_log2": 20, "block": 16384, "s": 16}, {"max_log2": 40, "block": 16384, "s": 8}]}))
    inner = torch.from_numpy(np.asarray(offs[1:-1], dtype=np.int64)).to("cuda:0")
    cut = torch.zeros(n, dtype=torch.bool, device="cuda:0")
    cut[inner[(inner > 0) & (inner < n)]] = True
    res = {"workload": f"4096 int32 segments, log-uniform sizes in [2^8, 2^20], {n} keys; even segments "
                       "uniform, odd 2^8-distinct", "tuning": table}
    default_lg = int(table.get("learned_above_log2", 16))
    for name, lg in (("default_table", default_lg), ("learned", 16), ("splitter", 40)):
        tj = json.dumps(dict(table, learned_above_log2=lg))
        ws = torch.empty(bsps.segmented_workspace_bytes(offs, bsps.I32, False, tj), dtype=torch.uint8,
                         device="cuda:0")

        def restage():
            work.copy_(base)

        def run():
            bsps.sort_segmented_(work, offs, tuning=tj, workspace=ws)

        ts = time_steps(torch, run, restage, K, Wm)
        e = summary(ts, n)
        ok = not bool(((work[1:] < work[:-1]) & ~cut[1:]).any().item())
        restage()
        st = bsps.sort_segmented_(work, offs, tuning=tj, workspace=ws, stats=True)
        e.update({"segments_sorted": ok, "graph_replayed_from_cache": st["graph_cached"], "blocks": st["blocks"],
                  "merged_segments": st["merged_segments"], "learned_segments": st["learned_segments"],
                  "learned_above_log2": lg, "mispredict_rate": st["mispredict_rate"],
                  "floor_fraction_6w": 6 * 4 * n / (e["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS})
        res[name] = e
        log(f"segmented/{name}: median {e['ms']:.3f} ms [{e['ms_min']:.3f}, {e['ms_max']:.3f}], "
            f"{n / e['ms'] / 1e6:.2f} Gkeys/s, sorted={ok}, cached graph={st['graph_cached']}")
        del ws
    del base, work, cut
    torch.cuda.empty_cache()
    return res


def bench_operating(bsps, torch, W, args):
    """Section 6.1's oversampling on the mid-size uniform workload: DET
    s = ceil(lg lg n) p, RAN s = 2 ceil(lg n)^2; the largest bucket over n/p
    against the paper's observed imbalance (below 15%, Section 6.4)."""
    n, p = 1 << 26, 128
    lg = math.log2(n)
    s_det = math.ceil(math.log2(lg)) * p
    s_ran = 2 * math.ceil(lg) ** 2
    keys = W.int32_keys(n, p, "uniform")
    base = to_dev(torch, keys)
    out = {"workload": f"2^26 int32 uniform, p={p}", "s_det": s_det, "s_ran": s_ran}
    for variant, vname, s in ((bsps.DET, "det", s_det), (bsps.RAN, "ran", s_ran)):
        r, o, _ = bench_sort(bsps, torch, base, max(5, min(args.steps, 10)), 1, p, s, variant)
        r["sorted"] = is_sorted(torch, o)
        t = base.clone()
        st = bsps.sort_(t, p, s, variant, seed=1, stats=True)
        r["max_bucket_ratio"] = st["max_bucket_ratio"]
        out[vname] = r
        del o, t
        log(f"operating/{vname} s={s}: median {r['ms']:.3f} ms, largest bucket {st['max_bucket_ratio']:.3f} n/p")
    del base
    torch.cuda.empty_cache()
    return out


def dominant(stages):
    """The permuting kernel with the largest total time per step."""
    cand = {k: v for k, v in stages.items() if k in PERMUTING and not (
        k == "tile_sort" and "k_lsd_sweep" in stages)}
    return max(cand, key=lambda k: cand[k]["ms_per_launch"] * cand[k]["launches_per_step"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--cpu-log2n", type=int, default=25)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="also time the oracle on the parity configurations (about two minutes)")
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

    log(f"c0: generating 2^{args.log2n} int32 keys")
    keys = W.int32_keys(1 << args.log2n, 256, "uniform")
    n, p, s, c0 = bench_c0(bsps, torch, W, args, keys)
    det = c0["det"]
    detail = {"det": det, "ran": c0["ran"], "stream_copy": c0["stream_copy"]}
    if "configs" in only:
        detail["configs"] = bench_configs(bsps, torch, W, args)
    if "variants" in only:
        detail["variants"] = bench_variants(bsps, torch, W, args, keys)
    if "learned" in only:
        detail["learned_vs_splitter"] = bench_learned(bsps, torch, W, args)
    if "int64_kv" in only:
        detail["int64_kv"] = bench_int64_kv(bsps, torch, W, args)
    if "segmented" in only:
        detail["segmented"] = bench_segmented(bsps, torch, W, args)
    if "operating" in only:
        detail["paper_operating_point"] = bench_operating(bsps, torch, W, args)

    # dominant kernel of the headline sort: a permuting pass reads and writes
    # every key once, 2 * 4 bytes per int32 key
    dom = dominant(det["stages"])
    alg_bytes = 2 * 4 * n
    achieved = alg_bytes / (det["stages"][dom]["ms_per_launch"] / 1e3) / 1e9
    workload = "C0"
    passes = sum(det["stages"][k]["launches_per_step"] for k in det["stages"] if k in PERMUTING and not (
        k == "tile_sort" and "k_lsd_sweep" in det["stages"]))
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(dom, workload), "kernel": dom,
                "alg_bytes_per_launch": alg_bytes, "attainable_copy_gbs": c0["stream_copy"]["gbs"],
                "frac_of_attainable": achieved / c0["stream_copy"]["gbs"],
                "pipeline": {"permuting_passes": passes,
                             "frac": passes * alg_bytes / (det["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS,
                             "floor_frac_6w": 6 * 4 * n / (det["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS}}
    cpu = None
    if not args.no_cpu:
        log(f"timing the CPU oracle on the headline input and on 2^{args.cpu_log2n} keys")
        cpu = cpu_baseline(keys, p, s, args.cpu_log2n)
        if args.cpu_configs:
            import oracle
            cpu["configs"] = cpu_configs(W, oracle.default_threads())
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
