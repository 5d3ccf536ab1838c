"""Benchmark: the vectorized Quicksort on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--n N]

A step is one complete sort (every level of partitions, the per-workgroup finish
and the in-LDS base cases) of one array of synthetic keys.  Every timed step sorts
its own pre-staged copy of the input, so all inputs are resident in HBM when the
timed region starts and nothing but sorting is timed.  Prints one JSON line.

The line also carries "learned_vs_plain": the 5e8-key lognormal-mixture workload
sorted by both methods (median of a few sorts each), the speedup of the learned
256-bucket splitter, whether both outputs are identical and the bucket balance of
the trained model against the same model untrained; and "batched": the
65,536-segment u32 batch sorted by one hipGraph replay (library defaults and the
autotuner's choice) against one vqs_sort call per segment; and "inplace": the same
input sorted in place (the paper's in-place partition order, no key scratch), its
time, key traffic and workspace against the default path's.

Roofline: the dominant kernel is the device-wide partition (level kernel).  Its
algorithmic traffic per launch is 2 * keys * key_size bytes (each key of the level
read once and written once); HIP events around each level launch of the timed
steps, on the library's stream, give the durations (only those launches are
recorded there, which costs the timed steps little; two more sorts after them, with
every launch recorded, give the solo and total kernel times).  Besides the 8 TB/s
peak, the bandwidth of a plain device-to-device copy of the input (measured the same
way) is reported as a second denominator ("copy_gbs", "frac_of_copy").  "passes" is
the number of full read+write sweeps over the keys the sort made, from the library's
key-traffic counters (level partitions and copy passes, single-workgroup partitions,
the load and store of every in-LDS sort; partitions inside LDS move no device
memory), and "end_to_end_frac" is passes x 2 x n x key size / step time / peak.

"cpu_baseline" is the CPU oracle on the host's cores (one thread and all threads, on
a sample of the same input), with np.sort and std::sort of that sample as context.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
METRIC = "Gkeys/s & % of HBM roofline, 1e8 u64 sort; learned-splitter vs plain"

WORKLOADS = {
    # name: (key type, default n, generator, description)
    "c2_uniform": (3, 100_000_000, "uniform", "1e8 u64 uniform over [0, 2^64), seed 2, ascending"),
    "c2_zipf": (3, 100_000_000, "zipf", "1e8 u64 Zipf(1.0) over 2^20 values, seed 3"),
    "c2_8distinct": (3, 100_000_000, "8distinct", "1e8 u64, 8 distinct values, seed 4"),
    "c2_sorted": (3, 100_000_000, "sorted", "1e8 u64 uniform, sorted"),
    "c2_reverse": (3, 100_000_000, "reverse", "1e8 u64 uniform, reverse sorted"),
    "c2_almost": (3, 100_000_000, "almost", "1e8 u64 sorted + 1% random pair swaps"),
    "c2_m3killer": (3, 100_000_000, "m3killer", "1e8 u64 median-of-3 killer permutation"),
    "c1_u32": (2, 1_000_000, None, "1e6 u32 uniform, seed 1"),
    "c3_f32_normal": (5, 250_000_000, "f32_normal", "2.5e8 f32 Normal(0,1), seed 7"),
    "c3_f32_exponential": (5, 250_000_000, "f32_exponential", "2.5e8 f32 Exponential(1), seed 8"),
    "c3_f64_uniform": (6, 100_000_000, "f64_uniform", "1e8 f64 uniform [0,1), seed 9"),
    "c3_u16_uniform": (1, 200_000_000, "u16_uniform", "2e8 u16 uniform, seed 10"),
    "c3_u128": (4, 50_000_000, "u128", "5e7 u128, hi over 2^16 values, seed 11"),
    # batched: 65,536 segments with log-uniform lengths in [16, 2^20], one hipGraph
    "c4_u32": (2, 0, "c4", "65,536 segments, lengths log-uniform [16, 2^20] (seed 12), u32 keys (seed 13)"),
    "c4_u64": (3, 0, "c4", "65,536 segments, lengths log-uniform [16, 2^20] (seed 12), u64 keys (seed 14)"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2_uniform", choices=sorted(WORKLOADS))
    ap.add_argument("--n", type=int, default=0, help="override the key count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=30_000_000,
                    help="keys of the CPU baseline's sample (the first keys of the same input)")
    ap.add_argument("--profile-json", default="", help="write per-launch kernel times here")
    ap.add_argument("--learned-n", type=int, default=500_000_000,
                    help="keys of the learned-splitter vs plain comparison (0: skip it)")
    ap.add_argument("--learned-reps", type=int, default=3)
    ap.add_argument("--per-array", action="store_true",
                    help="batched workloads: also time one vqs_sort call per segment")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched workloads: library defaults instead of the autotuner's choice")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 65,536-segment batch record of the default line")
    return ap.parse_args()


def bench_batched(args, kt: int, desc: str) -> None:
    """The 65,536-segment batch: keys generated on the GPU (SplitMix64 by index), the
    autotuner's settings chosen on the whole batch (with --no-tune the library
    defaults, e.g. for a profiled run that should trace only the timed sorts), then
    the whole batch sorted by one vqs_sort_segmented call replaying a hipGraph (total
    key count given, so a replay never waits on the host)."""
    import torch
    from paper_2205_05982_amd import vqs
    from paper_2205_05982_amd import workloads as W
    off = W.segment_offsets(65536, 12)
    n = int(off[-1])
    bits, seed = (32, 13) if kt == 2 else (64, 14)
    dev = torch.device("cuda", 0)
    src = W.counter_torch(seed, 0, n, bits, dev)
    work = torch.empty_like(src)
    o = torch.from_numpy(off).to(dev)
    stream = torch.cuda.current_stream()
    work.copy_(src)
    settings = {}
    if not args.no_tune:
        tuned = vqs.autotune_segmented(work, o, key_type=kt)
        settings = {k: tuned[k] for k in vqs.TUNED_FIELDS}
        print(f"# tuned on the whole batch: {settings}", file=sys.stderr, flush=True)
    times = []
    for r in range(args.warmup + args.steps):
        work.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        vqs.sort_segmented(work, o, key_type=kt, use_graph=1, total_keys=n, **settings)
        e1.record(stream)
        torch.cuda.synchronize()
        if vqs.last_error_bits():
            raise RuntimeError(f"device error bits {vqs.last_error_bits():#x}")
        if r >= args.warmup:
            times.append(e0.elapsed_time(e1))
    ms = float(np.mean(times))
    per_array = None
    if args.per_array:
        work.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(65536):
            vqs.sort(work[int(off[i]):int(off[i + 1])], key_type=kt)
        e1.record(stream)
        torch.cuda.synchronize()
        per_array = {"ms": round(e0.elapsed_time(e1), 1), "calls": 65536,
                     "speedup_of_batch": round(e0.elapsed_time(e1) / ms, 1)}
    ks = bits // 8
    line = {
        "metric": METRIC, "value": round(n / ms / 1e6, 4), "unit": "Gkeys/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": {2: "u32", 3: "u64"}[kt], "data": "synthetic",
        "config": {"workload": desc, "n": n, "segments": 65536, "method": "plain, one hipGraph", "key_bytes": ks,
                   "tuned": settings},
        "per_array_calls": per_array,
    }
    print(json.dumps(line), flush=True)


def batched_record(reps: int = 3, tune_keys: int = 0) -> dict:
    """The 65,536-segment u32 batch (lengths log-uniform in [16, 2^20], 6.1e9 keys):
    the autotuner's choice on a prefix of about tune_keys keys (0: the whole batch; the
    library's default solo threshold grows with the key count, so a threshold chosen on
    a prefix need not suit the whole batch), then the whole batch
    sorted by one hipGraph replay (total key count given, so a replay never waits on
    the host) with the library defaults and with the tuned settings, median of reps
    each, against one vqs_sort call per segment (once)."""
    import torch
    from paper_2205_05982_amd import vqs
    from paper_2205_05982_amd import workloads as W
    off = W.segment_offsets(65536, 12)
    n = int(off[-1])
    dev = torch.device("cuda", 0)
    src = W.counter_torch(13, 0, n, 32, dev)
    work = torch.empty_like(src)
    o = torch.from_numpy(off).to(dev)
    stream = torch.cuda.current_stream()
    work.copy_(src)
    t0 = time.time()
    tuned = vqs.autotune_segmented(work, o, key_type=2, max_keys=tune_keys)
    tune_s = time.time() - t0
    settings = {k: tuned[k] for k in vqs.TUNED_FIELDS}

    def timed(opts):
        ts = []
        for r in range(reps + 1):             # the first call captures the graph
            work.copy_(src)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            vqs.sort_segmented(work, o, key_type=2, use_graph=1, total_keys=n, **opts)
            e1.record(stream)
            torch.cuda.synchronize()
            if vqs.last_error_bits():
                raise RuntimeError(f"device error bits {vqs.last_error_bits():#x}")
            if r:
                ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    ms_default = timed({})
    ms_tuned = timed(settings)
    # the last output: every segment non-decreasing, same multiset
    a = work.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    bad = a[1:] < a[:-1]
    bad[o[1:-1] - 1] = False
    ok = not bool(bad.any().item())
    b = src.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    ok = ok and bool((a.sum() == b.sum()).item())
    del a, b, bad
    work.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(65536):
        vqs.sort(work[int(off[i]):int(off[i + 1])], key_type=2)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_per_array = e0.elapsed_time(e1)
    best = min(ms_default, ms_tuned)
    gbs = lambda ms: round(n * 4 / (ms * 1e-3) / 1e9, 1)
    del src, work
    torch.cuda.empty_cache()
    return {
        "workload": "65,536 u32 segments, lengths log-uniform [16, 2^20] (seed 12), keys seed 13",
        "n": n, "segments": 65536,
        "graph_ms_default": round(ms_default, 2), "graph_ms_tuned": round(ms_tuned, 2),
        "tuned": settings, "tune_prefix_keys": tune_keys or n, "tune_s": round(tune_s, 1),
        "gkeys": round(n / best / 1e6, 2), "gbs": gbs(best),
        "per_array_ms": round(ms_per_array, 1), "per_array_gbs": gbs(ms_per_array),
        "speedup_vs_per_array": round(ms_per_array / best, 1), "sorted": ok,
    }


def bucket_balance(vqs, keys) -> dict:
    """Bucket sizes of the model the learned sort trains on `keys` (library defaults)
    and of the same model before training (same input scaling), over every key:
    largest bucket / expected size n/256, rms relative deviation, empty buckets."""
    import torch
    trained = vqs.learned_fit(keys)
    untrained = torch.empty_like(trained)
    vqs.mlp_init(untrained, 16, torch.tensor([0.0, 1.0], dtype=torch.float32, device=keys.device))
    untrained[vqs.MLP_NPARAM:] = trained[vqs.MLP_NPARAM:]
    expected = keys.numel() / 256
    out = {}
    for name, params in (("trained", trained), ("untrained", untrained)):
        h = torch.bincount(vqs.mlp_buckets(params, keys).long(), minlength=256).double()
        dev = (h - expected) / expected
        out[name] = {"max_over_expected": round(float(h.max()) / expected, 3),
                     "rms_rel_dev": round(float(dev.pow(2).mean().sqrt()), 3),
                     "empty": int((h == 0).sum())}
        del h
    torch.cuda.empty_cache()
    return out


def learned_vs_plain(n: int, reps: int) -> dict:
    """The 5e8-key lognormal-mixture workload sorted by the plain method and by the
    learned 256-bucket splitter: median time of each over `reps` sorts (each of a
    fresh copy of the input already in HBM), whether the outputs are identical, and
    the splitter's own figures (training time, largest bucket, overflow buckets)."""
    import torch
    from paper_2205_05982_amd import vqs
    from paper_2205_05982_amd import workloads as W
    t0 = time.time()
    host = W.lognormal_mixture_u64(n, 15)
    print(f"# mixture input n={n} generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(host).to(dev)
    del host
    work = torch.empty_like(src)
    stream = torch.cuda.current_stream()
    res = {}
    outs = {}
    for name, method in (("plain", 0), ("learned", 1)):
        times = []
        # the first call warms up and, with per-launch timing on, gives the phase times
        for r in range(reps + 1):
            work.copy_(src)
            torch.cuda.synchronize()
            if r == 0:
                vqs.profile(True)
                vqs.profile_read()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            vqs.sort(work, key_type=3, method=method)
            e1.record(stream)
            torch.cuda.synchronize()
            if vqs.last_error_bits():
                raise RuntimeError(f"device error bits {vqs.last_error_bits():#x}")
            if r == 0:
                recs = vqs.profile_read()
                vqs.profile(False)
                phases = {}
                for x in recs:
                    phases[x["kind"]] = phases.get(x["kind"], 0.0) + x["ms"]
                continue
            times.append(e0.elapsed_time(e1))
        st = vqs.get_stats()
        res[name] = {"ms": round(float(np.median(times)), 3), "ms_all": [round(t, 3) for t in times],
                     "phase_ms": {k: round(v, 3) for k, v in phases.items() if v >= 0.005}}
        if method == 1:
            res[name].update({"max_bucket_over_expected": round(st["max_bucket"] / (n / 256), 3),
                              "overflow_buckets": st["overflow_buckets"],
                              "train_loss": st["train_loss"]})
        outs[name] = work.clone() if method == 0 else work
    balance = bucket_balance(vqs, src)
    identical = bool(torch.equal(outs["plain"].view(torch.int64), outs["learned"].view(torch.int64)))
    o = outs["learned"].view(torch.int64) ^ torch.tensor(-(2**63), dtype=torch.int64, device=dev)
    sorted_ok = bool((o[1:] >= o[:-1]).all().item())
    return {
        "workload": f"{n:.0e} u64: 90% mixture of 8 lognormals + 10% Zipf(1.2) duplicates, seed 15",
        "plain_ms": res["plain"]["ms"],
        "learned_ms": res["learned"]["ms"],
        "speedup": round(res["plain"]["ms"] / res["learned"]["ms"], 3),
        "plain_gkeys": round(n / res["plain"]["ms"] / 1e6, 3),
        "learned_gkeys": round(n / res["learned"]["ms"] / 1e6, 3),
        "identical_output": identical,
        "sorted": sorted_ok,
        "bucket_balance": balance,
        "learned": {k: v for k, v in res["learned"].items() if k != "ms"},
        "plain": {k: v for k, v in res["plain"].items() if k != "ms"},
        "reps": reps,
    }


def inplace_record(vqs, bufs, src, kt: int, n: int, ms_default: float, reps: int = 3) -> dict:
    """The same workload sorted in place (vqs_options.inplace: every partition in the
    order of the paper's in-place scan, no key scratch): median of reps sorts after a
    warm-up, its key traffic, its workspace against the default one, and whether its
    output equals the default path's."""
    import torch
    stream = torch.cuda.current_stream()
    times = []
    for r in range(reps + 1):
        bufs[0].copy_(src)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        vqs.sort(bufs[0], key_type=kt, inplace=1)
        e1.record(stream)
        torch.cuda.synchronize()
        if r:
            times.append(e0.elapsed_time(e1))
    st = vqs.get_stats()
    if vqs.last_error_bits():
        raise RuntimeError("device error bits in the in-place sort")
    bufs[1].copy_(src)
    vqs.sort(bufs[1], key_type=kt)
    torch.cuda.synchronize()
    same = bool(torch.equal(bufs[0], bufs[1]))
    ms = statistics.median(times)
    return {"ms": round(ms, 3), "gkeys_s": round(n / (ms * 1e-3) / 1e9, 4),
            "vs_default": round(ms_default / ms, 3),
            "passes": round((st["hbm_read_keys"] + st["hbm_write_keys"]) / (2.0 * n), 3),
            "levels": st["levels"], "workspace_bytes": vqs.workspace_bytes(n, kt, inplace=1),
            "workspace_bytes_default": vqs.workspace_bytes(n, kt), "identical_to_default": same}


def check_output(out, src, kt):
    """(sorted, same multiset) for the sorted tensor out of input src: non-decreasing
    in the key order; equal sums and sums of squares (mod 2^64) of the keys' words."""
    import torch
    sign = torch.tensor(-(2**63), dtype=torch.int64, device=out.device)
    if kt == 4:                                     # (lo, hi) pairs, compared (hi, lo)
        ow, iw = out.view(torch.int64), src.view(torch.int64)
        words = [(ow[:, 0], iw[:, 0]), (ow[:, 1], iw[:, 1])]
        hi, lo = ow[:, 1] ^ sign, ow[:, 0] ^ sign
        bad = (hi[1:] < hi[:-1]) | ((hi[1:] == hi[:-1]) & (lo[1:] < lo[:-1]))
    else:
        if kt in (3, 6):
            ow, iw = out.view(torch.int64), src.view(torch.int64)
        elif kt in (2, 5):
            ow, iw = (t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF for t in (out, src))
        else:
            ow, iw = (t.view(torch.int16).to(torch.int64) & 0xFFFF for t in (out, src))
        words = [(ow, iw)]
        okey = out if kt in (5, 6) else (ow ^ sign if kt == 3 else ow)
        bad = okey[1:] < okey[:-1]
    sorted_ok = not bool(bad.any().item())
    sum_ok = all(bool((a.sum() == b.sum()).item()) and bool(((a * a).sum() == (b * b).sum()).item())
                 for a, b in words)
    return sorted_ok, sum_ok


def measured_traffic():
    """HBM bytes per level-kernel launch (read + written) from the committed rocprofv3
    counter runs of this workload, or None when the kernel sources have changed since
    the counters were taken."""
    from paper_2205_05982_amd.profile_summary import kernel_source_hash
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                        "level_runs_kernel_u64_1e8_uniform.traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        js = json.load(f)
    if js.get("source_hash") != kernel_source_hash():
        return None
    return int(js["traffic_bytes_per_launch"])


def make_input(name: str, n: int) -> np.ndarray:
    from paper_2205_05982_amd import workloads as W
    kt, _, dist, _ = WORKLOADS[name]
    if name == "c1_u32":
        return W.uniform_u32(n, 1)
    if name.startswith("c3_"):
        return W.C3_CASES[dist][1](n)
    return W.c2(dist, n)


def cpu_threads() -> int:
    """Host threads for the all-core oracle timing: the cores this process may run on,
    capped by OMP_NUM_THREADS where the machine sets it (the process's CPU share)."""
    t = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        t = min(t, int(cap))
    return t


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(host, kt: int, m: int) -> dict:
    """The oracle timed on the host's cores on the first m keys of the input (median of
    three runs each): one thread, and all threads (the oracle's top recursion levels as
    parallel tasks, then its sort of the remaining ranges across the threads); np.sort
    and std::sort of the same keys as context."""
    import oracle
    oracle.build()
    threads = cpu_threads()
    src = host[:m]
    want = None

    def timed(fn):
        ts = []
        for _ in range(3):
            a = src.copy()
            t0 = time.perf_counter()
            fn(a)
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)), a

    t1, a1 = timed(lambda a: oracle.sort(a, kt))
    tp, ap = timed(lambda a: oracle.parallel_sort(a, kt, threads))
    if not np.array_equal(a1, ap):
        raise RuntimeError("the parallel oracle run differs from the one-threaded oracle")
    if kt == 4:
        tnp = None
    else:
        tnp, _ = timed(lambda a: a.sort(kind="quicksort"))
    tstd, astd = timed(lambda a: oracle.context_std_sort(a, kt))
    if not np.array_equal(a1, astd):
        raise RuntimeError("std::sort differs from the oracle")
    g = lambda t: round(m / t / 1e9, 5) if t else None
    return {"value": g(tp), "unit": "Gkeys/s", "cores": threads, "kind": "oracle",
            "sample": f"first {m} keys of the same input; scalar C oracle; median of 3 runs; "
                      f"{threads} threads: top recursion levels as parallel tasks, then the oracle on "
                      f"each remaining range ({tp:.2f} s)",
            "one_thread": {"value": g(t1), "seconds": round(t1, 3)},
            "cpu_model": cpu_model(),
            "context": {"np_sort_one_thread": g(tnp), "std_sort_one_thread": g(tstd),
                        "numpy": np.__version__}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build has no multi-GPU path (asked for {args.gpus}).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2205_05982_amd import vqs

    kt, n_default, gen, desc = WORKLOADS[args.workload]
    if gen == "c4":
        bench_batched(args, kt, desc)
        return
    n = args.n or n_default
    ks = vqs.KEY_SIZE[kt]
    dev = torch.device("cuda", 0)
    t0 = time.time()
    host = make_input(args.workload, n)
    print(f"# input {args.workload} n={n} generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    src = torch.from_numpy(host).to(dev)
    nbuf = args.steps + args.warmup
    bufs = [torch.empty_like(src) for _ in range(nbuf)]
    for b in bufs:
        b.copy_(src)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()

    # warmup (also allocates the library workspace)
    for i in range(args.warmup):
        vqs.sort(bufs[i], key_type=kt)
    torch.cuda.synchronize()
    err = vqs.last_error_bits()
    if err:
        raise RuntimeError(f"device error bits {err:#x}")
    print(f"# warmup done", file=sys.stderr, flush=True)

    vqs.profile(2)                # events around the level launches only
    vqs.profile_read()            # drop records of the warmup
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for i in range(args.steps):
        vqs.sort(bufs[args.warmup + i], key_type=kt)
    stop.record(stream)
    torch.cuda.synchronize()
    total_ms = start.elapsed_time(stop)
    recs = vqs.profile_read()
    vqs.profile(False)
    stats = vqs.get_stats()
    err = vqs.last_error_bits()
    if err:
        raise RuntimeError(f"device error bits {err:#x}")
    ms_step = total_ms / args.steps
    gkeys = n / (ms_step * 1e-3) / 1e9
    print(f"# timed {args.steps} steps: {ms_step:.3f} ms/step", file=sys.stderr, flush=True)

    # correctness of the last output: sorted, same multiset as the input
    out = bufs[-1]
    sorted_ok, sum_ok = check_output(out, src, kt)
    if not (sorted_ok and sum_ok):
        raise RuntimeError(f"bench output check failed: sorted={sorted_ok} multiset={sum_ok}")

    # roofline of the dominant kernel: the level (device-wide partition) kernel, from
    # the events around its launches in the timed steps
    lv_all = [r for r in recs if r["kind"] == "level_partition"]
    lv = [r for r in lv_all if r["keys"] > 0]
    lv_bytes = sum(2 * r["keys"] * ks for r in lv)
    lv_ms = sum(r["ms"] for r in lv)
    achieved = lv_bytes / (lv_ms * 1e-3) / 1e9 if lv_ms > 0 else 0.0
    levels_per_step = len(lv) / args.steps

    # the other kernels' times: two more sorts (after the timed steps) with every launch
    # recorded
    ndiag = min(2, len(bufs))
    for i in range(ndiag):
        bufs[i].copy_(src)
    torch.cuda.synchronize()
    vqs.profile(1)
    vqs.profile_read()
    for i in range(ndiag):
        vqs.sort(bufs[i], key_type=kt)
    torch.cuda.synchronize()
    diag = vqs.profile_read()
    vqs.profile(0)
    solo_ms = sum(r["ms"] for r in diag if r["kind"] == "solo") / ndiag
    all_ms = sum(r["ms"] for r in diag) / ndiag
    # full read+write sweeps over the keys: every key each level partition, copy pass,
    # single-workgroup partition and in-LDS sort reads and writes, counted by the library
    passes = (stats["hbm_read_keys"] + stats["hbm_write_keys"]) / (2.0 * n)
    e2e_frac = (passes * 2 * n * ks / (ms_step * 1e-3) / 1e9) / HBM_PEAK_GBS
    if args.profile_json:
        with open(args.profile_json, "w") as f:
            json.dump({"records": recs, "diagnostic_records": diag, "stats": stats}, f, indent=1)

    # a second denominator: the device-to-device copy of the input (one read and one
    # write of every key, like a partition pass), timed the same way
    cp_ms = []
    for r in range(4):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        bufs[0].copy_(src)
        e1.record(stream)
        torch.cuda.synchronize()
        if r:
            cp_ms.append(e0.elapsed_time(e1))
    copy_gbs = 2 * n * ks / (min(cp_ms) * 1e-3) / 1e9

    inplace = inplace_record(vqs, bufs, src, kt, n, ms_step) if len(bufs) >= 2 else None

    # free the timed buffers before the larger comparison
    del bufs, out
    torch.cuda.empty_cache()
    lvp = learned_vs_plain(args.learned_n, args.learned_reps) if args.learned_n else None
    batched = None if args.no_batched else batched_record()

    cpu = None if args.no_cpu_baseline else cpu_baseline(host, kt, min(args.cpu_sample, n))

    line = {
        "metric": METRIC,
        "value": round(gkeys, 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {1: "u16", 2: "u32", 3: "u64", 4: "u128", 5: "f32", 6: "f64"}[kt],
        "data": "synthetic",
        "config": {"workload": desc, "n": n, "method": "plain", "key_bytes": ks},
        "roofline": {
            "bound": "hbm",
            "kernel": ("level_runs_kernel (device-wide partition into tile-local runs)" if ks >= 8
                       else "level_kernel (device-wide partition, decoupled look-back)"),
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "copy_gbs": round(copy_gbs, 1),                  # measured device-to-device copy
            "frac_of_copy": round(achieved / copy_gbs, 4),
            "traffic": measured_traffic() if (args.workload == "c2_uniform" and n == 100_000_000) else None,
            "launches_per_step": round(levels_per_step, 2),
            # every level launch of the timed steps, empty ones included (the
            # population rocprofv3 averages over)
            "launch_avg_us_all": round(1e3 * sum(r["ms"] for r in lv_all) / max(len(lv_all), 1), 1),
            "bytes_per_launch_all": int(lv_bytes / max(len(lv_all), 1)),
            "level_ms_per_step": round(lv_ms / args.steps, 4),
            # from two more sorts with every launch recorded
            "solo_ms_per_step": round(solo_ms, 4),
            "kernels_ms_per_step": round(all_ms, 4),
            "passes": round(passes, 3),
            "end_to_end_frac": round(e2e_frac, 4),
        },
        "stats": {k: stats[k] for k in ("partitions", "degenerate", "basecases", "fallbacks", "max_depth",
                                       "levels", "solo_items", "hbm_read_keys", "hbm_write_keys")},
        "cpu_baseline": cpu,
        "learned_vs_plain": lvp,
        "batched": batched,
        "inplace": inplace,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
