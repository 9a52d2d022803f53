"""Benchmark of the melded-kernel library on one MI355X.

Workload (one step): the bitonic sort of 2^28 (u32 key, u32 payload = original
index) pairs in place in HBM, keys uniform from seed 1, through the library's
default form (MELD_AUTO: tile and per-stage forms tuned once). The input is
restored from a pristine copy before each step, outside the timed events;
inputs are synthetic and seeded (workloads/) and resident in HBM before the
timed region.

Printed: one JSON line with the sort's throughput (Gkeys/s), the duration of
every launch from HIP events on the launch stream and the roofline of the
dominant kernel, the melded/divergent speedup on seeds 1..3 (median, p10,
p90), the paper's published speedups (context), the two-sided loop region,
the 2^16-key sort, the odd-even and merge sorts, the segmented sort, the
serving loop, and the CPU oracle timed on this host (one thread and all the
threads it may use).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_PAIRS = 1 << 28
N_LANES = 1 << 24
PS = (0.1, 0.5, 0.9)
SEED = 1
# x read, y written, the table read once: 3 arrays of 2^24 fp32
REGION_COMPULSORY = 3 * 4 * N_LANES


def _progress(msg):
    """One line on stderr when a part of the run has finished."""
    print(f"bench: {msg} ({time.strftime('%H:%M:%S')})", file=sys.stderr, flush=True)


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=30, help="launches per per-kernel timing")
    ap.add_argument("--seg-reps", type=int, default=40,
                    help="timed segmented sorts per seed and form")
    ap.add_argument("--pair-reps", type=int, default=28,
                    help="timed 2^28-pair sorts per seed and form (28: about 1 s each)")
    ap.add_argument("--no-region", action="store_true", help="skip the region measurements")
    ap.add_argument("--no-sort", action="store_true",
                    help="skip the 2^16-key, odd-even and merge sorts")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-seg", action="store_true", help="skip the segmented sort")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the Poisson serving trace (0 skips serving)")
    ap.add_argument("--profile", nargs="?", const="region", default=None,
                    choices=["region", "region_sweep", "sort", "pairs", "next"],
                    help="short run for rocprofv3: 'region' (a 256 MiB copy, then the "
                         "region in each form), 'sort' (2^16 keys and the 4096-segment sort, "
                         "each form), 'pairs' (a 256 MiB copy, then one 2^28-pair sort per "
                         "form and three MELD_AUTO sorts) or 'next' (2^24 keys: odd-even "
                         "buckets of 2^13 and the merge sort, each form)")
    return ap.parse_args()


def _events_time(torch, fn, reps):
    """Average ms of fn() over reps back-to-back calls, HIP events on the current stream."""
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps


def _measured_traffic(name):
    """HBM bytes per launch of a kernel from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (profiles/<name>), scaled by the copy calibration; None when
    the kernel's sources have changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            rec = json.load(f)
        h = hashlib.sha1()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != rec["sources_sha1"]:
            return None
        return int(rec["traffic_bytes"])
    except (OSError, KeyError, ValueError):
        return None


def _dist(np, samples_ms, scale=1e3):
    """Median, p10 and p90 of timings in ms, scaled (default: to us)."""
    a = np.asarray(samples_ms, dtype=np.float64) * scale
    return {"median": round(float(np.median(a)), 2), "p10": round(float(np.percentile(a, 10)), 2),
            "p90": round(float(np.percentile(a, 90)), 2)}


def _tuned_region_form(meld, tt, tf):
    """The form MELD_AUTO chose for the 2^24-lane region at p = 0.5 with trips (tt, tf)."""
    names = {0: "divergent", 1: "melded", 2: "melded_inplace"}
    key = f"n=24 tab=24 tT={tt} tF={tf} p10=5"
    for e in json.loads(meld.plan_describe())["entries"]:
        if e["op"] == "region" and e["key"] == key:
            return names.get(e["form"], str(e["form"]))
    return None


PATHS = {"lds": 0, "lane_exchange": 1}  # MELD_OPT_LANE_EXCHANGE values


def _set_path(meld, x):
    """Phases k <= 64 of the sorts: 0 the LDS comparator network, 1 registers with
    DPP lane exchanges, -1 the library's choice."""
    meld.set_option(0, meld.OPT_LANE_EXCHANGE, x)


def _mixed_fraction(p, wave=64):
    return 1.0 - p ** wave - (1.0 - p) ** wave


def _cpu_info():
    """Host CPU model, logical CPUs and the CPUs this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count() or 1
    return {"cpu_model": model, "host_logical_cpus": os.cpu_count(), "affinity_cpus": allowed}


def _oracle_threads():
    """Host threads for the all-core oracle timings: the CPUs this process may use,
    at most 16 (the host share of one GPU on the GPU machines)."""
    return max(1, min(16, _cpu_info()["affinity_cpus"]))


def _pairs_inputs(torch, np, workloads, dev, seed, n):
    kin = torch.from_numpy(workloads.keys_u32(seed, n).view(np.int32)).to(dev)
    pin = torch.arange(n, dtype=torch.int32, device=dev)
    return kin, pin


def _check_pairs_sorted(torch, kin, k, p):
    """The timed output is the unique (key, payload) order of the input: keys
    non-decreasing, payloads increasing within equal keys, payload a permutation
    of 0..n-1 and k == kin[p] (these fix the sorted array exactly)."""
    ku = k.to(torch.int64) & 0xFFFFFFFF
    pu = p.to(torch.int64) & 0xFFFFFFFF
    # (key - 2^31) * 2^32 + payload orders like the unsigned (key, payload)
    # pair and fits a signed 64-bit integer
    comp = (ku - (1 << 31)) * (1 << 32) + pu
    if not bool((comp[1:] > comp[:-1]).all()):
        raise SystemExit("2^28-pair sort: output not in strictly increasing (key, payload) order")
    if not bool((torch.bincount(pu, minlength=k.numel()) == 1).all()):
        raise SystemExit("2^28-pair sort: payload is not a permutation")
    if not torch.equal(kin[pu], k):
        raise SystemExit("2^28-pair sort: keys do not follow their payloads")


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); "
              "the kernels shard by lane range / segment but no multi-GPU path is built",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2107_05681_amd as meld
    import workloads

    if not os.path.exists(meld.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.profile == "sort":
        _profile_sorts(torch, np, meld, workloads, dev)
        return
    if args.profile == "pairs":
        _profile_pairs(torch, np, meld, workloads, dev)
        return
    if args.profile == "next":
        _profile_next(torch, np, meld, workloads, dev)
        return
    if args.profile == "region":
        _profile_region(torch, np, meld, workloads, dev)
        return
    if args.profile == "region_sweep":
        _profile_region_sweep(torch, np, meld, workloads, dev)
        return

    # ---- Headline: bitonic sort of 2^28 (key, payload = index) pairs ----------
    n = N_PAIRS
    kin, pin = _pairs_inputs(torch, np, workloads, dev, SEED, n)
    k, p = torch.empty_like(kin), torch.empty_like(pin)

    def restore():
        k.copy_(kin)
        p.copy_(pin)

    for _ in range(max(args.warmup, 1)):  # the first MELD_AUTO call tunes this shape once
        restore()
        meld.sort_timed(k, p, variant="auto")
    torch.cuda.synchronize()
    step_ms, launches = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        restore()  # outside the events: each step sorts the pristine input
        ms = meld.sort_timed(k, p, variant="auto")
        launches.append(ms)
        step_ms.append(sum(ms))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    _check_pairs_sorted(torch, kin, k, p)
    ms_per_step = float(np.mean(step_ms))
    value = n / (ms_per_step * 1e-3) / 1e9
    plan = meld.sort_plan(n, pairs=True, variant="auto", device=0)
    roof, per_kind = _sort_roofline(np, plan, launches, n)
    hbm_moved = 16.0 * n * plan["hbm_passes"]
    del k, p
    torch.cuda.empty_cache()

    _progress("headline 2^28-pair sorts done")
    pairs_forms = _bench_pairs_forms(torch, np, meld, workloads, dev, kin, pin, args)
    _progress("divergent / melded 2^28-pair sorts done")
    del kin, pin
    torch.cuda.empty_cache()

    region_info = None
    if not args.no_region:
        region_info = _bench_region(torch, np, meld, workloads, dev, args)
        _progress("region done")

    sort16 = oddeven_info = merge_info = None
    if not args.no_sort:
        sort16 = _bench_sort16(torch, np, meld, workloads, dev, args)
        oddeven_info = _bench_oddeven(torch, np, meld, workloads, dev)
        merge_info = _bench_mergesort(torch, np, meld, workloads, dev)
        _progress("2^16-key, odd-even and merge sorts done")

    seg_info = None
    if not args.no_seg:
        seg_info = _bench_segmented(torch, np, meld, workloads, dev, args)
        _progress("segmented sort done")

    serve_info = None
    if args.serve_seconds > 0:
        serve_info = _bench_serving(meld, workloads, args.serve_seconds)
        _progress("serving done")

    cpu = None
    if not args.no_cpu:
        cpu = _cpu_baseline_pairs(np, workloads)
        _progress("CPU oracle, 2^28-pair sample done")
        if sort16 is not None:
            sort16["cpu_oracle"] = _cpu_sort_keys(np, workloads, 1 << 16)
        if seg_info is not None:
            seg_info["cpu_oracle"] = _cpu_segmented(np, workloads)
        if region_info is not None:
            region_info["cpu_oracle"] = _cpu_region(np, workloads)

    out = {
        "metric": "melded/divergent speedup; Gkeys/s and VALU lane utilisation (rocprof)",
        "value": round(value, 4),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "ms_per_step_dist": _dist(np, step_ms, scale=1.0),
        "wall_s_timed": round(wall, 4),
        "wall_note": "wall clock of the timed loop, including the untimed restore of the "
                     "2 GiB input before each step",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded SplitMix64 keys, payload = index; workloads/)",
        "config": {
            "workload": "bitonic sort of 2^28 (u32 key, u32 payload = original index) pairs, "
                        "keys uniform from seed 1, in place in HBM, MELD_AUTO",
            "n": n, "seed": SEED, "variant": "auto",
            "log_tile": plan["log_tile"], "low_phases": plan["low"],
            "high_phases": plan["high"], "hbm_passes": plan["hbm_passes"],
            "launches": len(plan["passes"]),
        },
        "sort_hbm": {"bytes_per_sort": int(hbm_moved),
                     "achieved_GBs": round(hbm_moved / (ms_per_step * 1e-3) / 1e9, 1),
                     "frac_of_peak": round(hbm_moved / (ms_per_step * 1e-3) / 1e9
                                           / HBM_PEAK_GBS, 4),
                     "note": "16 B per pair per HBM pass (8 read + 8 written) x the plan's "
                             "passes, over the whole sort"},
        "kernels": per_kind,
        "roofline": roof,
        "melded_vs_divergent": pairs_forms,
        "paper_context": PAPER_CONTEXT,
        "region": region_info,
        "sort_keys_2^16": sort16,
        "oddeven_buckets": oddeven_info,
        "mergesort": merge_info,
        "segmented": seg_info,
        "serving": serve_info,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


# Published numbers of the paper (Evaluation section, "Evaluation Setup and
# Benchmarks" and "Performance"): context only, measured on other hardware.
PAPER_CONTEXT = {
    "hardware": "AMD Radeon Pro Vega 20 (wave64, 64 KiB LDS, 1700 MHz), ROCm 4.2, LLVM 12",
    "synthetic_benchmarks_geomean_speedup": 1.36,
    "real_world_geomean_speedup_all_block_sizes": 1.15,
    "real_world_geomean_speedup_best_block_size": 1.16,
    "note": "compiler-melded code vs the same kernels at -O3; context only, not a target",
}

KIND_KERNEL = {
    "local": "bitonic_sort_regs_kernel (local sort of every tile)",
    "regs": "bitonic_global_kernel (streaming pass, up to 6 steps in registers)",
    "gather": "bitonic_pass_regs_kernel<L,R,L-R> (gathered streaming pass)",
    "merge": "bitonic_pass_regs_kernel<L,L,L> (merge tail of a phase)",
    "tile": "bitonic_sort_regs_kernel (single tile)",
}


def _pass_kernel(ps, log_tile):
    """Key and name of the kernel one launch of the plan runs (the streaming passes
    are a kernel per step count R)."""
    kind = ps["kind"]
    if kind == "regs":
        return f"regs{ps['steps']}", f"bitonic_global_kernel, R = {ps['steps']} (streaming pass)"
    if kind == "gather":
        r = ps["steps"]
        return (f"gather{r}", f"bitonic_pass_regs_kernel<true, 13, {r}, {13 - r}> "
                              "(gathered streaming pass)")
    if kind == "merge":
        return "merge", (f"bitonic_pass_regs_kernel<true, {log_tile}, {log_tile}, {log_tile}> "
                         "(merge tail of a phase)")
    return kind, KIND_KERNEL[kind]


def _sort_roofline(np, plan, launches, n):
    """Per launch kind of the timed sorts: launches, average and total time, and the
    HBM rate of its algorithmic bytes (16 B per pair per launch); the roofline of
    the kernel with the largest total time (the streaming passes are a kernel per
    step count, so the merge tail, 15 launches of one kernel, is the largest)."""
    kinds = [ps["kind"] for ps in plan["passes"]]
    keys = [_pass_kernel(ps, plan["log_tile"]) for ps in plan["passes"]]
    per, per_k = {}, {}
    for step in launches:
        if len(step) != len(kinds):
            raise SystemExit("sort: launches differ from the plan")
        for kind, (key, _), ms in zip(kinds, keys, step):
            per.setdefault(kind, []).append(ms)
            per_k.setdefault(key, []).append(ms)
    per_kind = {}
    for kind, ms in per.items():
        avg = float(np.mean(ms))
        per_kind[kind] = {"kernel": KIND_KERNEL[kind], "launches_per_sort": kinds.count(kind),
                          "avg_launch_us": round(avg * 1e3, 2),
                          "ms_per_sort": round(sum(ms) / len(launches), 4),
                          "alg_GBs": round(16.0 * n / (avg * 1e-3) / 1e9, 1)}
    names = dict(keys)
    dom = max(per_k, key=lambda k: sum(per_k[k]))
    avg_us = round(float(np.mean(per_k[dom])) * 1e3, 2)
    achieved = 16.0 * n / (avg_us * 1e-6) / 1e9
    roof = {"bound": "hbm", "kernel": names[dom], "kind": dom,
            "launches_per_sort": len(per_k[dom]) // len(launches),
            "avg_launch_us": avg_us, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _measured_traffic("sort_merge_traffic.json") if dom == "merge" else None,
            "alg_bytes_per_launch": int(16 * n),
            "note": "one launch reads and writes every (key, payload) pair once: 16 B per pair; "
                    "avg_launch_us from HIP events recorded between the launches of the timed "
                    "sorts on their stream"}
    return roof, per_kind


def _bench_pairs_forms(torch, np, meld, workloads, dev, kin1, pin, args):
    """2^28 pairs, divergent vs melded (same tile), interleaved, seeds 1..3, at least
    ~1 s of sorts per seed and form; the local-sort launch alone per form."""
    n = N_PAIRS
    k, p = torch.empty_like(kin1), torch.empty_like(pin)
    res = {}
    reps = max(4, args.pair_reps)
    for seed in (1, 2, 3):
        kin = kin1 if seed == SEED else _pairs_inputs(torch, np, workloads, dev, seed, n)[0]
        rec = {"reps": reps}
        for path, x in PATHS.items():
            _set_path(meld, x)
            t = {"divergent": [], "melded": []}
            for rep in range(reps + 1):
                for v in ("divergent", "melded"):
                    k.copy_(kin)
                    p.copy_(pin)
                    s = torch.cuda.Event(enable_timing=True)
                    e = torch.cuda.Event(enable_timing=True)
                    s.record()
                    meld.sort(k, p, variant=v)
                    e.record()
                    e.synchronize()
                    if rep > 0:
                        t[v].append(s.elapsed_time(e))
            d, m = float(np.median(t["divergent"])), float(np.median(t["melded"]))
            rec[path] = {"divergent_ms": _dist(np, t["divergent"], scale=1.0),
                         "melded_ms": _dist(np, t["melded"], scale=1.0),
                         "speedup": round(d / m, 4),
                         "melded_Gkeys_s": round(n / (m * 1e-3) / 1e9, 3)}
        _set_path(meld, -1)
        rec["speedup"] = rec["lane_exchange"]["speedup"]
        res[f"seed_{seed}"] = rec
        if seed != SEED:
            del kin
    res["median_speedup"] = round(float(np.median(
        [res[f"seed_{s}"]["speedup"] for s in (1, 2, 3)])), 4)
    res["median_speedup_lds_path"] = round(float(np.median(
        [res[f"seed_{s}"]["lds"]["speedup"] for s in (1, 2, 3)])), 4)
    # the local sort alone: the network's first t (t + 1) / 2 steps are exactly that launch
    plan = meld.sort_plan(n, pairs=True, variant="melded", device=0)
    local = plan["passes"][0]["steps"]
    res["local_sort_kernel"] = {"steps": local, "log_tile": plan["log_tile"]}
    for path, x in PATHS.items():
        _set_path(meld, x)
        tl = {}
        for v in ("divergent", "melded"):
            tl[v] = _time_sorts(torch, np, lambda v=v: meld.sort_steps(k, p, local, variant=v),
                                lambda: (k.copy_(kin1), p.copy_(pin)), 11)
        res["local_sort_kernel"][path] = {"divergent_ms": round(tl["divergent"], 4),
                                          "melded_ms": round(tl["melded"], 4),
                                          "speedup": round(tl["divergent"] / tl["melded"], 4)}
    _set_path(meld, -1)
    lx = res["local_sort_kernel"]
    lx["melded_lane_exchange_vs_melded_lds"] = round(lx["lds"]["melded_ms"]
                                                     / lx["lane_exchange"]["melded_ms"], 4)
    del k, p
    torch.cuda.empty_cache()
    return res


def _profile_region(torch, np, meld, workloads, dev):
    """A 256 MiB copy (calibration of the byte counters), then the region at p in
    {0.1, 0.5, 0.9} in each form."""
    x, tab, st, sf = workloads.region_inputs(SEED, N_LANES)
    xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(tab).to(dev)
    y = torch.empty_like(xd)
    src = torch.empty(1 << 26, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)  # calibration copy: 256 MiB read + 256 MiB written
    for v in ("melded", "melded", "melded", "divergent", "melded_inplace"):
        for p in PS:
            meld.divergent_region(xd, td, SEED, workloads.thr_from_p(p), st, sf, variant=v,
                                  out=y)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "region", "copy_bytes": 2 * src.numel() * 4}))


def _profile_region_sweep(torch, np, meld, workloads, dev):
    """p = 0.5, 2^24 lanes: for trips (10, 10), (20, 20) and (32, 32), the divergent and
    melded forms, then each form's memory path alone (gathers only)."""
    x, tab, st, sf = workloads.region_inputs(SEED, N_LANES)
    xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(tab).to(dev)
    y = torch.empty_like(xd)
    thr = workloads.thr_from_p(0.5)
    for tt, tf in ((10, 10), (20, 20), (32, 32)):
        st_t, sf_t = dict(st, trips=tt), dict(sf, trips=tf)
        for only in (False, True):
            for v in ("divergent", "melded"):
                meld.divergent_region(xd, td, SEED, thr, st_t, sf_t, variant=v, out=y,
                                      gathers_only=only)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "region_sweep"}))


def _bench_region(torch, np, meld, workloads, dev, args):
    """The two-sided loop region over 2^24 lanes at p in {0.1, 0.5, 0.9}: per-form
    timings (interleaved), the tuned step, sensitivity cases and variants."""
    x, tab, st, sf = workloads.region_inputs(SEED, N_LANES)
    xd = torch.from_numpy(x).to(dev)
    td = torch.from_numpy(tab).to(dev)
    thr = {p: workloads.thr_from_p(p) for p in PS}
    ys = {p: torch.empty_like(xd) for p in PS}

    def region(p, variant):
        meld.divergent_region(xd, td, SEED, thr[p], st, sf, variant=variant, out=ys[p])

    def step():
        for p in PS:
            region(p, "auto")

    for _ in range(3):
        step()
    torch.cuda.synchronize()
    step_ms = _events_time(torch, step, 20)

    per_p = {}
    for p in PS:
        for _ in range(3):
            region(p, "divergent")
            region(p, "melded")
        td_ms, tm_ms, ti_ms = [], [], []
        for _ in range(7):
            td_ms.append(_events_time(torch, lambda: region(p, "divergent"), args.reps))
            tm_ms.append(_events_time(torch, lambda: region(p, "melded"), args.reps))
            ti_ms.append(_events_time(torch, lambda: region(p, "melded_inplace"), args.reps))
        d, m = float(np.median(td_ms)), float(np.median(tm_ms))
        mi = float(np.median(ti_ms))
        ceil = {v: _gathers_only_us(torch, np, meld, xd, td, thr[p], st, sf, ys[p], v, args)
                for v in ("divergent", "melded")}
        e_t = p * st["trips"] + (1 - p) * sf["trips"]
        alg_bytes = N_LANES * (8 + 4 * e_t)
        per_p[str(p)] = {
            "divergent_us": round(d * 1e3, 2), "melded_us": round(m * 1e3, 2),
            "speedup": round(d / m, 4),
            "divergent_us_dist": _dist(np, td_ms), "melded_us_dist": _dist(np, tm_ms),
            "melded_inplace_us": round(mi * 1e3, 2),
            "speedup_inplace": round(d / mi, 4),
            "mixed_wave_fraction": round(_mixed_fraction(p), 5),
            "melded_gather_GBs": round(alg_bytes / (m * 1e-3) / 1e9, 1),
            "melded_compulsory_frac": round(REGION_COMPULSORY / (m * 1e-3) / 1e9
                                            / HBM_PEAK_GBS, 4),
            "divergent_compulsory_frac": round(REGION_COMPULSORY / (d * 1e-3) / 1e9
                                               / HBM_PEAK_GBS, 4),
            "gathers_only_us": {v: round(c, 2) for v, c in ceil.items()},
            "frac_of_gathers_only": {"divergent": round(ceil["divergent"] / (d * 1e3), 4),
                                     "melded": round(ceil["melded"] / (m * 1e3), 4)},
        }

    # Sensitivity: both sides gathering the same entries (sides differ only in
    # multiplier and trip count), p = 0.5.
    same = {}
    st_s = dict(st, off=sf["off"], step=sf["step"])

    def region_same(variant):
        meld.divergent_region(xd, td, SEED, thr[0.5], st_s, sf, variant=variant, out=ys[0.5])

    for v in ("divergent", "melded", "melded_inplace"):
        region_same(v)
        same[v] = float(np.median([_events_time(torch, lambda: region_same(v), args.reps)
                                   for _ in range(3)]))
    same_index = {"p": 0.5, "divergent_us": round(same["divergent"] * 1e3, 2),
                  "melded_us": round(same["melded"] * 1e3, 2),
                  "melded_inplace_us": round(same["melded_inplace"] * 1e3, 2),
                  "speedup": round(same["divergent"] / same["melded"], 4),
                  "speedup_inplace": round(same["divergent"] / same["melded_inplace"], 4)}

    # Sensitivity: other trip counts of the workload's range (8..32 per side).
    trips_sweep = {}
    for tt, tf in ((8, 8), (8, 32), (32, 8), (20, 20), (32, 32)):
        st_t, sf_t = dict(st, trips=tt), dict(sf, trips=tf)

        def region_trips(variant):
            meld.divergent_region(xd, td, SEED, thr[0.5], st_t, sf_t, variant=variant,
                                  out=ys[0.5])

        tm = {}
        for v in ("divergent", "melded", "auto"):
            region_trips(v)  # "auto": the tuner times the forms for this shape once
            tm[v] = float(np.median([_events_time(torch, lambda: region_trips(v), args.reps)
                                     for _ in range(3)]))
        ceil = {v: _gathers_only_us(torch, np, meld, xd, td, thr[0.5], st_t, sf_t, ys[0.5], v,
                                    args) for v in ("divergent", "melded")}
        trips_sweep[f"{tt},{tf}"] = {"divergent_us": round(tm["divergent"] * 1e3, 2),
                                     "melded_us": round(tm["melded"] * 1e3, 2),
                                     "speedup": round(tm["divergent"] / tm["melded"], 4),
                                     "auto_us": round(tm["auto"] * 1e3, 2),
                                     "auto_form": _tuned_region_form(meld, tt, tf),
                                     "gathers_only_us": {v: round(c, 2) for v, c in ceil.items()},
                                     "gathers_only_speedup": round(ceil["divergent"]
                                                                   / ceil["melded"], 4)}

    variants = _bench_region_variants(torch, np, meld, workloads, xd, td, ys[0.5], args)
    seeds = _bench_seeds(torch, np, meld, workloads, dev, args)

    # Check the step's outputs once (every form equal, bit for bit).
    for p in PS:
        region(p, "auto")
        a = ys[p].clone()
        for other in ("divergent", "melded", "melded_inplace"):
            region(p, other)
            if not torch.equal(a.view(torch.int32), ys[p].view(torch.int32)):
                raise SystemExit(f"auto and {other} region differ at p={p}")

    launch_us = step_ms * 1e3 / len(PS)
    return {
        "workload": "two-sided loop region: 2^24 fp32 lanes x p in {0.1,0.5,0.9}, branch bit "
                    "Bernoulli(p) from hash(seed,i), each side 8-32 fma+gather steps into a "
                    "2^24-entry (64 MiB) fp32 table",
        "trips_true": st["trips"], "trips_false": sf["trips"],
        "step_ms": round(step_ms, 4), "G_lanes_s": round(len(PS) * N_LANES / step_ms / 1e6, 2),
        "roofline": {
            "bound": "hbm", "kernel": "region_melded_kernel (MELD_AUTO step, one launch per p)",
            "avg_launch_us": round(launch_us, 2),
            "achieved": round(REGION_COMPULSORY / (launch_us * 1e-6) / 1e9, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(REGION_COMPULSORY / (launch_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
            "traffic": _measured_traffic("region_melded_traffic.json"),
            "alg_bytes_per_launch": int(REGION_COMPULSORY),
            "note": "compulsory bytes: x read, y written and the 64 MiB table read once "
                    "(3 x 64 MiB); the gathers re-read table entries from L2 / MALL, so the "
                    "kernel is bound by the vector-memory address path, not by HBM"},
        "melded_vs_divergent": per_p,
        "same_index_sides": same_index,
        "trips_sweep_p0.5": trips_sweep,
        "region_variants": variants,
        "seeds": seeds,
    }


def _gathers_only_us(torch, np, meld, xd, td, thr, st, sf, y, variant, args):
    """Median us of the region's memory path alone in one form (meld_probe_region_gathers:
    the same lanes, branch, addresses, exec masks and batching, no fma chain)."""
    def run():
        meld.divergent_region(xd, td, SEED, thr, st, sf, variant=variant, out=y,
                              gathers_only=True)
    run()
    return float(np.median([_events_time(torch, run, args.reps) for _ in range(3)])) * 1e3


def _bench_seeds(torch, np, meld, workloads, dev, args):
    """The region (2^24 lanes, p = 0.5, each seed's own trip counts and tables)
    and the 2^16-key sort for seeds 1, 2 and 3: speedup per seed and the median."""
    region, sort = {}, {}
    thr = workloads.thr_from_p(0.5)
    for seed in (1, 2, 3):
        x, tab, st, sf = workloads.region_inputs(seed, N_LANES)
        xd, tdv = torch.from_numpy(x).to(dev), torch.from_numpy(tab).to(dev)
        y = torch.empty_like(xd)
        t = {}
        for v in ("divergent", "melded"):
            run = (lambda v=v: meld.divergent_region(xd, tdv, seed, thr, st, sf, variant=v, out=y))
            run()
            t[v] = float(np.median([_events_time(torch, run, args.reps) for _ in range(5)]))
        region[str(seed)] = {"trips": [st["trips"], sf["trips"]],
                             "divergent_us": round(t["divergent"] * 1e3, 2),
                             "melded_us": round(t["melded"] * 1e3, 2),
                             "speedup": round(t["divergent"] / t["melded"], 4)}
        kin = torch.from_numpy(workloads.keys_u32(seed, 1 << 16).view(np.int32)).to(dev)
        k = torch.empty_like(kin)
        ts = {v: _time_sorts(torch, np, lambda v=v: meld.sort(k, None, variant=v),
                             lambda: k.copy_(kin), 21) for v in ("divergent", "melded")}
        sort[str(seed)] = {"divergent_us": round(ts["divergent"] * 1e3, 2),
                           "melded_us": round(ts["melded"] * 1e3, 2),
                           "speedup": round(ts["divergent"] / ts["melded"], 4)}
        del xd, tdv, y, kin, k
    torch.cuda.empty_cache()
    med = lambda d: round(float(np.median([v["speedup"] for v in d.values()])), 4)
    return {"region_p0.5_2^24": {**region, "median_speedup": med(region)},
            "sort_keys_2^16": {**sort, "median_speedup": med(sort)}}


def _bench_region_variants(torch, np, meld, workloads, xd, td, y, args):
    """NEXT-row variants of the region at 2^24 lanes: the three-way region (SB4
    pattern) with equal thirds, equal trip counts, and biased (the middle way
    never taken); the two-sided region with per-lane trip counts in [8, 32]."""
    w0 = dict(workloads.SIDE_TRUE, trips=workloads.way_trips(SEED, 0))
    w1 = dict(workloads.SIDE_MID, trips=workloads.way_trips(SEED, 1))
    w2 = dict(workloads.SIDE_FALSE, trips=workloads.way_trips(SEED, 2))
    third, two_thirds, half = (workloads.thr_from_p(1 / 3), workloads.thr_from_p(2 / 3),
                               workloads.thr_from_p(0.5))

    def measure(run):
        t = {}
        for v in ("divergent", "melded", "melded_inplace", "auto"):
            run(v)  # "auto": the tuner times the three forms for this shape once
            t[v] = float(np.median([_events_time(torch, lambda: run(v), args.reps)
                                    for _ in range(3)]))
        return {"divergent_us": round(t["divergent"] * 1e3, 2),
                "melded_us": round(t["melded"] * 1e3, 2),
                "melded_inplace_us": round(t["melded_inplace"] * 1e3, 2),
                "auto_us": round(t["auto"] * 1e3, 2),
                "speedup": round(t["divergent"] / t["melded"], 4)}

    out = {}
    cases = {
        "three_way_thirds": (third, two_thirds, w0, w1, w2),
        "three_way_thirds_trips_20": (third, two_thirds, dict(w0, trips=20), dict(w1, trips=20),
                                      dict(w2, trips=20)),
        "three_way_biased_middle_never": (half, half, w0, w1, w2),
    }
    for name, (t0, t1, a, b, c) in cases.items():
        out[name] = measure(lambda v: meld.region3(xd, td, SEED, t0, t1, a, b, c, variant=v,
                                                   out=y))
        out[name]["trips"] = [a["trips"], b["trips"], c["trips"]]
    st = dict(workloads.SIDE_TRUE, trips_lo=8, trips_hi=32)
    sf = dict(workloads.SIDE_FALSE, trips_lo=8, trips_hi=32)
    out["per_lane_trips_8_32_p0.5"] = measure(
        lambda v: meld.region_lanetrips(xd, td, SEED, half, st, sf, variant=v, out=y))
    return out


def _bench_oddeven(torch, np, meld, workloads, dev):
    """Batcher's odd-even merge network on buckets (the PCM network): 2^28 keys in
    buckets of 2^13 and 2^10, divergent vs melded."""
    n = 1 << 28
    kin = torch.from_numpy(workloads.keys_u32(SEED, n).view(np.int32)).to(dev)
    k = torch.empty_like(kin)
    res = {}
    for log_b in (13, 10):
        t = {}
        for v in ("divergent", "melded"):
            t[v] = _time_sorts(torch, np, lambda: meld.oddeven_sort_buckets(k, log_b, variant=v),
                               lambda: k.copy_(kin), 4)
        res[f"buckets_2^{log_b}"] = {"divergent_ms": round(t["divergent"], 3),
                                     "melded_ms": round(t["melded"], 3),
                                     "speedup": round(t["divergent"] / t["melded"], 4),
                                     "melded_Gkeys_s": round(n / (t["melded"] * 1e-3) / 1e9, 3)}
    del kin, k
    torch.cuda.empty_cache()
    return {"keys": n, **res}


def _bench_mergesort(torch, np, meld, workloads, dev):
    """Bottom-up merge sort (the MS network of the paper): 2^20 keys (the paper's size)
    and 2^24, divergent vs melded; merge passes alone = total - the run sort."""
    res = {}
    for log_n in (20, 24):
        n = 1 << log_n
        kin = torch.from_numpy(workloads.keys_u32(SEED, n).view(np.int32)).to(dev)
        k = torch.empty_like(kin)
        t = {}
        for v in ("divergent", "melded"):
            for passes, tag in ((-1, "all"), (0, "runs")):
                t[v + tag] = _time_sorts(
                    torch, np, lambda: meld.merge_sort(k, max_passes=passes, variant=v),
                    lambda: k.copy_(kin), 7)
        md, mm = t["divergentall"] - t["divergentruns"], t["meldedall"] - t["meldedruns"]
        res[f"keys_2^{log_n}"] = {"divergent_ms": round(t["divergentall"], 3),
                                  "melded_ms": round(t["meldedall"], 3),
                                  "speedup": round(t["divergentall"] / t["meldedall"], 4),
                                  "merge_passes_divergent_ms": round(md, 3),
                                  "merge_passes_melded_ms": round(mm, 3),
                                  "merge_passes_speedup": round(md / mm, 4) if mm > 0 else None,
                                  "melded_Gkeys_s": round(n / (t["meldedall"] * 1e-3) / 1e9, 3)}
        del kin, k
    torch.cuda.empty_cache()
    return res


def _bench_sort16(torch, np, meld, workloads, dev, args):
    """2^16 keys (seed 1): divergent vs melded end to end, interleaved, and the
    local-sort launch alone."""
    n = 1 << 16
    kin = torch.from_numpy(workloads.keys_u32(SEED, n).view(np.int32)).to(dev)
    k = torch.empty_like(kin)
    plan = meld.sort_plan(n, pairs=False, variant="melded", device=0)
    local = plan["passes"][0]["steps"]
    out = {"log_tile": plan["log_tile"], "hbm_passes": plan["hbm_passes"],
           "hbm_frac_note": "not meaningful: 256 KiB per pass, the sort is bound "
                            "by launch and per-tile latency"}
    for path, x in PATHS.items():
        _set_path(meld, x)
        times = {"divergent": [], "melded": []}
        for rep in range(41):
            for v in ("divergent", "melded"):
                k.copy_(kin)
                s = torch.cuda.Event(enable_timing=True)
                e = torch.cuda.Event(enable_timing=True)
                s.record()
                meld.sort(k, None, variant=v)
                e.record()
                e.synchronize()
                if rep > 0:
                    times[v].append(s.elapsed_time(e))
        d, m = float(np.median(times["divergent"])), float(np.median(times["melded"]))
        # the local-sort kernel alone: the network's first t (t + 1) / 2 steps
        # are exactly that launch
        tl = {v: _time_sorts(torch, np, lambda v=v: meld.sort_steps(k, None, local, variant=v),
                             lambda: k.copy_(kin), 21) for v in ("divergent", "melded")}
        out[path] = {"divergent_us": round(d * 1e3, 2), "melded_us": round(m * 1e3, 2),
                     "speedup": round(d / m, 4),
                     "melded_Gkeys_s": round(n / (m * 1e-3) / 1e9, 3),
                     "divergent_us_dist": _dist(np, times["divergent"]),
                     "melded_us_dist": _dist(np, times["melded"]),
                     "hbm_frac": round(8.0 * n * plan["hbm_passes"] / (m * 1e-3) / 1e9
                                       / HBM_PEAK_GBS, 5),
                     "local_sort_kernel": {
                         "steps": local,
                         "divergent_us": round(tl["divergent"] * 1e3, 2),
                         "melded_us": round(tl["melded"] * 1e3, 2),
                         "speedup": round(tl["divergent"] / tl["melded"], 4)}}
    _set_path(meld, -1)
    out["melded_lane_exchange_vs_melded_lds"] = round(
        out["lds"]["melded_us"] / out["lane_exchange"]["melded_us"], 4)
    # MELD_AUTO (its tile and forms tuned on the first call) and the seeds 1..3
    meld.sort(k.copy_(kin), None, variant="auto")
    auto_plan = meld.sort_plan(n, pairs=False, variant="auto", device=0)
    out["auto"] = {"plan": {key: auto_plan[key] for key in
                            ("log_tile", "low", "high", "low_path", "hbm_passes")}}
    for seed in (1, 2, 3):
        ks = kin if seed == SEED else torch.from_numpy(
            workloads.keys_u32(seed, n).view(np.int32)).to(dev)
        t = {v: [] for v in ("divergent", "melded", "auto")}
        for rep in range(41):
            for v in t:
                k.copy_(ks)
                s = torch.cuda.Event(enable_timing=True)
                e = torch.cuda.Event(enable_timing=True)
                s.record()
                meld.sort(k, None, variant=v)
                e.record()
                e.synchronize()
                if rep > 0:
                    t[v].append(s.elapsed_time(e))
        med = {v: float(np.median(x)) for v, x in t.items()}
        out["auto"][f"seed_{seed}"] = {
            "divergent_us": round(med["divergent"] * 1e3, 2),
            "melded_us": round(med["melded"] * 1e3, 2),
            "auto_us": round(med["auto"] * 1e3, 2),
            "auto_us_dist": _dist(np, t["auto"]),
            "speedup": round(med["divergent"] / med["melded"], 4),
            "auto_Gkeys_s": round(n / (med["auto"] * 1e-3) / 1e9, 3)}
    return out


def _profile_sorts(torch, np, meld, workloads, dev):
    """One launch sequence per form: 2^16-key sort, then the 4096-segment sort, on the
    lane-exchange path; then the same on the LDS comparator network."""
    keys = torch.from_numpy(workloads.keys_u32(SEED, 1 << 16).view(np.int32)).to(dev)
    off = workloads.segment_offsets(SEED, 4096)
    od = torch.from_numpy(off.view(np.int32)).to(dev)
    seg = torch.from_numpy(workloads.keys_u32(SEED, int(off[-1])).view(np.int32)).to(dev)
    meld.set_option(0, meld.OPT_USE_GRAPHS, 0)
    for x in (PATHS["lane_exchange"], PATHS["lds"]):
        _set_path(meld, x)
        for v in ("divergent", "melded"):
            meld.sort(keys.clone(), variant=v)
        for lo, hi in (("divergent", "divergent"), ("melded", "melded")):
            meld.segmented_sort(seg.clone(), od, low=lo, high=hi)
    _set_path(meld, -1)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "sort"}))


def _profile_pairs(torch, np, meld, workloads, dev):
    """A 256 MiB copy (calibration of the byte counters), one 2^28-pair sort per
    form, then three MELD_AUTO sorts (the bench's step)."""
    n = N_PAIRS
    kin, pin = _pairs_inputs(torch, np, workloads, dev, SEED, n)
    k, p = torch.empty_like(kin), torch.empty_like(pin)
    src = torch.empty(1 << 26, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)  # calibration copy: 256 MiB read + 256 MiB written
    for v in ("divergent", "melded", "auto", "auto", "auto"):
        k.copy_(kin)
        p.copy_(pin)
        meld.sort(k, p, variant=v)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "pairs", "copy_bytes": 2 * src.numel() * 4}))


def _profile_next(torch, np, meld, workloads, dev):
    """2^24 keys (seed 1): odd-even buckets of 2^13, then the merge sort, once per form."""
    kin = torch.from_numpy(workloads.keys_u32(SEED, 1 << 24).view(np.int32)).to(dev)
    k = torch.empty_like(kin)
    for v in ("divergent", "melded"):
        k.copy_(kin)
        meld.oddeven_sort_buckets(k, 13, variant=v)
    for v in ("divergent", "melded"):
        k.copy_(kin)
        meld.merge_sort(k, variant=v)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "next"}))


def _time_sorts(torch, np, run, restore, reps):
    ts = []
    for _ in range(reps):
        restore()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        run()
        e.record()
        e.synchronize()
        ts.append(s.elapsed_time(e))
    return float(np.median(ts))


def _bench_segmented(torch, np, meld, workloads, dev, args):
    """4096 segments, lengths log-uniform in [2^6, 2^16]: one graph replay per sort;
    per-stage forms on seed 1, MELD_AUTO and both forms on seeds 1..3 with at least
    ~1 s of sorts per seed and form."""
    out = {"segments": 4096}
    # (low form, high form, path of the phases k <= 64): lane exchanges unless
    # named "_lds"
    forms = {"divergent": ("divergent", "divergent", 1), "melded": ("melded", "melded", 1),
             "melded_low_only": ("melded", "divergent", 1),
             "melded_high_only": ("divergent", "melded", 1),
             "divergent_lds": ("divergent", "divergent", 0), "melded_lds": ("melded", "melded", 0)}
    seeds = {}
    for seed in (1, 2, 3):
        off = workloads.segment_offsets(seed, 4096)
        n = int(off[-1])
        od = torch.from_numpy(off.view(np.int32)).to(dev)
        pristine = torch.from_numpy(workloads.keys_u32(seed, n).view(np.int32)).to(dev)
        work = torch.empty_like(pristine)
        names = forms if seed == SEED else {k: forms[k] for k in ("divergent", "melded")}
        t = {name: [] for name in names}
        for rep in range(args.seg_reps + 1):
            for name, (lo, hi, x) in names.items():
                _set_path(meld, x)
                work.copy_(pristine)
                s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                s.record()
                meld.segmented_sort(work, od, low=lo, high=hi)
                e.record()
                e.synchronize()
                if rep > 0:
                    t[name].append(s.elapsed_time(e))
        _set_path(meld, -1)
        work.copy_(pristine)
        meld.segmented_sort(work, od, variant="auto")  # tunes this shape class once
        ms_auto = _time_sorts(torch, np, lambda: meld.segmented_sort(work, od, variant="auto"),
                              lambda: work.copy_(pristine), 11)
        rec = {"keys": n, "auto_ms": round(ms_auto, 4),
               "auto_Gkeys_s": round(n / (ms_auto * 1e-3) / 1e9, 3)}
        for name in names:
            rec[name + "_ms"] = _dist(np, t[name], scale=1.0)
        rec["speedup_melded"] = round(rec["divergent_ms"]["median"] / rec["melded_ms"]["median"],
                                      4)
        if "melded_lds_ms" in rec:
            rec["speedup_melded_lds_path"] = round(
                rec["divergent_lds_ms"]["median"] / rec["melded_lds_ms"]["median"], 4)
            rec["melded_lane_exchange_vs_melded_lds"] = round(
                rec["melded_lds_ms"]["median"] / rec["melded_ms"]["median"], 4)
        seeds[f"seed_{seed}"] = rec
        if seed == SEED:
            (ml, al), (mh, ah) = meld.probe_segments(od)
            out["mixed_fraction_low_phases"] = round(ml / al, 4) if al else 0.0
            out["mixed_fraction_high_phases"] = round(mh / ah, 4) if ah else 0.0
            out["low_phase_share_of_work"] = round(al / (al + ah), 4)
        meld.segmented_sort_check(0)
        del od, pristine, work
    out.update(seeds)
    out["median_speedup_melded"] = round(float(np.median(
        [seeds[f"seed_{s}"]["speedup_melded"] for s in (1, 2, 3)])), 4)
    for e in json.loads(meld.plan_describe())["entries"]:
        if e["op"] == "segsort":
            out.setdefault("tuned_plans", {})[e["key"]] = {
                "low": "melded" if e["lo"] else "divergent",
                "high": "melded" if e["hi"] else "divergent",
                "low_path": "lane_exchange" if e.get("xch") else "lds"}
    torch.cuda.empty_cache()
    return out


def _bench_serving(meld, workloads, seconds):
    """Poisson 2000 req/s, sorts 2^10..2^22 keys and region jobs 2^16..2^20 lanes (p = 0.5)."""
    from paper_2107_05681_amd import serve
    trace = workloads.serving_trace(SEED, rate=2000.0, duration_s=seconds)
    with serve.Server(budget_bytes=8 << 30, slots=8, variant="melded", table_seed=SEED,
                      table_log2=24) as srv:
        done = serve.replay(srv, trace, timeout_s=120 + 10 * seconds)
        st = srv.stats()
    summ = serve.latency_summary(done)
    return {"rate_per_s": 2000, "seconds": seconds, "jobs": summ["jobs"],
            "failed": st["failed"], "p50_ms": round(summ["p50_ms"], 3),
            "p99_ms": round(summ["p99_ms"], 3), "wait_p50_ms": round(summ["wait_p50_ms"], 3),
            "wait_p99_ms": round(summ["wait_p99_ms"], 3),
            "latency_from": "each job's scheduled Poisson arrival (submitted ahead; the server "
                            "admits it at its arrival) to its completion",
            "submit_lead_p50_ms": round(summ["submit_lead_p50_ms"], 3),
            "submit_lead_min_ms": round(summ["submit_lead_min_ms"], 3),
            "busy_fraction": round(summ["busy_fraction"], 4),
            "jobs_per_s": round(summ["jobs_per_s"], 1),
            "Gkeys_s": round(summ["keys_per_s"] / 1e9, 4),
            "Glanes_s": round(summ["lanes_per_s"] / 1e9, 4), "launches": st["launches"],
            "batched_jobs": st["batched_jobs"], "max_concurrent": st["max_concurrent"],
            "max_inflight_MB": round(st["max_inflight_bytes"] / 1e6, 1), "budget_GB": 8.6}


def _timed_repeat(fn, min_s):
    """Runs fn() until at least min_s seconds have passed (at least once);
    returns (runs, seconds)."""
    runs, t0 = 0, time.perf_counter()
    while runs == 0 or time.perf_counter() - t0 < min_s:
        fn()
        runs += 1
    return runs, time.perf_counter() - t0


def _cpu_baseline_pairs(np, workloads):
    """The CPU oracle's (key, payload) sort on this host: all the threads it may use
    (chunk sorts + pairwise merges) on 2^27 pairs, and one thread on 2^24 pairs;
    keys from seed 1, payload = index, like the GPU step."""
    import oracle

    threads = _oracle_threads()
    n_all, n_one = 1 << 27, 1 << 24
    k = workloads.keys_u32(SEED, n_all)
    v = workloads.iota_u32(n_all)
    t0 = time.perf_counter()
    oracle.sort_pairs_u32_threads(k, v, threads)
    dt_all = time.perf_counter() - t0
    k1, v1 = workloads.keys_u32(SEED, n_one), workloads.iota_u32(n_one)
    t1 = time.perf_counter()
    oracle.sort_pairs_u32(k1, v1)
    dt_one = time.perf_counter() - t1
    info = _cpu_info()
    return {"value": round(n_all / dt_all / 1e9, 4), "unit": "Gkeys/s", "cores": threads,
            "kind": "oracle",
            "one_thread_value": round(n_one / dt_one / 1e9, 4),
            "sample": f"oracle sort of 2^27 (key, payload = index) pairs, keys from seed 1, on "
                      f"{threads} host threads (chunk std::sort + pairwise std::merge): "
                      f"{dt_all:.2f} s wall; one_thread_value: oracle_sort_pairs_u32 of 2^24 "
                      f"pairs on one thread, {dt_one:.2f} s",
            "threads_note": "at most 16 threads: the host share of one GPU on this machine",
            **info}


def _cpu_sort_keys(np, workloads, n):
    """The oracle's keys sort of the 2^16-key input, one thread, repeated >= 1 s."""
    import oracle
    keys = workloads.keys_u32(SEED, n)
    runs, dt = _timed_repeat(lambda: oracle.sort_u32(keys), 1.0)
    return {"one_thread_Gkeys_s": round(runs * n / dt / 1e9, 4), "runs": runs,
            "sample": f"oracle_sort_u32 of the same 2^16 keys, {runs} runs, {dt:.2f} s"}


def _cpu_segmented(np, workloads):
    """The oracle's segmented sort of the 4096-segment input (seed 1): one thread,
    and the segments split over the threads it may use."""
    import oracle
    off = workloads.segment_offsets(SEED, 4096)
    n = int(off[-1])
    keys = workloads.keys_u32(SEED, n)
    t1 = time.perf_counter()
    oracle.segmented_sort_u32(keys, off)
    dt_one = time.perf_counter() - t1
    threads = _oracle_threads()
    cuts = np.linspace(0, 4096, threads + 1).astype(np.int64)

    def part(i):
        a, b = cuts[i], cuts[i + 1]
        lo, hi = int(off[a]), int(off[b])
        oracle.segmented_sort_u32(keys[lo:hi], (off[a:b + 1] - off[a]).astype(np.uint32))

    ts = [threading.Thread(target=part, args=(i,)) for i in range(threads)]
    t0 = time.perf_counter()
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    dt_all = time.perf_counter() - t0
    return {"Gkeys_s": round(n / dt_all / 1e9, 4), "cores": threads,
            "one_thread_Gkeys_s": round(n / dt_one / 1e9, 4),
            "sample": f"oracle_segmented_sort_u32 of the 4096 segments ({n} keys): one "
                      f"thread {dt_one:.2f} s; segments split over {threads} threads "
                      f"{dt_all:.2f} s"}


def _cpu_region(np, workloads):
    """The oracle's region over 2^24 lanes at p in {0.1, 0.5, 0.9}: lanes split over
    the threads it may use (one step), and one thread on 2^22 lanes per p."""
    import oracle

    x, tab, st, sf = workloads.region_inputs(SEED, N_LANES)
    thr = {p: workloads.thr_from_p(p) for p in PS}
    threads = _oracle_threads()
    y = np.empty_like(x)
    chunk = (N_LANES + threads - 1) // threads

    def work(p, lo, hi):
        oracle.region_f32_into(x[lo:hi], y[lo:hi], tab, SEED, thr[p], st, sf, lo)

    t0 = time.perf_counter()
    for p in PS:
        ts = [threading.Thread(target=work, args=(p, i * chunk, min(N_LANES, (i + 1) * chunk)))
              for i in range(threads)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
    dt = time.perf_counter() - t0
    one = 1 << 22
    t1 = time.perf_counter()
    for p in PS:
        work(p, 0, one)
    dt1 = time.perf_counter() - t1
    return {"G_lanes_s": round(len(PS) * N_LANES / dt / 1e9, 4), "cores": threads,
            "one_thread_G_lanes_s": round(len(PS) * one / dt1 / 1e9, 4),
            "sample": f"one step (3 x 2^24 lanes) split over {threads} threads, {dt:.2f} s; "
                      f"one thread over 2^22 lanes per p, {dt1:.2f} s"}


if __name__ == "__main__":
    main()
