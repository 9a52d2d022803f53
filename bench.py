"""Benchmark of the melded-kernel library on one MI355X.

Workload (one step): the two-sided loop region over 2^24 fp32 lanes, once
at each branch probability p in {0.1, 0.5, 0.9}, gathering from a 2^24-entry
(64 MiB) fp32 table; each side is a loop of 8..32 fma + gather steps and the
sides differ only in constants and trip count. Inputs are synthetic and
seeded (workloads/), resident in HBM before the timed region. The step runs
the library's default form (MELD_AUTO, the melded kernel).

Printed: one JSON line with the whole-step throughput (lanes/s, reported as
"Gkeys/s" with one key = one region lane), the melded/divergent speedup per
p from interleaved per-kernel timings, the roofline of the dominant kernel
(melded, p = 0.5) from HIP events on the launch stream, the bitonic sort of
2^28 (key, payload) pairs and of 2^16 keys in both forms, and the CPU oracle
timed on this host.
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
N_LANES = 1 << 24
PS = (0.1, 0.5, 0.9)
SEED = 1


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=30, help="launches per per-kernel timing")
    ap.add_argument("--no-sort", action="store_true", help="skip the sort measurements")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-seg", action="store_true", help="skip the segmented sort")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the Poisson serving trace (0 skips serving)")
    ap.add_argument("--profile", nargs="?", const="region", default=None,
                    choices=["region", "sort", "pairs", "next"],
                    help="short run for rocprofv3: 'region' (a 256 MiB copy, then a few "
                         "steps), 'sort' (2^16 keys and the 4096-segment sort, each form), "
                         "'pairs' (one 2^28-pair sort per form) or 'next' (2^24 keys: "
                         "odd-even buckets of 2^13 and the merge sort, each form)")
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


def _measured_traffic():
    """HBM bytes per launch of the melded region kernel (p = 0.5) from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs, scaled by the copy calibration; None
    when the kernel source has changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "region_melded_traffic.json")
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


def _mixed_fraction(p, wave=64):
    return 1.0 - p ** wave - (1.0 - p) ** wave


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

    if args.profile == "sort":
        _profile_sorts(torch, np, meld, workloads, dev)
        return
    if args.profile == "pairs":
        _profile_pairs(torch, np, meld, workloads, dev)
        return
    if args.profile == "next":
        _profile_next(torch, np, meld, workloads, dev)
        return
    if args.profile:
        src = torch.empty(1 << 26, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)  # calibration copy: 256 MiB read + 256 MiB written
        for _ in range(3):
            for p in PS:
                region(p, "melded")
        for p in PS:
            region(p, "divergent")
        for p in PS:
            region(p, "melded_inplace")
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "copy_bytes": 2 * src.numel() * 4}))
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_events = _events_time(torch, step, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = ms_events
    value = len(PS) * N_LANES / (ms_per_step * 1e-3) / 1e9

    # Per-kernel times, divergent and melded interleaved.
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
        e_t = p * st["trips"] + (1 - p) * sf["trips"]
        alg_bytes = N_LANES * (8 + 4 * e_t)
        per_p[str(p)] = {
            "divergent_us": round(d * 1e3, 2), "melded_us": round(m * 1e3, 2),
            "speedup": round(d / m, 4),
            "divergent_us_dist": _dist(np, td_ms), "melded_us_dist": _dist(np, tm_ms),
            "melded_inplace_us": round(mi * 1e3, 2),
            "speedup_inplace": round(d / mi, 4),
            "mixed_wave_fraction": round(_mixed_fraction(p), 5),
            "melded_alg_GBs": round(alg_bytes / (m * 1e-3) / 1e9, 1),
            "divergent_alg_GBs": round(alg_bytes / (d * 1e-3) / 1e9, 1),
        }

    # Sensitivity: the same region with both sides gathering the same entries
    # (sides differ only in multiplier and trip count), p = 0.5.
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

    # Sensitivity: other trip counts of the workload's range (8..32 per side),
    # p = 0.5, canonical sides.
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
        trips_sweep[f"{tt},{tf}"] = {"divergent_us": round(tm["divergent"] * 1e3, 2),
                                     "melded_us": round(tm["melded"] * 1e3, 2),
                                     "speedup": round(tm["divergent"] / tm["melded"], 4),
                                     "auto_us": round(tm["auto"] * 1e3, 2),
                                     "auto_form": _tuned_region_form(meld, tt, tf)}

    variants = _bench_region_variants(torch, np, meld, workloads, xd, td, ys[0.5], args)
    seeds = _bench_seeds(torch, np, meld, workloads, dev, args)

    # Roofline of the dominant kernel over the timed region itself: the step is
    # one melded launch per p, so its average launch takes ms_per_step / 3.
    alg_step = sum(N_LANES * (8 + 4 * (p * st["trips"] + (1 - p) * sf["trips"])) for p in PS)
    alg_bytes = alg_step / len(PS)
    launch_us = ms_per_step * 1e3 / len(PS)
    achieved = alg_bytes / (launch_us * 1e-6) / 1e9

    # Check the timed outputs of the step once (melded == divergent, bit for bit).
    for p in PS:
        region(p, "auto")
        a = ys[p].clone()
        for other in ("divergent", "melded_inplace"):
            region(p, other)
            if not torch.equal(a.view(torch.int32), ys[p].view(torch.int32)):
                raise SystemExit(f"melded and {other} region differ at p={p}")

    sort_info = None
    if not args.no_sort:
        sort_info = _bench_sort(torch, np, meld, workloads, dev, args)

    oddeven_info = merge_info = None
    if not args.no_sort:
        oddeven_info = _bench_oddeven(torch, np, meld, workloads, dev)
        merge_info = _bench_mergesort(torch, np, meld, workloads, dev)

    seg_info = None
    if not args.no_seg:
        seg_info = _bench_segmented(torch, np, meld, workloads, dev)

    serve_info = None
    if args.serve_seconds > 0:
        serve_info = _bench_serving(meld, workloads, args.serve_seconds)

    cpu = None
    if not args.no_cpu:
        cpu = _cpu_baseline(np, workloads, x, tab, st, sf, thr)

    out = {
        "metric": "melded/divergent speedup; Gkeys/s and VALU lane utilisation (rocprof)",
        "value": round(value, 3),
        "unit": "Gkeys/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "wall_s_timed": round(wall, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded SplitMix64 inputs, workloads/)",
        "config": {
            "workload": "divergent-region: 2^24 fp32 lanes x p in {0.1,0.5,0.9}, "
                        "branch bit Bernoulli(p) from hash(seed,i), each side 8-32 fma+gather "
                        "steps into a 2^24-entry (64 MiB) fp32 table",
            "key": "one region lane",
            "lanes_per_step": len(PS) * N_LANES,
            "trips_true": st["trips"], "trips_false": sf["trips"],
            "variant": "auto (melded)",
        },
        "melded_vs_divergent": per_p,
        "same_index_sides": same_index,
        "trips_sweep_p0.5": trips_sweep,
        "region_variants": variants,
        "seeds": seeds,
        "roofline": {
            "bound": "hbm", "kernel": "region_melded_kernel (timed step, one launch per p)",
            "avg_launch_us": round(launch_us, 2),
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": _measured_traffic(),
            "alg_bytes_per_launch": int(alg_bytes),
            "note": "algorithmic bytes count every table gather (8 + 4 t bytes per lane); "
                    "the gathers hit in L2/MALL, so frac can exceed 1; traffic is the "
                    "counter-measured HBM bytes per launch",
        },
        "sort": sort_info,
        "oddeven_buckets": oddeven_info,
        "mergesort": merge_info,
        "segmented": seg_info,
        "serving": serve_info,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


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


def _bench_sort(torch, np, meld, workloads, dev, args):
    res = {}
    # 2^28 (key, payload = index) pairs.
    n = 1 << 28
    keys = workloads.keys_u32(SEED, n)
    kin = torch.from_numpy(keys.view(np.int32)).to(dev)
    del keys
    pin = torch.arange(n, dtype=torch.int32, device=dev)
    k = torch.empty_like(kin)
    p = torch.empty_like(pin)
    times = {"divergent": [], "melded": []}
    for rep in range(4):
        for v in ("divergent", "melded"):
            k.copy_(kin)
            p.copy_(pin)
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            meld.sort(k, p, variant=v)
            e.record()
            e.synchronize()
            if rep > 0:
                times[v].append(s.elapsed_time(e))
    d, m = float(np.median(times["divergent"])), float(np.median(times["melded"]))
    plan = meld.sort_plan(n, pairs=True, variant="melded", device=0)
    passes = plan["hbm_passes"]
    moved = 16.0 * n * passes  # 8 B read + 8 B written per pair and pass
    res["pairs_2^28"] = {"divergent_ms": round(d, 3), "melded_ms": round(m, 3),
                         "speedup": round(d / m, 4),
                         "melded_Gkeys_s": round(n / (m * 1e-3) / 1e9, 3),
                         "log_tile": plan["log_tile"], "hbm_passes": passes,
                         "melded_hbm_GBs": round(moved / (m * 1e-3) / 1e9, 1),
                         "hbm_frac": round(moved / (m * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del kin, pin, k, p
    torch.cuda.empty_cache()
    # 2^16 keys.
    n = 1 << 16
    kin = torch.from_numpy(workloads.keys_u32(SEED, n).view(np.int32)).to(dev)
    k = torch.empty_like(kin)
    times = {"divergent": [], "melded": []}
    for rep in range(21):
        for v in ("divergent", "melded"):
            k.copy_(kin)
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            meld.sort(k, None, variant=v)
            e.record()
            e.synchronize()
            if rep > 0:
                times[v].append(s.elapsed_time(e))
    d, m = float(np.median(times["divergent"])), float(np.median(times["melded"]))
    # the local-sort kernel alone: the network's first t (t + 1) / 2 steps are
    # exactly that launch
    plan = meld.sort_plan(n, pairs=False, variant="melded", device=0)
    local = plan["passes"][0]["steps"]
    tl = {v: _time_sorts(torch, np, lambda v=v: meld.sort_steps(k, None, local, variant=v),
                         lambda: k.copy_(kin), 21) for v in ("divergent", "melded")}
    res["keys_2^16"] = {"divergent_us": round(d * 1e3, 2), "melded_us": round(m * 1e3, 2),
                        "speedup": round(d / m, 4),
                        "melded_Gkeys_s": round(n / (m * 1e-3) / 1e9, 3),
                        "divergent_us_dist": _dist(np, times["divergent"]),
                        "melded_us_dist": _dist(np, times["melded"]),
                        "log_tile": plan["log_tile"], "hbm_passes": plan["hbm_passes"],
                        "hbm_frac": round(8.0 * n * plan["hbm_passes"] / (m * 1e-3) / 1e9
                                          / HBM_PEAK_GBS, 5),
                        "hbm_frac_note": "not meaningful: 256 KiB per pass, the sort is bound "
                                         "by launch and per-tile latency",
                        "local_sort_kernel": {
                            "steps": local,
                            "divergent_us": round(tl["divergent"] * 1e3, 2),
                            "melded_us": round(tl["melded"] * 1e3, 2),
                            "speedup": round(tl["divergent"] / tl["melded"], 4)}}
    return res


def _profile_sorts(torch, np, meld, workloads, dev):
    """One launch sequence per form: 2^16-key sort, then the 4096-segment sort."""
    keys = torch.from_numpy(workloads.keys_u32(SEED, 1 << 16).view(np.int32)).to(dev)
    for v in ("divergent", "melded"):
        meld.sort(keys.clone(), variant=v)
    off = workloads.segment_offsets(SEED, 4096)
    od = torch.from_numpy(off.view(np.int32)).to(dev)
    seg = torch.from_numpy(workloads.keys_u32(SEED, int(off[-1])).view(np.int32)).to(dev)
    meld.set_option(0, meld.OPT_USE_GRAPHS, 0)
    for lo, hi in (("divergent", "divergent"), ("melded", "melded")):
        meld.segmented_sort(seg.clone(), od, low=lo, high=hi)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "sort"}))


def _profile_pairs(torch, np, meld, workloads, dev):
    """One 2^28-pair sort per form."""
    n = 1 << 28
    kin = torch.from_numpy(workloads.keys_u32(SEED, n).view(np.int32)).to(dev)
    pin = torch.arange(n, dtype=torch.int32, device=dev)
    k, p = torch.empty_like(kin), torch.empty_like(pin)
    for v in ("divergent", "melded"):
        k.copy_(kin)
        p.copy_(pin)
        meld.sort(k, p, variant=v)
    torch.cuda.synchronize()
    print(json.dumps({"profile_run": "pairs"}))


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


def _bench_segmented(torch, np, meld, workloads, dev):
    """4096 segments, lengths log-uniform in [2^6, 2^16]: one graph replay per sort."""
    off = workloads.segment_offsets(SEED, 4096)
    n = int(off[-1])
    od = torch.from_numpy(off.view(np.int32)).to(dev)
    pristine = torch.from_numpy(workloads.keys_u32(SEED, n).view(np.int32)).to(dev)
    work = torch.empty_like(pristine)
    forms = {"divergent": ("divergent", "divergent"), "melded": ("melded", "melded"),
             "melded_low_only": ("melded", "divergent"), "melded_high_only": ("divergent", "melded")}
    out = {"segments": 4096, "keys": n}
    for name, (lo, hi) in forms.items():
        ms = _time_sorts(torch, np, lambda: meld.segmented_sort(work, od, low=lo, high=hi),
                         lambda: work.copy_(pristine), 7)
        out[name + "_ms"] = round(ms, 4)
    work.copy_(pristine)
    meld.segmented_sort(work, od, variant="auto")  # tunes this shape class once
    ms = _time_sorts(torch, np, lambda: meld.segmented_sort(work, od, variant="auto"),
                     lambda: work.copy_(pristine), 7)
    out["auto_ms"] = round(ms, 4)
    out["auto_Gkeys_s"] = round(n / (ms * 1e-3) / 1e9, 3)
    out["speedup_melded"] = round(out["divergent_ms"] / out["melded_ms"], 4)
    (ml, al), (mh, ah) = meld.probe_segments(od)
    out["mixed_fraction_low_phases"] = round(ml / al, 4) if al else 0.0
    out["mixed_fraction_high_phases"] = round(mh / ah, 4) if ah else 0.0
    out["low_phase_share_of_work"] = round(al / (al + ah), 4)
    for e in json.loads(meld.plan_describe())["entries"]:
        if e["op"] == "segsort":
            out["tuned_plan"] = {"low": "melded" if e["lo"] else "divergent",
                                 "high": "melded" if e["hi"] else "divergent"}
    meld.segmented_sort_check(0)
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
            "busy_fraction": round(summ["busy_fraction"], 4),
            "jobs_per_s": round(summ["jobs_per_s"], 1),
            "Gkeys_s": round(summ["keys_per_s"] / 1e9, 4),
            "Glanes_s": round(summ["lanes_per_s"] / 1e9, 4), "launches": st["launches"],
            "batched_jobs": st["batched_jobs"], "max_concurrent": st["max_concurrent"],
            "max_inflight_MB": round(st["max_inflight_bytes"] / 1e6, 1), "budget_GB": 8.6}


def _cpu_baseline(np, workloads, x, tab, st, sf, thr):
    """The CPU oracle on this host: whole steps (3 x 2^24 lanes), lanes split over
    threads, repeated for at least 1 s of wall time; then one thread on a
    2^22-lane slice of each p."""
    import oracle

    threads = max(1, min(16, os.cpu_count() or 1))
    y = np.empty_like(x)
    chunk = (N_LANES + threads - 1) // threads

    def work(p, lo, hi):
        oracle.region_f32_into(x[lo:hi], y[lo:hi], tab, SEED, thr[p], st, sf, lo)

    steps = 0
    t0 = time.perf_counter()
    while steps < 3 or time.perf_counter() - t0 < 1.0:
        for p in PS:
            ts = [threading.Thread(target=work,
                                   args=(p, i * chunk, min(N_LANES, (i + 1) * chunk)))
                  for i in range(threads)]
            for t in ts:
                t.start()
            for t in ts:
                t.join()
        steps += 1
    dt = time.perf_counter() - t0
    one = 1 << 22
    t1 = time.perf_counter()
    for p in PS:
        work(p, 0, one)
    dt1 = time.perf_counter() - t1
    return {"value": round(steps * len(PS) * N_LANES / dt / 1e9, 4), "unit": "Gkeys/s",
            "cores": threads, "kind": "oracle",
            "one_thread_value": round(len(PS) * one / dt1 / 1e9, 4),
            "sample": f"{steps} full steps (3 x 2^24 lanes each, p in {{0.1,0.5,0.9}}), lanes "
                      f"split over {threads} host threads, {dt:.2f} s wall "
                      f"(~{dt * threads:.0f} s of CPU work); one_thread_value: one thread over "
                      f"2^22 lanes per p, {dt1:.2f} s"}


if __name__ == "__main__":
    main()
