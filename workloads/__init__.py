"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

This package holds no arithmetic of the method itself: it draws counter-based
SplitMix64 numbers (Steele, Lea and Flood, OOPSLA 2014) and turns them into
the inputs of each workload (sort keys, payloads, region inputs and table,
trip counts, segment lengths, serving arrivals). The definitions live in
``gen.c``; this module loads the compiled library and returns numpy arrays.

Workload recipes (the paper gives no inputs of its own; these stand in for
its bitonic-sort input of uniformly random integer keys, Evaluation section,
"Bitonic Sort (BIT)", and for its synthetic divergent-loop kernels, same
section, "Synthetic Benchmarks"):

* sort keys: ``H(seed,1,i) >> 32``, uniform u32; payload = original index.
* region: ``x[i] = (H(seed,2,i) >> 40) * 2^-24``,
  ``tab[m] = 0.5 + (H(seed,3,m) >> 41) * 2^-24`` over a 2^24-entry table,
  branch threshold ``thr = floor(p * 2^32)``, trip counts ``8 + H(seed,5,s) % 25``
  for side (way) s; the three-way region uses ways 0, 1, 2 with thresholds
  thr0 <= thr1; per-lane trip counts are drawn by the method itself (stream 11).
* segments: lengths log-uniform in ``[2^lo, 2^hi]`` from ``H(seed,6,s)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libmeldgen.so")

# Canonical side constants of the two-sided loop region (multiplier a,
# table offset, index stride). The true side reads the lower half of the
# table, the false side the upper half.
REGION_TAB_LOG2 = 24
SIDE_TRUE = dict(a=0.5, off=0, step=1031)
SIDE_FALSE = dict(a=0.75, off=1 << 23, step=2053)
# The middle way of the three-way region (if / else-if / else): ways 0, 1, 2
# are SIDE_TRUE, SIDE_MID, SIDE_FALSE.
SIDE_MID = dict(a=0.625, off=1 << 22, step=1543)

_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libmeldgen.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
             _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u64, u32, sz = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t
        vp = ctypes.c_void_p
        lib.gen_hash.argtypes = [u64, u64, u64]
        lib.gen_hash.restype = u64
        lib.gen_mix64.argtypes = [u64]
        lib.gen_mix64.restype = u64
        lib.gen_keys_u32.argtypes = [u64, u64, vp, sz]
        lib.gen_iota_u32.argtypes = [u64, vp, sz]
        lib.gen_x_f32.argtypes = [u64, u64, vp, sz]
        lib.gen_tab_f32.argtypes = [u64, vp, sz]
        lib.gen_trips.argtypes = [u64, ctypes.POINTER(u32), ctypes.POINTER(u32)]
        lib.gen_way_trips.argtypes = [u64, u32]
        lib.gen_way_trips.restype = u32
        lib.gen_segment_offsets.argtypes = [u64, u32, u32, u32, vp]
        lib.gen_segment_offsets.restype = u64
        lib.gen_uniform.argtypes = [u64, u64, u64]
        lib.gen_uniform.restype = ctypes.c_double
        _lib = lib
    return _lib


def mix64(z: int) -> int:
    return int(_load().gen_mix64(z))


def hash64(seed: int, tag: int, i: int) -> int:
    return int(_load().gen_hash(seed, tag, i))


def uniform(seed: int, tag: int, i: int) -> float:
    return float(_load().gen_uniform(seed, tag, i))


def keys_u32(seed: int, n: int, i0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _load().gen_keys_u32(seed, i0, out.ctypes.data, n)
    return out


def iota_u32(n: int, i0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.uint32)
    _load().gen_iota_u32(i0, out.ctypes.data, n)
    return out


def x_f32(seed: int, n: int, i0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.float32)
    _load().gen_x_f32(seed, i0, out.ctypes.data, n)
    return out


def tab_f32(seed: int, m: int = 1 << REGION_TAB_LOG2) -> np.ndarray:
    out = np.empty(m, dtype=np.float32)
    _load().gen_tab_f32(seed, out.ctypes.data, m)
    return out


def trips(seed: int) -> tuple[int, int]:
    t, f = ctypes.c_uint32(), ctypes.c_uint32()
    _load().gen_trips(seed, ctypes.byref(t), ctypes.byref(f))
    return int(t.value), int(f.value)


def way_trips(seed: int, way: int) -> int:
    """Trip count of way `way` of a multi-way region: 8 + H(seed, 5, way) % 25."""
    return int(_load().gen_way_trips(seed, way))


def region3_inputs(seed: int, n: int, tab_log2: int = REGION_TAB_LOG2):
    """x, tab and the three ways (dicts with a, off, step, trips) of the three-way region."""
    ways = [dict(SIDE_TRUE), dict(SIDE_MID), dict(SIDE_FALSE)]
    for w, d in enumerate(ways):
        d["trips"] = way_trips(seed, w)
    if tab_log2 != REGION_TAB_LOG2:
        ways[1]["off"] = 1 << (tab_log2 - 2)
        ways[2]["off"] = 1 << (tab_log2 - 1)
    return x_f32(seed, n), tab_f32(seed, 1 << tab_log2), ways[0], ways[1], ways[2]


def segment_offsets(seed: int, nseg: int, lo_log2: int = 6, hi_log2: int = 16) -> np.ndarray:
    out = np.empty(nseg + 1, dtype=np.uint32)
    _load().gen_segment_offsets(seed, nseg, lo_log2, hi_log2, out.ctypes.data)
    return out


def thr_from_p(p: float) -> int:
    """Integer branch threshold: lane i takes the true side iff (H(seed,4,i) >> 32) < thr."""
    if not 0.0 <= p <= 1.0:
        raise ValueError("p must lie in [0, 1]")
    return int(p * 4294967296.0)


def region_inputs(seed: int, n: int, tab_log2: int = REGION_TAB_LOG2):
    """x, tab and the two sides (dicts with a, off, step, trips) of the region workload."""
    t_true, t_false = trips(seed)
    side_t = dict(SIDE_TRUE, trips=t_true)
    side_f = dict(SIDE_FALSE, trips=t_false)
    if tab_log2 != REGION_TAB_LOG2:
        side_f["off"] = 1 << (tab_log2 - 1)
    return x_f32(seed, n), tab_f32(seed, 1 << tab_log2), side_t, side_f


def serving_trace(seed: int, rate: float, duration_s: float, sort_log2=(10, 22),
                  region_log2=(16, 20), p_region: float = 0.5, p_branch: float = 0.5,
                  tab_log2: int = REGION_TAB_LOG2):
    """Poisson arrivals of sort and region jobs (a list of dicts, arrival order).

    Job i: gap to the previous arrival -ln(1 - u7) / rate with u7 = uniform(seed, 7, i);
    kind region iff uniform(seed, 8, i) < p_region; size floor(2^(lo + (hi - lo) u9))
    with u9 = uniform(seed, 9, i); the job's own seed H(seed, 10, i) drives its input
    stream (keys or x) and, for a region job, its branch bits and trip counts.
    """
    import math
    jobs, t, i = [], 0.0, 0
    thr = thr_from_p(p_branch)
    while True:
        t += -math.log(1.0 - uniform(seed, 7, i)) / rate
        if t > duration_s:
            return jobs
        region = uniform(seed, 8, i) < p_region
        lo, hi = region_log2 if region else sort_log2
        n = int(2.0 ** (lo + (hi - lo) * uniform(seed, 9, i)))
        js = hash64(seed, 10, i)
        job = dict(arrival_s=t, kind=1 if region else 0, n=n, seed=js, thr=thr)
        if region:
            tt, tf = trips(js)
            job["side_true"] = dict(SIDE_TRUE, trips=tt)
            job["side_false"] = dict(SIDE_FALSE, trips=tf)
            if tab_log2 != REGION_TAB_LOG2:
                job["side_false"]["off"] = 1 << (tab_log2 - 1)
        jobs.append(job)
        i += 1
