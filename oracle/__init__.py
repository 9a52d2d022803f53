"""CPU oracle — TEST INFRASTRUCTURE ONLY.

Plain host implementations of what the melded kernel library computes
(sorts, the bitonic network of the paper's Figure 1, the two-sided loop
region, divergence rates). Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. It shares no code
with the GPU library; both consume inputs from ``workloads``.

The C++ source is ``oracle.cpp`` (g++ -O2 -ffp-contract=off, no fast-math).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


class SideRange(ctypes.Structure):
    _fields_ = [("a", ctypes.c_float), ("off", ctypes.c_uint32), ("step", ctypes.c_uint32),
                ("trips_lo", ctypes.c_uint32), ("trips_hi", ctypes.c_uint32)]


class Side(ctypes.Structure):
    _fields_ = [("a", ctypes.c_float), ("off", ctypes.c_uint32),
                ("step", ctypes.c_uint32), ("trips", ctypes.c_uint32)]


def build(force: bool = True) -> str:
    """Compile oracle.cpp into liboracle.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
             _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        u64, u32, sz, i64 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_size_t, ctypes.c_int64
        vp = ctypes.c_void_p
        lib.oracle_mix64.argtypes = [u64]
        lib.oracle_mix64.restype = u64
        lib.oracle_branch_hash.argtypes = [u64, u64]
        lib.oracle_branch_hash.restype = u64
        lib.oracle_sort_u32.argtypes = [vp, sz]
        lib.oracle_sort_u32.restype = None
        lib.oracle_sort_pairs_u32_threads.argtypes = [vp, vp, sz, ctypes.c_uint]
        lib.oracle_sort_pairs_u32_threads.restype = ctypes.c_int
        lib.oracle_sort_pairs_u32.argtypes = [vp, vp, sz]
        lib.oracle_sort_pairs_u32.restype = None
        lib.oracle_segmented_sort_u32.argtypes = [vp, vp, sz]
        lib.oracle_segmented_sort_u32.restype = ctypes.c_int
        lib.oracle_bitonic_num_steps.argtypes = [sz]
        lib.oracle_bitonic_num_steps.restype = u64
        lib.oracle_bitonic_emulate.argtypes = [vp, vp, sz, i64]
        lib.oracle_bitonic_emulate.restype = ctypes.c_int
        lib.oracle_region_f32.argtypes = [vp, vp, u64, sz, vp, sz, u64, u64, Side, Side]
        lib.oracle_region_f32.restype = ctypes.c_int
        lib.oracle_region3_f32.argtypes = [vp, vp, u64, sz, vp, sz, u64, u64, u64, Side, Side,
                                           Side]
        lib.oracle_region3_f32.restype = ctypes.c_int
        lib.oracle_lane_trips.argtypes = [u64, u64, u32, u32]
        lib.oracle_lane_trips.restype = u32
        lib.oracle_region_lanetrips_f32.argtypes = [vp, vp, u64, sz, vp, sz, u64, u64, SideRange,
                                                    SideRange]
        lib.oracle_region_lanetrips_f32.restype = ctypes.c_int
        lib.oracle_oddeven_emulate.argtypes = [vp, sz, i64]
        lib.oracle_oddeven_emulate.restype = ctypes.c_int
        lib.oracle_oddeven_num_comparators.argtypes = [sz]
        lib.oracle_oddeven_num_comparators.restype = u64
        lib.oracle_count_true.argtypes = [u64, u64, u64, sz]
        lib.oracle_count_true.restype = u64
        lib.oracle_mixed_waves.argtypes = [u64, u64, sz, u32]
        lib.oracle_mixed_waves.restype = u64
        lib.oracle_mixed_fraction_closed_form.argtypes = [ctypes.c_double, u32]
        lib.oracle_mixed_fraction_closed_form.restype = ctypes.c_double
        _lib = lib
    return _lib


def _u32(a) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a.copy()


def mix64(z: int) -> int:
    return int(_load().oracle_mix64(z))


def branch_hash(seed: int, i: int) -> int:
    return int(_load().oracle_branch_hash(seed, i))


def sort_u32(keys) -> np.ndarray:
    k = _u32(keys)
    _load().oracle_sort_u32(k.ctypes.data, k.size)
    return k


def sort_pairs_u32(keys, vals):
    k, v = _u32(keys), _u32(vals)
    if k.shape != v.shape:
        raise ValueError("keys and vals differ in length")
    _load().oracle_sort_pairs_u32(k.ctypes.data, v.ctypes.data, k.size)
    return k, v


def sort_pairs_u32_threads(keys, vals, threads: int):
    """sort_pairs_u32 on ``threads`` host threads (chunk sorts + pairwise merges)."""
    k, v = _u32(keys), _u32(vals)
    if k.shape != v.shape:
        raise ValueError("keys and vals differ in length")
    if _load().oracle_sort_pairs_u32_threads(k.ctypes.data, v.ctypes.data, k.size,
                                             int(threads)) != 0:
        raise ValueError("threads must be positive")
    return k, v


def segmented_sort_u32(keys, offsets) -> np.ndarray:
    k = _u32(keys)
    off = _u32(offsets)
    nseg = off.size - 1
    if nseg > 0 and int(off[-1]) > k.size:
        raise ValueError("offsets run past the key array")
    rc = _load().oracle_segmented_sort_u32(k.ctypes.data, off.ctypes.data, max(nseg, 0))
    if rc != 0:
        raise ValueError("offsets must start at 0 and be non-decreasing")
    return k


def bitonic_num_steps(n_pow2: int) -> int:
    return int(_load().oracle_bitonic_num_steps(n_pow2))


def bitonic_emulate(keys, vals=None, max_steps: int = -1):
    """Run the first ``max_steps`` steps of the Figure 1 network (all if negative)."""
    k = _u32(keys)
    v = None if vals is None else _u32(vals)
    rc = _load().oracle_bitonic_emulate(k.ctypes.data, None if v is None else v.ctypes.data,
                                        k.size, max_steps)
    if rc != 0:
        raise ValueError("length must be a power of two")
    return k if v is None else (k, v)


def _side(d) -> Side:
    return Side(float(d["a"]), int(d["off"]), int(d["step"]), int(d["trips"]))


def region_f32(x, tab, seed: int, thr: int, side_true: dict, side_false: dict,
               i0: int = 0) -> np.ndarray:
    """Lanes i0 .. i0+len(x)-1 of the two-sided loop region."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    tab = np.ascontiguousarray(tab, dtype=np.float32)
    y = np.empty_like(x)
    rc = _load().oracle_region_f32(x.ctypes.data, y.ctypes.data, i0, x.size, tab.ctypes.data,
                                   tab.size, seed, thr, _side(side_true), _side(side_false))
    if rc != 0:
        raise ValueError("table length must be a power of two and thr <= 2^32")
    return y


def region_f32_into(x: np.ndarray, y: np.ndarray, tab: np.ndarray, seed: int, thr: int,
                    side_true: dict, side_false: dict, i0: int) -> None:
    """Unchecked variant writing into a caller-owned y (used to time the oracle in chunks)."""
    _load().oracle_region_f32(x.ctypes.data, y.ctypes.data, i0, x.size, tab.ctypes.data,
                              tab.size, seed, thr, _side(side_true), _side(side_false))


def region3_f32(x, tab, seed: int, thr0: int, thr1: int, s0: dict, s1: dict, s2: dict,
                i0: int = 0) -> np.ndarray:
    """Lanes i0 .. i0+len(x)-1 of the three-way region."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    tab = np.ascontiguousarray(tab, dtype=np.float32)
    y = np.empty_like(x)
    rc = _load().oracle_region3_f32(x.ctypes.data, y.ctypes.data, i0, x.size, tab.ctypes.data,
                                    tab.size, seed, thr0, thr1, _side(s0), _side(s1), _side(s2))
    if rc != 0:
        raise ValueError("table length must be a power of two and thr0 <= thr1 <= 2^32")
    return y


def _side_range(d) -> "SideRange":
    return SideRange(float(d["a"]), int(d["off"]), int(d["step"]), int(d["trips_lo"]),
                     int(d["trips_hi"]))


def lane_trips(seed: int, i: int, lo: int, hi: int) -> int:
    return int(_load().oracle_lane_trips(seed, i, lo, hi))


def region_lanetrips_f32(x, tab, seed: int, thr: int, side_true: dict, side_false: dict,
                         i0: int = 0) -> np.ndarray:
    """Lanes i0 .. i0+len(x)-1 of the two-sided region with per-lane trip counts
    (sides given as dicts with a, off, step, trips_lo, trips_hi)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    tab = np.ascontiguousarray(tab, dtype=np.float32)
    y = np.empty_like(x)
    rc = _load().oracle_region_lanetrips_f32(x.ctypes.data, y.ctypes.data, i0, x.size,
                                             tab.ctypes.data, tab.size, seed, thr,
                                             _side_range(side_true), _side_range(side_false))
    if rc != 0:
        raise ValueError("table length must be a power of two, thr <= 2^32, lo <= hi")
    return y


def oddeven_emulate(keys, max_steps: int = -1) -> np.ndarray:
    """Batcher's odd-even merge network (its first max_steps steps) on a copy of keys."""
    k = np.array(keys, dtype=np.uint32, copy=True)
    if _load().oracle_oddeven_emulate(k.ctypes.data, k.size, max_steps) != 0:
        raise ValueError("length must be a power of two")
    return k


def oddeven_num_comparators(n: int) -> int:
    return int(_load().oracle_oddeven_num_comparators(n))


def count_true(seed: int, thr: int, n: int, i0: int = 0) -> int:
    return int(_load().oracle_count_true(seed, thr, i0, n))


def mixed_waves(seed: int, thr: int, n: int, wave: int = 64) -> int:
    return int(_load().oracle_mixed_waves(seed, thr, n, wave))


def mixed_fraction_closed_form(p: float, wave: int = 64) -> float:
    return float(_load().oracle_mixed_fraction_closed_form(p, wave))
