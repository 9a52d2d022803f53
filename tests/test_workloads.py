"""Checks of the seeded input generators (distribution, ranges, determinism)."""
import numpy as np

import workloads

M64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def _py_mix64(z):
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _py_hash(seed, tag, i):
    return _py_mix64((_py_mix64((seed + tag * GOLDEN) & M64) + i) & M64)


def test_known_answers_against_python_definition():
    k = workloads.keys_u32(1, 8, i0=5)
    assert k.tolist() == [_py_hash(1, 1, 5 + j) >> 32 for j in range(8)]
    x = workloads.x_f32(2, 8)
    assert x.tolist() == [float(_py_hash(2, 2, j) >> 40) * 2.0 ** -24 for j in range(8)]
    t = workloads.tab_f32(3, 8)
    assert t.tolist() == [0.5 + float(_py_hash(3, 3, j) >> 41) * 2.0 ** -24 for j in range(8)]
    assert workloads.trips(4) == (8 + _py_hash(4, 5, 0) % 25, 8 + _py_hash(4, 5, 1) % 25)


def test_key_uniformity_chi_square():
    k = workloads.keys_u32(1, 1 << 20)
    counts = np.bincount(k >> np.uint32(24), minlength=256)
    e = k.size / 256
    chi2 = float(((counts - e) ** 2 / e).sum())
    # 255 dof: mean 255, sd ~22.6; 6 sd bound
    assert chi2 < 255 + 6 * 22.6


def test_ranges():
    x = workloads.x_f32(1, 1 << 16)
    assert x.min() >= 0 and x.max() < 1
    t = workloads.tab_f32(1, 1 << 16)
    assert t.min() >= 0.5 and t.max() < 1
    for s in range(1, 50):
        tt, tf = workloads.trips(s)
        assert 8 <= tt <= 32 and 8 <= tf <= 32


def test_segment_offsets():
    off = workloads.segment_offsets(1, 4096)
    lens = np.diff(off.astype(np.int64))
    assert off[0] == 0 and lens.min() >= 64 and lens.max() <= 65536
    # log-uniform: log2(len) roughly uniform on [6, 16]
    lg = np.log2(lens)
    assert abs(lg.mean() - 11.0) < 0.2
    # E[len] = (2^16 - 2^6) / (10 ln 2) ~ 9446
    assert abs(lens.mean() - 9446) / 9446 < 0.08
    assert np.array_equal(off, workloads.segment_offsets(1, 4096))


def test_thr_from_p():
    assert workloads.thr_from_p(0.0) == 0
    assert workloads.thr_from_p(1.0) == 1 << 32
    assert workloads.thr_from_p(0.5) == 1 << 31
    assert workloads.thr_from_p(0.1) == 429496729
    assert workloads.thr_from_p(0.9) == 3865470566


def test_way_trips_extend_the_two_sides():
    for seed in (1, 2, 3, 99):
        t_true, t_false = workloads.trips(seed)
        assert workloads.way_trips(seed, 0) == t_true
        assert workloads.way_trips(seed, 1) == t_false
        assert all(8 <= workloads.way_trips(seed, w) <= 32 for w in range(3))
    x, tab, w0, w1, w2 = workloads.region3_inputs(5, 100, tab_log2=12)
    assert len(x) == 100 and len(tab) == 1 << 12
    assert (w0["off"], w1["off"], w2["off"]) == (0, 1 << 10, 1 << 11)
