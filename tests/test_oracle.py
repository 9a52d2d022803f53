"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test checks the oracle against the mathematics or a published value:
the SplitMix64 published outputs, brute force over every input of a tiny
size, the 0-1 principle for the comparator network of the paper's Figure 1
(Knuth, TAOCP vol. 3, 5.3.4), the per-phase invariant of that network,
closed forms of the two-sided loop region, exact rational arithmetic with
correct fp32 rounding, and the binomial law of the mixed-wave fraction.
"""
import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


def _py_mix64(z):
    # Written out from the published SplitMix64 definition (independent of the C code).
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _golden_splitmix():
    with open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) as f:
        return [int(l, 16) for l in f if l.strip() and not l.startswith("#")]


# --------------------------------------------------------------------------- generator


def test_mix64_matches_published_splitmix64_outputs():
    expect = _golden_splitmix()
    golden = 0x9E3779B97F4A7C15
    for n, e in enumerate(expect, start=1):
        z = (n * golden) & M64
        assert oracle.mix64(z) == e
        assert workloads.mix64(z) == e
        assert _py_mix64(z) == e


def test_branch_hash_is_tag4_stream():
    golden = 0x9E3779B97F4A7C15
    for seed in (0, 1, 7, 2**63 + 5):
        key = _py_mix64((seed + 4 * golden) & M64)
        for i in (0, 1, 63, 64, 1 << 24, (1 << 32) + 3):
            assert oracle.branch_hash(seed, i) == _py_mix64((key + i) & M64)
            assert workloads.hash64(seed, 4, i) == oracle.branch_hash(seed, i)


# --------------------------------------------------------------------------- sorts


def _is_sorted_permutation(out, inp):
    out = list(out)
    return all(a <= b for a, b in zip(out, out[1:])) and \
        sorted(out) == sorted(inp) and len(out) == len(inp)


@pytest.mark.parametrize("n", range(0, 8))
def test_sort_brute_force_all_small_inputs(n):
    # Every vector over {0,1,2} of length n (3^n inputs, duplicates included)
    # plus extreme values.
    alphabet = [0, 1, 0xFFFFFFFF] if n <= 6 else [0, 0xFFFFFFFF]
    for vec in itertools.product(alphabet, repeat=n):
        out = oracle.sort_u32(np.array(vec, dtype=np.uint32))
        assert _is_sorted_permutation(out.tolist(), vec)


def test_sort_is_unsigned():
    out = oracle.sort_u32(np.array([0x80000000, 1, 0x7FFFFFFF, 0xFFFFFFFF, 0], dtype=np.uint32))
    assert out.tolist() == [0, 1, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF]


def test_sort_pairs_composite_order_brute_force():
    rng = np.random.default_rng(5)
    for n in range(0, 7):
        for _ in range(200):
            k = rng.integers(0, 3, n).astype(np.uint32)
            v = rng.integers(0, 3, n).astype(np.uint32)
            ok, ov = oracle.sort_pairs_u32(k, v)
            pairs = list(zip(ok.tolist(), ov.tolist()))
            # lexicographic (key, payload) non-decreasing and a permutation of the input pairs
            assert all(a <= b for a, b in zip(pairs, pairs[1:]))
            assert sorted(pairs) == sorted(zip(k.tolist(), v.tolist()))


def test_sort_pairs_with_index_payload_is_stable_key_sort():
    k = workloads.keys_u32(3, 5000) % np.uint32(50)  # many ties
    v = workloads.iota_u32(5000)
    ok, ov = oracle.sort_pairs_u32(k, v)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(ov, order.astype(np.uint32))
    assert np.array_equal(ok, k[order])
    assert np.array_equal(k[ov], ok)


@pytest.mark.parametrize("threads", [1, 2, 3, 7, 16])
def test_sort_pairs_threads_is_the_stable_key_sort(threads):
    # The threaded oracle sort (chunks + pairwise merges) against numpy's stable
    # argsort, on sizes that cut into uneven chunks, with heavy ties.
    for n in (0, 1, 2, 5, 17, 1000, 40_003):
        k = workloads.keys_u32(4 + n, n) % np.uint32(37)
        v = workloads.iota_u32(n)
        ok, ov = oracle.sort_pairs_u32_threads(k, v, threads)
        order = np.argsort(k, kind="stable").astype(np.uint32)
        assert np.array_equal(ov, order), (n, threads)
        assert np.array_equal(ok, k[order]), (n, threads)


def test_sort_pairs_threads_brute_force_small():
    rng = np.random.default_rng(6)
    for n in range(0, 7):
        for _ in range(100):
            k = rng.integers(0, 3, n).astype(np.uint32)
            v = rng.integers(0, 3, n).astype(np.uint32)
            ok, ov = oracle.sort_pairs_u32_threads(k, v, 1 + n % 4)
            assert list(zip(ok.tolist(), ov.tolist())) == sorted(zip(k.tolist(), v.tolist()))
    with pytest.raises(ValueError):
        oracle.sort_pairs_u32_threads(np.zeros(3, np.uint32), np.zeros(3, np.uint32), 0)


def test_segmented_sort_respects_boundaries():
    off = np.array([0, 0, 1, 5, 5, 12, 40], dtype=np.uint32)
    keys = workloads.keys_u32(9, 40)
    out = oracle.segmented_sort_u32(keys, off)
    for s in range(len(off) - 1):
        a, b = int(off[s]), int(off[s + 1])
        seg = out[a:b].tolist()
        assert _is_sorted_permutation(seg, keys[a:b].tolist())


def test_segmented_sort_rejects_bad_offsets():
    keys = np.zeros(10, dtype=np.uint32)
    with pytest.raises(ValueError):
        oracle.segmented_sort_u32(keys, np.array([0, 5, 3, 10], dtype=np.uint32))
    with pytest.raises(ValueError):
        oracle.segmented_sort_u32(keys, np.array([1, 5, 10], dtype=np.uint32))
    out = oracle.segmented_sort_u32(keys, np.array([0], dtype=np.uint32))
    assert out.size == 10


# --------------------------------------------------------------------------- Figure 1 network


def test_bitonic_step_count():
    # log2(N) (log2(N) + 1) / 2 steps
    for p in range(0, 12):
        assert oracle.bitonic_num_steps(1 << p) == p * (p + 1) // 2


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_bitonic_zero_one_principle(n):
    # A comparator network sorts every input iff it sorts every 0/1 input.
    for bits in range(1 << n):
        vec = np.array([(bits >> b) & 1 for b in range(n)], dtype=np.uint32)
        out = oracle.bitonic_emulate(vec)
        ones = int(vec.sum())
        assert out.tolist() == [0] * (n - ones) + [1] * ones


def test_bitonic_emulator_equals_sort_random():
    for p in (1, 5, 10, 12):
        n = 1 << p
        k = workloads.keys_u32(p, n)
        v = workloads.iota_u32(n)
        assert np.array_equal(oracle.bitonic_emulate(k), np.sort(k))
        ek, ev = oracle.bitonic_emulate(k, v)
        order = np.argsort(k, kind="stable")
        assert np.array_equal(ek, k[order]) and np.array_equal(ev, order.astype(np.uint32))


def test_bitonic_pairs_heavy_ties():
    n = 256
    k = workloads.keys_u32(4, n) % np.uint32(4)
    v = (workloads.keys_u32(5, n) % np.uint32(3)).astype(np.uint32)
    ek, ev = oracle.bitonic_emulate(k, v)
    pairs = list(zip(ek.tolist(), ev.tolist()))
    assert pairs == sorted(zip(k.tolist(), v.tolist()))


def test_bitonic_phase_invariant():
    # After phase k (all steps j = k/2 .. 1), block b of size k is sorted
    # ascending when b is even and descending when b is odd, since the
    # direction of element i in phase k is given by bit k of i.
    p = 8
    n = 1 << p
    k0 = workloads.keys_u32(11, n)
    steps = 0
    for lk in range(1, p + 1):
        steps += lk
        out = oracle.bitonic_emulate(k0, max_steps=steps)
        kk = 1 << lk
        for b in range(n // kk):
            blk = out[b * kk:(b + 1) * kk]
            ref = np.sort(blk)
            if b % 2 == 0:
                assert np.array_equal(blk, ref)
            else:
                assert np.array_equal(blk, ref[::-1])
        # blocks hold the same multisets as the input blocks (no element crossed a k-block)
        for b in range(n // kk):
            assert np.array_equal(np.sort(out[b * kk:(b + 1) * kk]), np.sort(k0[b * kk:(b + 1) * kk]))


def test_bitonic_first_step_is_one_comparator_layer():
    # Step 1 (k = 2, j = 1): pairs (2m, 2m+1), ascending for even m, descending for odd m.
    k0 = np.array([5, 3, 1, 9, 7, 7, 8, 2], dtype=np.uint32)
    out = oracle.bitonic_emulate(k0, max_steps=1)
    assert out.tolist() == [3, 5, 9, 1, 7, 7, 8, 2]


def test_bitonic_rejects_non_pow2():
    with pytest.raises(ValueError):
        oracle.bitonic_emulate(np.zeros(6, dtype=np.uint32))


# --------------------------------------------------------------------------- region


def _sides(tT, tF, aT=0.5, aF=0.75, offF=1 << 9, stepT=1031, stepF=2053):
    return (dict(a=aT, off=0, step=stepT, trips=tT), dict(a=aF, off=offF, step=stepF, trips=tF))


def _taken(seed, thr, i):
    golden = 0x9E3779B97F4A7C15
    h = _py_mix64((_py_mix64((seed + 4 * golden) & M64) + i) & M64)
    return (h >> 32) < thr


def test_region_geometric_closed_form():
    # a = 1/2, tab = 1, x = 0: acc_t = 2 - 2^(1-t), exact in fp32 for t <= 24.
    n = 130
    tab = np.ones(1 << 10, dtype=np.float32)
    x = np.zeros(n, dtype=np.float32)
    for t in (0, 1, 2, 5, 24):
        st, sf = _sides(t, t, aT=0.5, aF=0.5)
        y = oracle.region_f32(x, tab, seed=1, thr=1 << 31, side_true=st, side_false=sf)
        expect = np.float32(2.0 - 2.0 ** (1 - t)) if t else np.float32(0.0)
        assert np.all(y == expect)


def test_region_index_formula_with_zero_multiplier():
    # a = 0: fma(acc, 0, g) = g, so y is the table entry of the last step;
    # tab[m] = m makes y the index itself.
    L = 12
    tab = np.arange(1 << L, dtype=np.float32)
    n = 300
    x = workloads.x_f32(2, n)
    st, sf = _sides(7, 13, aT=0.0, aF=0.0, offF=1 << (L - 1), stepT=1031, stepF=2053)
    seed, thr = 3, 1 << 31
    i0 = (1 << 32) - 150  # lane indices cross 2^32: index arithmetic wraps modulo 2^32
    y = oracle.region_f32(x, tab, seed=seed, thr=thr, side_true=st, side_false=sf, i0=i0)
    for j in range(n):
        i = i0 + j
        s = st if _taken(seed, thr, i) else sf
        idx = (i + s["off"] + (s["trips"] - 1) * s["step"]) % (1 << 32) % (1 << L)
        assert y[j] == np.float32(idx)


def test_region_trip_count_and_side_selection():
    # a = 1, tab = 1, x = 0: y = number of steps of the lane's side, exactly.
    n = 4096
    tab = np.ones(1 << 8, dtype=np.float32)
    x = np.zeros(n, dtype=np.float32)
    st, sf = _sides(9, 31, aT=1.0, aF=1.0, offF=128)
    seed, thr = 17, workloads.thr_from_p(0.3)
    y = oracle.region_f32(x, tab, seed=seed, thr=thr, side_true=st, side_false=sf)
    expect = np.array([9.0 if _taken(seed, thr, i) else 31.0 for i in range(n)], dtype=np.float32)
    assert np.array_equal(y, expect)
    # thr = 0: every lane false; thr = 2^32: every lane true
    assert np.all(oracle.region_f32(x, tab, 17, 0, st, sf) == 31.0)
    assert np.all(oracle.region_f32(x, tab, 17, 1 << 32, st, sf) == 9.0)


def _round_f32(v: Fraction) -> np.float32:
    """Correctly rounded (nearest, ties to even) fp32 of an exact rational."""
    if v == 0:
        return np.float32(0.0)
    c = np.float32(float(v))
    cands = [np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))]
    best = None
    for cand in cands:
        err = abs(Fraction(float(cand)) - v)
        key = (err, int(np.array(cand, dtype=np.float32).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, cand)
    return np.float32(best[1])


def test_region_matches_exact_rational_fma():
    # Each step is one correctly rounded fused multiply-add acc*a + g:
    # recompute with exact rationals and round once per step.
    L = 12
    seed, thr = 23, workloads.thr_from_p(0.5)
    tab = workloads.tab_f32(seed, 1 << L)
    n = 96
    x = workloads.x_f32(seed, n)
    st, sf = _sides(11, 6, aT=0.5, aF=0.75, offF=1 << (L - 1))
    st["a"] = 0.8125  # exercise rounding in the product too
    sf["a"] = 1.3
    y = oracle.region_f32(x, tab, seed=seed, thr=thr, side_true=st, side_false=sf)
    for i in range(n):
        s = st if _taken(seed, thr, i) else sf
        a = Fraction(float(np.float32(s["a"])))
        acc = np.float32(x[i])
        for k in range(s["trips"]):
            idx = (i + s["off"] + k * s["step"]) % (1 << L)
            acc = _round_f32(Fraction(float(acc)) * a + Fraction(float(tab[idx])))
        assert y[i] == acc, (i, y[i], acc)


def test_region_fma_is_not_two_roundings():
    # acc = a = 1 + 2^-12, g = -1: the exact acc*a + g = 2^-11 + 2^-24 is an
    # fp32 number, while rounding the product first gives 2^-11.
    acc0 = np.float32(1 + 2**-12)
    tab = np.full(4, -1.0, dtype=np.float32)
    side = dict(a=float(acc0), off=0, step=1, trips=1)
    y = oracle.region_f32(np.array([acc0], dtype=np.float32), tab, 0, 1 << 32, side, side)
    assert y[0] == np.float32(2**-11 + 2**-24)
    two_roundings = np.float32(np.float32(acc0 * acc0) - np.float32(1.0))
    assert two_roundings == np.float32(2**-11) and y[0] != two_roundings


def test_region_rejects_bad_table():
    with pytest.raises(ValueError):
        oracle.region_f32(np.zeros(4, np.float32), np.ones(6, np.float32), 0, 0,
                          *_sides(1, 1))
    with pytest.raises(ValueError):
        oracle.region_f32(np.zeros(4, np.float32), np.ones(8, np.float32), 0, (1 << 32) + 1,
                          *_sides(1, 1))


# --------------------------------------------------------------------------- divergence rate


def test_branch_rate_binomial():
    n = 1 << 20
    for p in (0.1, 0.5, 0.9):
        thr = workloads.thr_from_p(p)
        c = oracle.count_true(1, thr, n)
        sd = (n * p * (1 - p)) ** 0.5
        assert abs(c - n * p) < 6 * sd


def test_mixed_waves_extremes_and_closed_form():
    n = 1 << 18
    assert oracle.mixed_waves(1, 0, n) == 0
    assert oracle.mixed_waves(1, 1 << 32, n) == 0
    for p in (0.02, 0.1, 0.5, 0.9):
        thr = workloads.thr_from_p(p)
        waves = n // 64
        got = oracle.mixed_waves(1, thr, n) / waves
        q = oracle.mixed_fraction_closed_form(p)
        assert abs(q - (1 - p ** 64 - (1 - p) ** 64)) < 1e-12
        sd = (q * (1 - q) / waves) ** 0.5
        assert abs(got - q) < 6 * sd + 1e-9
    # every configured p gives more than half of the waves mixed
    for p in (0.1, 0.5, 0.9):
        assert oracle.mixed_fraction_closed_form(p) > 0.5


def test_mixed_waves_brute_force_small():
    for seed in (1, 2):
        thr = workloads.thr_from_p(0.05)
        n = 64 * 40 + 17  # ragged last wave
        bits = [_taken(seed, thr, i) for i in range(n)]
        mixed = 0
        for b in range(0, n, 64):
            w = bits[b:b + 64]
            mixed += 1 if (any(w) and not all(w)) else 0
        assert oracle.mixed_waves(seed, thr, n) == mixed


# ---- three-way region (SB4-like) -------------------------------------------

def _side3(seed, thr0, thr1, i):
    golden = 0x9E3779B97F4A7C15
    h = _py_mix64((_py_mix64((seed + 4 * golden) & M64) + i) & M64) >> 32
    return 0 if h < thr0 else (1 if h < thr1 else 2)


def _three_sides(t0, t1, t2, a=(0.5, 0.625, 0.75)):
    return (dict(a=a[0], off=0, step=1031, trips=t0), dict(a=a[1], off=1 << 8, step=1543, trips=t1),
            dict(a=a[2], off=1 << 9, step=2053, trips=t2))


def test_region3_reduces_to_the_two_way_region():
    # With one of the three ways empty the chain is the two-sided region.
    L = 12
    seed = 29
    tab = workloads.tab_f32(seed, 1 << L)
    x = workloads.x_f32(seed, 700)
    s0, s1, s2 = _three_sides(7, 12, 9)
    t_lo, t_hi = workloads.thr_from_p(0.3), workloads.thr_from_p(0.7)
    # thr1 = 2^32: side 2 never taken
    assert np.array_equal(oracle.region3_f32(x, tab, seed, t_lo, 1 << 32, s0, s1, s2),
                          oracle.region_f32(x, tab, seed, t_lo, s0, s1))
    # thr0 = 0: side 0 never taken
    assert np.array_equal(oracle.region3_f32(x, tab, seed, 0, t_hi, s0, s1, s2),
                          oracle.region_f32(x, tab, seed, t_hi, s1, s2))
    # thr0 = thr1: the middle way is never taken (the biased three-way case)
    assert np.array_equal(oracle.region3_f32(x, tab, seed, t_lo, t_lo, s0, s1, s2),
                          oracle.region_f32(x, tab, seed, t_lo, s0, s2))


def test_region3_trip_count_and_side_selection():
    # a = 1, tab = 1, x = 0: y is the trip count of the lane's way, exactly;
    # the way follows the if / else-if / else order of the two thresholds.
    n = 4096
    tab = np.ones(1 << 8, dtype=np.float32)
    x = np.zeros(n, dtype=np.float32)
    s0, s1, s2 = _three_sides(5, 9, 17, a=(1.0, 1.0, 1.0))
    seed, thr0, thr1 = 31, workloads.thr_from_p(0.25), workloads.thr_from_p(0.6)
    y = oracle.region3_f32(x, tab, seed, thr0, thr1, s0, s1, s2)
    trips = (5.0, 9.0, 17.0)
    expect = np.array([trips[_side3(seed, thr0, thr1, i)] for i in range(n)], dtype=np.float32)
    assert np.array_equal(y, expect)
    counts = [int(np.sum(y == t)) for t in trips]
    assert counts[0] == oracle.count_true(seed, thr0, n)
    assert counts[0] + counts[1] == oracle.count_true(seed, thr1, n)


def test_region3_index_formula_with_zero_multiplier():
    L = 12
    tab = np.arange(1 << L, dtype=np.float32)
    n = 300
    x = workloads.x_f32(2, n)
    s0, s1, s2 = _three_sides(7, 13, 4, a=(0.0, 0.0, 0.0))
    seed, thr0, thr1 = 3, 1 << 30, 3 << 30
    i0 = (1 << 32) - 150  # lane indices cross 2^32: index arithmetic wraps modulo 2^32
    y = oracle.region3_f32(x, tab, seed, thr0, thr1, s0, s1, s2, i0=i0)
    for j in range(n):
        i = i0 + j
        s = (s0, s1, s2)[_side3(seed, thr0, thr1, i)]
        idx = (i + s["off"] + (s["trips"] - 1) * s["step"]) % (1 << 32) % (1 << L)
        assert y[j] == np.float32(idx)


def test_region3_rejects_bad_thresholds():
    tab = np.ones(16, dtype=np.float32)
    x = np.zeros(4, dtype=np.float32)
    s0, s1, s2 = _three_sides(1, 2, 3)
    with pytest.raises(ValueError):
        oracle.region3_f32(x, tab, 1, 5, 4, s0, s1, s2)  # thr0 > thr1
    with pytest.raises(ValueError):
        oracle.region3_f32(x, tab, 1, 0, (1 << 32) + 1, s0, s1, s2)
    with pytest.raises(ValueError):
        oracle.region3_f32(x, np.ones(12, dtype=np.float32), 1, 0, 1, s0, s1, s2)


# ---- per-lane trip counts --------------------------------------------------

def test_lane_trips_is_tag11_stream_and_covers_its_range():
    golden = 0x9E3779B97F4A7C15
    seed, lo, hi = 7, 8, 32
    vals = [oracle.lane_trips(seed, i, lo, hi) for i in range(5000)]
    for i in (0, 1, 2, 4999):
        h = _py_mix64((_py_mix64((seed + 11 * golden) & M64) + i) & M64) >> 32
        assert vals[i] == lo + h % (hi - lo + 1)
    assert min(vals) == lo and max(vals) == hi
    assert set(vals) == set(range(lo, hi + 1))
    # a degenerate range is a constant
    assert all(oracle.lane_trips(seed, i, 9, 9) == 9 for i in range(50))


def _range_sides(loT, hiT, loF, hiF, aT=0.5, aF=0.75):
    return (dict(a=aT, off=0, step=1031, trips_lo=loT, trips_hi=hiT),
            dict(a=aF, off=1 << 9, step=2053, trips_lo=loF, trips_hi=hiF))


def test_lanetrips_with_fixed_trips_is_the_region():
    L = 12
    seed = 41
    tab = workloads.tab_f32(seed, 1 << L)
    x = workloads.x_f32(seed, 500)
    thr = workloads.thr_from_p(0.4)
    rt, rf = _range_sides(11, 11, 6, 6)
    st, sf = _sides(11, 6, offF=1 << 9)
    assert np.array_equal(oracle.region_lanetrips_f32(x, tab, seed, thr, rt, rf),
                          oracle.region_f32(x, tab, seed, thr, st, sf))


def test_lanetrips_counts_per_lane():
    # a = 1, tab = 1, x = 0: y is the lane's own trip count, drawn in its
    # side's range.
    n = 3000
    tab = np.ones(1 << 8, dtype=np.float32)
    x = np.zeros(n, dtype=np.float32)
    rt, rf = _range_sides(8, 16, 20, 32, aT=1.0, aF=1.0)
    seed, thr = 43, workloads.thr_from_p(0.5)
    y = oracle.region_lanetrips_f32(x, tab, seed, thr, rt, rf)
    for i in range(n):
        s = rt if _taken(seed, thr, i) else rf
        assert y[i] == np.float32(oracle.lane_trips(seed, i, s["trips_lo"], s["trips_hi"]))
        assert s["trips_lo"] <= y[i] <= s["trips_hi"]
    with pytest.raises(ValueError):
        oracle.region_lanetrips_f32(x, tab, seed, thr, _range_sides(5, 4, 1, 2)[0], rf)


# ---- Batcher's odd-even merge network (PCM) ----------------------------------

def test_oddeven_comparator_count_closed_form():
    # Knuth, TAOCP vol. 3, 5.3.4: Batcher's odd-even merge sort uses
    # (t^2 - t + 4) 2^(t-2) - 1 comparators on n = 2^t elements.
    for t in range(1, 13):
        expect = ((t * t - t + 4) << t) // 4 - 1
        assert oracle.oddeven_num_comparators(1 << t) == expect, t


@pytest.mark.parametrize("n", [2, 4, 8, 16])
def test_oddeven_zero_one_principle(n):
    # Sorting every 0-1 input proves a comparator network sorts (Knuth 5.3.4).
    v = np.arange(1 << n, dtype=np.uint32)
    bits = ((v[:, None] >> np.arange(n, dtype=np.uint32)) & 1).astype(np.uint32)
    for row in bits:
        out = oracle.oddeven_emulate(row)
        assert np.all(out[:-1] <= out[1:])


def test_oddeven_hand_worked_four_elements():
    # n = 4: steps (p, k) = (1, 1): (0,1) (2,3); (2, 2): (0,2) (1,3); (2, 1): (1,2).
    x = np.array([3, 2, 1, 0], np.uint32)
    assert oracle.oddeven_emulate(x, 1).tolist() == [2, 3, 0, 1]
    assert oracle.oddeven_emulate(x, 2).tolist() == [0, 1, 2, 3]
    y = np.array([0, 2, 1, 3], np.uint32)  # only the last comparator (1, 2) acts
    assert oracle.oddeven_emulate(y, 2).tolist() == [0, 2, 1, 3]
    assert oracle.oddeven_emulate(y, 3).tolist() == [0, 1, 2, 3]


def test_oddeven_sorts_random_and_step_count():
    for log_n in (5, 10, 13):
        n = 1 << log_n
        keys = workloads.keys_u32(50 + log_n, n)
        steps = log_n * (log_n + 1) // 2
        out = oracle.oddeven_emulate(keys)
        assert np.array_equal(out, np.sort(keys))
        assert np.array_equal(oracle.oddeven_emulate(keys, steps), out)
        assert np.array_equal(oracle.oddeven_emulate(keys, steps + 7), out)
        assert not np.array_equal(oracle.oddeven_emulate(keys, steps - 1), out)
    with pytest.raises(ValueError):
        oracle.oddeven_emulate(np.zeros(12, np.uint32))
