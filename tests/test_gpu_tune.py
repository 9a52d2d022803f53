"""GPU checks of the divergence probes and the autotuner (MELD_AUTO)."""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
meld = pytest.importorskip("paper_2107_05681_amd")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(_dev())


@pytest.mark.parametrize("n", [1, 64, 1000, (1 << 18) + 7])
@pytest.mark.parametrize("p", [0.0, 0.02, 0.5, 0.9, 1.0])
def test_region_probe_matches_oracle(n, p):
    _dev()
    thr = workloads.thr_from_p(p)
    mixed, ones, waves = meld.probe_region(n, 3, thr)
    assert mixed == oracle.mixed_waves(3, thr, n)
    assert ones == oracle.count_true(3, thr, n)
    assert waves == (n + 63) // 64


def _network_brute(log_t):
    half = 1 << (log_t - 1)
    res = []
    for m in range(1, log_t + 1):
        mixed = waves = 0
        for jb in range(m):
            j = 1 << jb
            c = np.arange(half, dtype=np.int64)
            lo = ((c & ~(j - 1)) << 1) | (c & (j - 1))
            up = ((lo >> m) & 1) == 0
            for w in range(0, half, 64):
                u = up[w:w + 64]
                mixed += int(u.any() and not u.all())
                waves += 1
        res.append((mixed, waves))
    return res


@pytest.mark.parametrize("log_t", [1, 3, 7, 10, 13])
def test_network_probe_matches_brute_force(log_t):
    _dev()
    got = meld.probe_network(log_t)
    assert got == _network_brute(log_t)
    # closed form: the direction is lane-divergent exactly in the phases k <= 64
    # (below a full wave of comparators every phase but the last)
    for m, (mixed, waves) in enumerate(got, start=1):
        if (1 << m) <= 64 and m < log_t:
            assert mixed == waves
        else:
            assert mixed == 0


def _segments_brute(lengths):
    # The segmented kernel's lane mapping, written out with numpy: one wave of
    # 64 consecutive comparators per segment of <= 128 keys; otherwise chunks
    # of 2^cm keys (cm = min(class, 14)) sorted by a team of nt = 2^(cm-4)
    # lanes that deals comparators t + i*nt in phases <= 2^6 and holds 16 keys
    # per lane (direction: lane bit p-4) in the register phases.
    acc = [0, 0, 0, 0]
    for ln in lengths:
        if ln <= 1:
            continue
        log_p = int(np.ceil(np.log2(ln)))
        half = 1 << (log_p - 1)
        cm = min(log_p, 14)
        nt = 1 << max(cm - 4, 0)
        chunks = 1 << (log_p - cm)
        for m in range(1, log_p + 1):
            mixed_cmp = 0
            if log_p <= 7:
                c = np.arange(half)
                up = ((c >> (m - 1)) & 1) == 0
                for w in range(0, half, 64):
                    u = up[w:w + 64]
                    if u.any() and not u.all():
                        mixed_cmp += u.size
            elif m <= cm:
                t = np.arange(nt)
                if m <= 6:
                    for i in range((1 << (cm - 1)) // nt):
                        up = (((t + i * nt) >> (m - 1)) & 1) == 0
                        for w in range(0, nt, 64):
                            u = up[w:w + 64]
                            if u.any() and not u.all():
                                mixed_cmp += u.size
                else:
                    up = ((t >> (m - 4)) & 1) == 0
                    for w in range(0, nt, 64):
                        u = up[w:w + 64]
                        if u.any() and not u.all():
                            mixed_cmp += 8 * u.size
                mixed_cmp *= chunks
            stage = 0 if (1 << m) <= 64 else 2
            acc[stage] += m * mixed_cmp
            acc[stage + 1] += m * half
    return (acc[0], acc[1]), (acc[2], acc[3])


def test_segments_probe_matches_brute_force():
    lengths = [0, 1, 2, 3, 64, 65, 100, 128, 129, 300, 600, 1000, 4096, 16384, 20000, 40000,
               65536]
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint32)
    assert meld.probe_segments(_to_dev(off)) == _segments_brute(lengths)


def test_auto_results_match_oracle_and_plans_are_recorded(tmp_path):
    dev = _dev()
    cache = str(tmp_path / "tune.json")
    meld.tune(cache)
    # single-array sort, pairs, multi-tile
    n = (1 << 16) + 3
    keys = workloads.keys_u32(21, n)
    vals = workloads.iota_u32(n)
    rk, rv = oracle.sort_pairs_u32(keys, vals)
    kd, vd = _to_dev(keys), _to_dev(vals)
    meld.sort(kd, vd, variant="auto")
    torch.cuda.synchronize()
    assert np.array_equal(kd.cpu().numpy().view(np.uint32), rk)
    assert np.array_equal(vd.cpu().numpy().view(np.uint32), rv)
    # segmented
    off = workloads.segment_offsets(4, 300)
    sk = workloads.keys_u32(4, int(off[-1]))
    sd = _to_dev(sk)
    meld.segmented_sort(sd, _to_dev(off), variant="auto")
    torch.cuda.synchronize()
    meld.segmented_sort_check(0)
    assert np.array_equal(sd.cpu().numpy().view(np.uint32), oracle.segmented_sort_u32(sk, off))
    # region
    x, tab, st, sf = workloads.region_inputs(5, 1 << 16, tab_log2=16)
    thr = workloads.thr_from_p(0.5)
    y = meld.divergent_region(torch.from_numpy(x).to(dev), torch.from_numpy(tab).to(dev), 5, thr,
                              st, sf, variant="auto")
    assert np.array_equal(y.cpu().numpy().view(np.uint32),
                          oracle.region_f32(x, tab, 5, thr, st, sf).view(np.uint32))
    desc = json.loads(meld.plan_describe())
    ops = {e["op"] for e in desc["entries"]}
    assert {"sort", "segsort", "region"} <= ops
    for e in desc["entries"]:
        # the ops with two forms only (entries left by earlier tests of the
        # same context) time two candidates, the others at least three
        assert e["trials"] >= (2 if e["op"] in ("oddeven", "mergesort") else 3) and e["ms"] > 0
        if e["op"] == "segsort":
            # fractions of mixed comparator-steps per stage (the probe itself is
            # pinned against brute force in test_segments_probe_matches_brute_force)
            assert 0.0 <= e["mixed_lo"] <= 1.0 and 0.0 <= e["mixed_hi"] <= 1.0
    # the cache file round-trips into a fresh context without re-tuning
    saved = json.load(open(cache))
    assert len(saved["entries"]) == len(desc["entries"])
    lib = meld.load_library()
    ctx2 = ctypes.c_void_p()
    assert lib.meld_create(0, ctypes.byref(ctx2)) == meld.OK
    try:
        assert lib.meld_tune(ctx2, cache.encode()) == meld.OK
        buf = ctypes.create_string_buffer(1 << 16)
        assert lib.meld_plan_describe(ctx2, buf, len(buf)) == meld.OK
        again = json.loads(buf.value.decode())
        assert again["entries"] == saved["entries"]
    finally:
        lib.meld_destroy(ctx2)


def test_malformed_cache_is_rejected(tmp_path):
    _dev()
    bad = tmp_path / "bad.json"
    bad.write_text('{"version": 1, "arch": "x", "runtime": 1, "entries": [\n{"op": "sort", "key": 5}\n]}\n')
    lib = meld.load_library()
    ctx2 = ctypes.c_void_p()
    assert lib.meld_create(0, ctypes.byref(ctx2)) == meld.OK
    try:
        assert lib.meld_tune(ctx2, str(bad).encode()) == meld.EINVAL
    finally:
        lib.meld_destroy(ctx2)


def test_forced_variants_bypass_the_tuner():
    _dev()
    before = json.loads(meld.plan_describe())["entries"]
    n = 5000
    keys = workloads.keys_u32(9, n)
    kd = _to_dev(keys)
    meld.sort(kd, variant="divergent")
    torch.cuda.synchronize()
    assert np.array_equal(kd.cpu().numpy().view(np.uint32), np.sort(keys))
    assert json.loads(meld.plan_describe())["entries"] == before
