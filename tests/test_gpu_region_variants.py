"""GPU parity of the region variants against the CPU oracle: the three-way
region (if / else-if / else, the paper's SB4 pattern, melded by region
replication) and the two-sided region with per-lane trip counts.

Bar: bit-exact fp32 (one correctly rounded fma per step, the same order on
both sides), checked on uint32 views, for the divergent, melded and
melded-in-place forms and MELD_AUTO.
"""
import numpy as np
import pytest

import _oracle_par
import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
meld = pytest.importorskip("paper_2107_05681_amd")

VARIANTS = ("divergent", "melded", "melded_inplace", "auto")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                          np.asarray(b, np.float32).view(np.uint32))


def _dev_arrays(x, tab):
    dev = _dev()
    return (torch.from_numpy(np.ascontiguousarray(x)).to(dev),
            torch.from_numpy(np.ascontiguousarray(tab)).to(dev))


# ---- three-way ----------------------------------------------------------

TRIPS3 = [None, (8, 20, 32), (32, 8, 16), (5, 5, 5), (0, 7, 3), (12, 12, 30), (30, 12, 12)]
THRESH = [(1 / 3, 2 / 3), (0.1, 0.2), (0.45, 0.45), (0.0, 0.0), (1.0, 1.0), (0.0, 0.5)]


@pytest.mark.parametrize("trips", TRIPS3)
@pytest.mark.parametrize("ps", THRESH)
def test_region3_parity(trips, ps):
    seed = 4
    n = (1 << 15) + 37
    x, tab, w0, w1, w2 = workloads.region3_inputs(seed, n, tab_log2=18)
    if trips is not None:
        w0["trips"], w1["trips"], w2["trips"] = trips
    thr0, thr1 = workloads.thr_from_p(ps[0]), workloads.thr_from_p(ps[1])
    ref = oracle.region3_f32(x, tab, seed, thr0, thr1, w0, w1, w2)
    xd, td = _dev_arrays(x, tab)
    for v in VARIANTS:
        y = meld.region3(xd, td, seed, thr0, thr1, w0, w1, w2, variant=v)
        torch.cuda.synchronize()
        assert _same_bits(y.cpu().numpy(), ref), (v, trips, ps)


def test_region3_full_size_every_lane():
    # The timed configuration: 2^24 lanes over the 64 MiB table, ways a third
    # each; every lane of every form against the oracle.
    dev = _dev()
    seed, n = 1, 1 << 24
    x, tab, w0, w1, w2 = workloads.region3_inputs(seed, n)
    xd = torch.from_numpy(x).to(dev)
    td = torch.from_numpy(tab).to(dev)
    thr0, thr1 = workloads.thr_from_p(1 / 3), workloads.thr_from_p(2 / 3)
    ref = _oracle_par.by_chunks(
        lambda s0, s1: oracle.region3_f32(x[s0:s1], tab, seed, thr0, thr1, w0, w1, w2, i0=s0), n)
    for v in VARIANTS[:3]:
        got = meld.region3(xd, td, seed, thr0, thr1, w0, w1, w2, variant=v).cpu().numpy()
        assert _same_bits(got, ref), v


@pytest.mark.parametrize("n", [1, 63, 65, 257])
def test_region3_edge_sizes(n):
    seed = 6
    x, tab, w0, w1, w2 = workloads.region3_inputs(seed, n, tab_log2=4)
    w0["trips"], w1["trips"], w2["trips"] = 17, 0, 3
    thr0, thr1 = workloads.thr_from_p(0.3), workloads.thr_from_p(0.6)
    ref = oracle.region3_f32(x, tab, seed, thr0, thr1, w0, w1, w2)
    xd, td = _dev_arrays(x, tab)
    for v in VARIANTS:
        assert _same_bits(meld.region3(xd, td, seed, thr0, thr1, w0, w1, w2, variant=v).cpu(),
                          ref), (v, n)


def test_region3_rejects_bad_thresholds():
    dev = _dev()
    x = torch.zeros(64, dtype=torch.float32, device=dev)
    tab = torch.ones(16, dtype=torch.float32, device=dev)
    s = meld.side(1, 0, 1, 3)
    with pytest.raises(meld.MeldError) as e:
        meld.region3(x, tab, 1, 10, 5, s, s, s)
    assert e.value.status == meld.EINVAL
    with pytest.raises(meld.MeldError):
        meld.region3(x, tab, 1, 0, (1 << 32) + 1, s, s, s)
    with pytest.raises(meld.MeldError):
        meld.region3(x, tab, 1, 0, 0, s, s, meld.side(1, 0, 1, 70000))


# ---- per-lane trip counts --------------------------------------------------

def _ranges(loT, hiT, loF, hiF):
    return (dict(workloads.SIDE_TRUE, trips_lo=loT, trips_hi=hiT),
            dict(workloads.SIDE_FALSE, trips_lo=loF, trips_hi=hiF))


RANGES = [(8, 32, 8, 32), (8, 16, 20, 32), (10, 10, 5, 5), (0, 3, 0, 0), (1, 40, 16, 17)]


@pytest.mark.parametrize("rng_", RANGES)
@pytest.mark.parametrize("p", [0.1, 0.5, 0.9, 1.0])
def test_region_lanetrips_parity(rng_, p):
    seed = 8
    n = (1 << 15) + 11
    x, tab, _, _ = workloads.region_inputs(seed, n, tab_log2=18)
    st, sf = _ranges(*rng_)
    sf["off"] = 1 << 17
    thr = workloads.thr_from_p(p)
    ref = oracle.region_lanetrips_f32(x, tab, seed, thr, st, sf)
    xd, td = _dev_arrays(x, tab)
    for v in VARIANTS:
        y = meld.region_lanetrips(xd, td, seed, thr, st, sf, variant=v)
        torch.cuda.synchronize()
        assert _same_bits(y.cpu().numpy(), ref), (v, rng_, p)


def test_region_lanetrips_full_size_every_lane():
    # The timed configuration: 2^24 lanes, 64 MiB table, trips in [8, 32] per
    # lane on both sides, p = 0.5; every lane of every form against the oracle.
    dev = _dev()
    seed, n = 1, 1 << 24
    x, tab, _, _ = workloads.region_inputs(seed, n)
    st, sf = _ranges(8, 32, 8, 32)
    thr = workloads.thr_from_p(0.5)
    xd = torch.from_numpy(x).to(dev)
    td = torch.from_numpy(tab).to(dev)
    ref = _oracle_par.by_chunks(
        lambda s0, s1: oracle.region_lanetrips_f32(x[s0:s1], tab, seed, thr, st, sf, i0=s0), n)
    for v in VARIANTS[:3]:
        got = meld.region_lanetrips(xd, td, seed, thr, st, sf, variant=v).cpu().numpy()
        assert _same_bits(got, ref), v


def test_region_lanetrips_counts_exactly():
    # a = 1, tab = 1, x = 0: every lane's result is its own trip count.
    n = 20000
    x = np.zeros(n, np.float32)
    tab = np.ones(1 << 6, np.float32)
    st, sf = _ranges(3, 30, 12, 20)
    st["a"] = sf["a"] = 1.0
    sf["off"] = 32
    seed, thr = 9, workloads.thr_from_p(0.5)
    ref = oracle.region_lanetrips_f32(x, tab, seed, thr, st, sf)
    xd, td = _dev_arrays(x, tab)
    for v in VARIANTS[:3]:
        y = meld.region_lanetrips(xd, td, seed, thr, st, sf, variant=v).cpu().numpy()
        assert np.array_equal(y, ref)
        assert y.min() >= 3 and y.max() <= 30


def test_region_lanetrips_rejects_bad_range():
    dev = _dev()
    x = torch.zeros(64, dtype=torch.float32, device=dev)
    tab = torch.ones(16, dtype=torch.float32, device=dev)
    st, sf = _ranges(5, 4, 1, 2)
    with pytest.raises(meld.MeldError) as e:
        meld.region_lanetrips(x, tab, 1, 0, st, sf)
    assert e.value.status == meld.EINVAL
    st, sf = _ranges(1, 70000, 1, 2)
    with pytest.raises(meld.MeldError):
        meld.region_lanetrips(x, tab, 1, 0, st, sf)
