"""GPU parity of the two-sided loop region (both forms) against the CPU oracle.

Bar: bit-exact fp32 (every step is one correctly rounded fma on both sides,
in the same order), checked on uint32 views of the results.
"""
import ctypes

import numpy as np
import pytest

import _oracle_par
import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
meld = pytest.importorskip("paper_2107_05681_amd")

VARIANTS = ("divergent", "melded", "melded_inplace")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _run(x, tab, seed, thr, st, sf, variant):
    dev = _dev()
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(dev)
    td = torch.from_numpy(np.ascontiguousarray(tab)).to(dev)
    y = meld.divergent_region(xd, td, seed, thr, st, sf, variant=variant)
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _same_bits(a, b):
    return np.array_equal(np.asarray(a, np.float32).view(np.uint32),
                          np.asarray(b, np.float32).view(np.uint32))


TRIP_PAIRS = [(8, 8), (8, 32), (32, 8), (20, 20), (32, 32), None]


@pytest.mark.parametrize("p", [0.0, 0.1, 0.5, 0.9, 1.0])
@pytest.mark.parametrize("trips", TRIP_PAIRS)
def test_region_parity_small(p, trips):
    seed = 3
    n = (1 << 15) + 37  # many waves plus a ragged tail
    x, tab, st, sf = workloads.region_inputs(seed, n, tab_log2=18)
    if trips is not None:
        st["trips"], sf["trips"] = trips
    thr = workloads.thr_from_p(p)
    ref = oracle.region_f32(x, tab, seed, thr, st, sf)
    for v in VARIANTS:
        got = _run(x, tab, seed, thr, st, sf, v)
        assert _same_bits(got, ref), (v, p, trips)


def test_region_full_size_every_lane():
    # The timed configuration: 2^24 lanes over the 2^24-entry (64 MiB) table,
    # the seeded trip counts, p in {0.1, 0.5, 0.9}; every lane of every form
    # against the oracle.
    dev = _dev()
    seed, n = 1, 1 << 24
    x, tab, st, sf = workloads.region_inputs(seed, n)
    xd = torch.from_numpy(x).to(dev)
    td = torch.from_numpy(tab).to(dev)
    for p in (0.1, 0.5, 0.9):
        thr = workloads.thr_from_p(p)
        ref = _oracle_par.by_chunks(
            lambda s0, s1: oracle.region_f32(x[s0:s1], tab, seed, thr, st, sf, i0=s0), n)
        for v in VARIANTS:
            got = meld.divergent_region(xd, td, seed, thr, st, sf, variant=v).cpu().numpy()
            assert _same_bits(got, ref), (p, v)


def test_region_closed_form_trip_counts():
    # a = 1, tab = 1, x = 0: y equals the trip count of the lane's side.
    n = 5000
    tab = np.ones(1 << 6, np.float32)
    x = np.zeros(n, np.float32)
    st = dict(a=1.0, off=0, step=1, trips=13)
    sf = dict(a=1.0, off=32, step=3, trips=29)
    seed, thr = 7, workloads.thr_from_p(0.4)
    ones = np.array([oracle.branch_hash(seed, i) >> 32 < thr for i in range(n)])
    for v in VARIANTS:
        y = _run(x, tab, seed, thr, st, sf, v)
        assert np.array_equal(y, np.where(ones, 13.0, 29.0).astype(np.float32))


@pytest.mark.parametrize("n", [1, 63, 64, 65, 255, 257])
def test_region_edge_sizes(n):
    seed = 5
    x, tab, st, sf = workloads.region_inputs(seed, n, tab_log2=4)  # tiny table: indices wrap
    st["trips"], sf["trips"] = 0, 17  # one side does nothing
    thr = workloads.thr_from_p(0.5)
    ref = oracle.region_f32(x, tab, seed, thr, st, sf)
    for v in VARIANTS:
        assert _same_bits(_run(x, tab, seed, thr, st, sf, v), ref)


def test_region_n_zero_is_noop():
    dev = _dev()
    x = torch.empty(0, dtype=torch.float32, device=dev)
    tab = torch.ones(16, dtype=torch.float32, device=dev)
    y = meld.divergent_region(x, tab, 1, 0, meld.side(1, 0, 1, 3), meld.side(1, 0, 1, 3))
    assert y.numel() == 0


def test_region_rejects_bad_arguments():
    dev = _dev()
    x = torch.zeros(128, dtype=torch.float32, device=dev)
    s = meld.side(1, 0, 1, 3)
    with pytest.raises(meld.MeldError) as e:
        meld.divergent_region(x, torch.ones(12, dtype=torch.float32, device=dev), 1, 0, s, s)
    assert e.value.status == meld.EINVAL and "power of two" in str(e.value)
    tab = torch.ones(16, dtype=torch.float32, device=dev)
    with pytest.raises(meld.MeldError):
        meld.divergent_region(x, tab, 1, (1 << 32) + 1, s, s)
    with pytest.raises(meld.MeldError):
        meld.divergent_region(x, tab, 1, 0, meld.side(1, 0, 1, 70000), s)
    # a host pointer through the C ABI
    lib = meld.load_library()
    host = (ctypes.c_float * 128)()
    y = torch.empty_like(x)
    st = lib.meld_divergent_region_f32(meld.context(0), ctypes.cast(host, ctypes.c_void_p),
                                       ctypes.c_void_p(y.data_ptr()), 128,
                                       ctypes.c_void_p(tab.data_ptr()), 16, 1, 0, s, s, 1, None)
    assert st == meld.EINVAL


@pytest.mark.parametrize("p", [0.1, 0.5, 0.9])
def test_gathers_only_probe_reads_the_region_addresses(p):
    # meld_probe_region_gathers: every form reads exactly the region's table
    # entries; y = x ^ tab[idx_0] ^ ... ^ tab[idx_{t-1}] as bits, per the lane's
    # side (numpy, with the oracle's branch bits).
    seed, n, tab_log2 = 4, (1 << 14) + 19, 16
    x, tab, st, sf = workloads.region_inputs(seed, n, tab_log2=tab_log2)
    st["trips"], sf["trips"] = 5, 19
    thr = workloads.thr_from_p(p)
    mask = (1 << tab_log2) - 1
    taken = np.array([(oracle.branch_hash(seed, i) >> 32) < thr for i in range(n)])
    lanes = np.arange(n, dtype=np.uint64)
    tb = tab.view(np.uint32)
    want = x.view(np.uint32).copy()
    for side, sel in ((st, taken), (sf, ~taken)):
        for k in range(side["trips"]):
            idx = ((lanes + side["off"] + k * side["step"]) % (1 << 32)).astype(np.uint64) & mask
            want[sel] ^= tb[idx[sel]]
    dev = _dev()
    xd, td = torch.from_numpy(x).to(dev), torch.from_numpy(tab).to(dev)
    for v in VARIANTS:
        y = meld.divergent_region(xd, td, seed, thr, st, sf, variant=v, gathers_only=True)
        assert np.array_equal(y.cpu().numpy().view(np.uint32), want), (v, p)
