"""GPU parity of the bottom-up merge sort (the paper's MS benchmark), divergent
and melded merge steps, against the CPU oracle. Bar: bit-exact (sorted u32
keys are unique); after every number of merge passes each run equals the
oracle's sort of that segment (merging two sorted runs has one result, their
sorted union)."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
meld = pytest.importorskip("paper_2107_05681_amd")

VARIANTS = ("divergent", "melded", "auto")


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(_dev())


def _host(t):
    return t.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("n", [2, 1000, 1024, 1025, 2048, 5000, (1 << 16) + 3, 3 * (1 << 18) + 7,
                               1 << 20])
def test_merge_sort_sizes(n):
    keys = workloads.keys_u32(90, n)
    ref = oracle.sort_u32(keys)
    for v in VARIANTS:
        kd = _to_dev(keys)
        meld.merge_sort(kd, variant=v)
        torch.cuda.synchronize()
        assert np.array_equal(_host(kd), ref), (n, v)


@pytest.mark.parametrize("n", [(1 << 14) + 100, 1 << 15])
def test_merge_sort_pass_parity(n):
    keys = workloads.keys_u32(91, n)
    p = 0
    while (1 << (10 + p)) < n * 2:
        run = 1 << (10 + p)
        off = np.array(list(range(0, n, run)) + [n], np.uint32)
        ref = oracle.segmented_sort_u32(keys, off)
        for v in ("divergent", "melded"):
            kd = _to_dev(keys)
            meld.merge_sort(kd, max_passes=p, variant=v)
            torch.cuda.synchronize()
            assert np.array_equal(_host(kd), ref), (n, p, v)
        p += 1


def test_merge_sort_ties_and_extremes():
    n = (1 << 17) + 5
    keys = (workloads.keys_u32(92, n) % np.uint32(4)).astype(np.uint32)
    keys[::41] = 0xFFFFFFFF
    keys[::43] = 0
    ref = oracle.sort_u32(keys)
    for v in VARIANTS:
        kd = _to_dev(keys)
        meld.merge_sort(kd, variant=v)
        torch.cuda.synchronize()
        assert np.array_equal(_host(kd), ref), v


def test_merge_sort_large_against_oracle():
    n = 1 << 22
    keys = workloads.keys_u32(93, n)
    ref = oracle.sort_u32(keys)
    for v in ("divergent", "melded"):
        kd = _to_dev(keys)
        meld.merge_sort(kd, variant=v)
        torch.cuda.synchronize()
        assert np.array_equal(_host(kd), ref), v


def test_merge_sort_with_cut_kernel_against_oracle():
    # More than 2048 tiles of 2048 keys: the passes of runs >= 2^11 take their
    # merge-path cuts from the separate cut kernel (8-way search); a ragged
    # last pair in every pass, and heavy ties (keys drawn from 64 values).
    n = (1 << 22) + (1 << 21) + 13
    keys = workloads.keys_u32(94, n)
    for k in (keys, keys & np.uint32(63)):
        ref = oracle.sort_u32(k)
        for v in ("divergent", "melded"):
            kd = _to_dev(k)
            meld.merge_sort(kd, variant=v)
            torch.cuda.synchronize()
            assert np.array_equal(_host(kd), ref), v
    # pass by pass: after p passes each run of 2^(10+p) keys is sorted
    kd = _to_dev(keys)
    meld.merge_sort(kd, max_passes=3, variant="melded")
    torch.cuda.synchronize()
    got, run = _host(kd), 1 << 13
    for s0 in range(0, n, run):
        assert np.array_equal(got[s0:s0 + run], oracle.sort_u32(keys[s0:s0 + run])), s0


def test_merge_sort_timed_size_against_oracle():
    # The timed configuration: 2^24 keys of seed 1, both forms.
    n = 1 << 24
    keys = workloads.keys_u32(1, n)
    ref = oracle.sort_u32(keys)
    for v in ("divergent", "melded"):
        kd = _to_dev(keys)
        meld.merge_sort(kd, variant=v)
        torch.cuda.synchronize()
        assert np.array_equal(_host(kd), ref), v


def test_merge_sort_noop_and_errors():
    for n in (0, 1):
        kd = _to_dev(np.array([7] * n, np.uint32))
        meld.merge_sort(kd)
        assert _host(kd).tolist() == [7] * n
    import ctypes
    lib = meld.load_library()
    host = (ctypes.c_uint32 * 64)()
    st = lib.meld_merge_sort_u32(meld.context(0), ctypes.cast(host, ctypes.c_void_p), 64, -1, 1,
                                 None)
    assert st == meld.EINVAL
