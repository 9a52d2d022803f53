"""GPU parity of the segmented sort (every per-stage form) against the CPU oracle.

Bar: bit-exact. Each segment's sorted keys are unique, so the whole output
is unique.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
meld = pytest.importorskip("paper_2107_05681_amd")

STAGE_FORMS = [("divergent", "divergent"), ("melded", "melded"), ("melded", "divergent"),
               ("divergent", "melded")]
# Each per-stage form on both paths of the phases k <= 64 of segments above
# 128 keys: the LDS comparator network (0) and registers with DPP lane
# exchanges (1).
FORMS = [(lo, hi, x) for x in (0, 1) for lo, hi in STAGE_FORMS]


@pytest.fixture(autouse=True)
def _default_path():
    yield
    if torch.cuda.is_available():
        meld.set_option(0, meld.OPT_LANE_EXCHANGE, -1)


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(_dev())


def _to_host(t):
    return t.cpu().numpy().view(np.uint32)


def _offsets(lengths):
    return np.concatenate([[0], np.cumsum(lengths)]).astype(np.uint32)


def _run(keys, off, low, high, x=-1):
    kd = _to_dev(keys)
    od = _to_dev(off)
    meld.set_option(0, meld.OPT_LANE_EXCHANGE, x)
    meld.segmented_sort(kd, od, low=low, high=high)
    torch.cuda.synchronize()
    meld.segmented_sort_check(0)
    return _to_host(kd)


def test_segmented_full_size_log_uniform():
    # 4096 segments, lengths log-uniform in [2^6, 2^16] (about 3.9e7 keys).
    off = workloads.segment_offsets(1, 4096)
    n = int(off[-1])
    keys = workloads.keys_u32(1, n)
    ref = oracle.segmented_sort_u32(keys, off)
    for low, high, x in FORMS:
        got = _run(keys, off, low, high, x)
        assert np.array_equal(got, ref), (low, high, x)


def test_segmented_edge_lengths():
    lengths = [0, 1, 2, 3, 5, 63, 64, 65, 127, 128, 129, 255, 256, 257, 4095, 32767, 32768,
               32769, 40000, 65535, 65536, 0, 1, 2]
    off = _offsets(lengths)
    n = int(off[-1])
    keys = workloads.keys_u32(7, n)
    keys[::13] = 0xFFFFFFFF  # equal to the padding value
    keys[5::17] = 0
    keys[::29] = keys[1::29][: keys[::29].size] if n > 29 else keys[::29]
    ref = oracle.segmented_sort_u32(keys, off)
    for low, high, x in FORMS:
        got = _run(keys, off, low, high, x)
        assert np.array_equal(got, ref), (low, high, x)


def test_segmented_zero_one_principle():
    # Every 0/1 vector of length 16 as its own segment: 2^16 segments.
    bits = np.arange(1 << 16, dtype=np.uint32)
    keys = ((bits[:, None] >> np.arange(16, dtype=np.uint32)) & 1).astype(np.uint32).ravel()
    off = (np.arange((1 << 16) + 1, dtype=np.uint64) * 16).astype(np.uint32)
    ones = np.array([bin(b).count("1") for b in range(1 << 16)])
    expect = (np.arange(16)[None, :] >= (16 - ones)[:, None]).astype(np.uint32).ravel()
    for low, high in STAGE_FORMS[:2]:
        got = _run(keys, off, low, high)
        assert np.array_equal(got, expect), (low, high)


def test_segmented_many_tiny_segments():
    rng = np.random.default_rng(3)
    lengths = rng.integers(0, 9, 200_001)
    off = _offsets(lengths)
    keys = workloads.keys_u32(3, int(off[-1])) % np.uint32(7)
    ref = oracle.segmented_sort_u32(keys, off)
    for low, high in STAGE_FORMS[:2]:
        assert np.array_equal(_run(keys, off, low, high), ref)


def test_segmented_one_class_each_size():
    # One segment per size class 2..2^16 plus a ragged length in each class.
    lengths = []
    for c in range(1, 17):
        lengths += [1 << c, (1 << (c - 1)) + 1]
    off = _offsets(lengths)
    keys = workloads.keys_u32(11, int(off[-1]))
    ref = oracle.segmented_sort_u32(keys, off)
    for low, high, x in FORMS:
        assert np.array_equal(_run(keys, off, low, high, x), ref), (low, high, x)


@pytest.mark.parametrize("bad", ["decreasing", "too_long", "first_nonzero"])
def test_segmented_invalid_offsets_leave_keys_untouched(bad):
    if bad == "decreasing":
        off = np.array([0, 100, 50, 300], np.uint32)
        n = 300
    elif bad == "too_long":
        off = np.array([0, 10, 10 + 65537], np.uint32)
        n = 10 + 65537
    else:
        off = np.array([5, 100, 200], np.uint32)
        n = 200
    keys = workloads.keys_u32(2, n)
    kd = _to_dev(keys)
    meld.segmented_sort(kd, _to_dev(off))
    with pytest.raises(meld.MeldError) as e:
        meld.segmented_sort_check(0)
    assert e.value.status == meld.EINVAL
    assert np.array_equal(_to_host(kd), keys)
    meld.segmented_sort_check(0)  # the flag was cleared
    # a valid call afterwards works
    good = np.array([0, 50, 120], np.uint32)
    k2 = workloads.keys_u32(4, 120)
    assert np.array_equal(_run(k2, good, "melded", "melded"), oracle.segmented_sort_u32(k2, good))


def test_segmented_offsets_beyond_keys_rejected():
    # offsets[nseg] = 300 for a keys array of 200: the explicit forms flag it on
    # the device and touch no key; MELD_AUTO, which reads offsets[nseg] to size
    # its trials, rejects the call at once.
    keys = workloads.keys_u32(2, 200)
    off = _to_dev(np.array([0, 100, 300], np.uint32))
    for v in ("divergent", "melded", "staged"):
        kd = _to_dev(keys)
        if v == "staged":  # per-stage forms: meld_segmented_sort_u32_staged
            meld.segmented_sort(kd, off, low="melded", high="divergent")
        else:
            meld.segmented_sort(kd, off, variant=v)
        with pytest.raises(meld.MeldError) as e:
            meld.segmented_sort_check(0)
        assert e.value.status == meld.EINVAL and "beyond n_keys" in str(e.value), v
        assert np.array_equal(_to_host(kd), keys), v
    kd = _to_dev(keys)
    with pytest.raises(meld.MeldError) as e:
        meld.segmented_sort(kd, off, variant="auto")
    assert e.value.status == meld.EINVAL
    torch.cuda.synchronize()
    assert np.array_equal(_to_host(kd), keys)
    meld.segmented_sort_check(0)  # nothing flagged by the rejected call


def test_segmented_no_segments_is_noop():
    kd = _to_dev(np.array([3, 2, 1], np.uint32))
    meld.segmented_sort(kd, _to_dev(np.array([0], np.uint32)))
    assert _to_host(kd).tolist() == [3, 2, 1]


def test_segmented_graph_replays_match_eager():
    # The default path replays a captured hipGraph; compare several replays,
    # separated by unrelated eager work and synchronisations, with the eager
    # (one launch at a time) result.
    off = workloads.segment_offsets(5, 1024)
    n = int(off[-1])
    keys = workloads.keys_u32(5, n)
    dev = _dev()
    od = _to_dev(off)
    pristine = _to_dev(keys)
    meld.set_option(0, meld.OPT_USE_GRAPHS, 0)
    try:
        eager = pristine.clone()
        meld.segmented_sort(eager, od)
        torch.cuda.synchronize()
    finally:
        meld.set_option(0, meld.OPT_USE_GRAPHS, 1)
    work = torch.empty_like(pristine)
    junk = torch.randn(1 << 20, device=dev)
    for rep in range(5):
        work.copy_(pristine)
        junk = junk * 1.0001 + 1.0  # eager work between replays
        meld.segmented_sort(work, od)
        if rep % 2:
            torch.cuda.synchronize()
        assert torch.equal(work, eager), rep
    meld.segmented_sort_check(0)
    assert np.array_equal(_to_host(eager), oracle.segmented_sort_u32(keys, off))


def test_segmented_graph_not_replayed_after_scratch_growth():
    # A fresh context: MELD_AUTO at 100 segments captures a graph over the
    # context's queue arrays; a call at 200 segments (another shape class)
    # grows and reallocates them; the first call again must not replay a graph
    # that points at the freed arrays.
    dev = _dev()
    ctx = meld.new_context(0)
    try:
        runs = []
        for nseg, seed in ((100, 21), (200, 22)):
            off = workloads.segment_offsets(seed, nseg)
            keys = workloads.keys_u32(seed, int(off[-1]))
            runs.append((keys, off, _to_dev(off), _to_dev(keys)))
        k1, off1, od1, kd1 = runs[0]
        k2, off2, od2, kd2 = runs[1]
        meld.segmented_sort(kd1, od1, variant="auto", ctx=ctx)
        meld.segmented_sort(kd2, od2, variant="auto", ctx=ctx)
        torch.cuda.synchronize()
        assert np.array_equal(_to_host(kd2), oracle.segmented_sort_u32(k2, off2))
        kd1.copy_(_to_dev(k1))  # same pointers as the first call
        meld.segmented_sort(kd1, od1, variant="auto", ctx=ctx)
        torch.cuda.synchronize()
        meld.segmented_sort_check(0, ctx=ctx)
        assert np.array_equal(_to_host(kd1), oracle.segmented_sort_u32(k1, off1))
        # and the graph of the grown size still replays correctly
        kd2.copy_(_to_dev(k2))
        meld.segmented_sort(kd2, od2, variant="auto", ctx=ctx)
        torch.cuda.synchronize()
        assert np.array_equal(_to_host(kd2), oracle.segmented_sort_u32(k2, off2))
        assert dev is not None
    finally:
        meld.destroy_context(ctx)
