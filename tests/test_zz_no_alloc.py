"""meld_sort_u32_noalloc, the entry point that allocates nothing, against
meld_sort_u32 through the C ABI.

Bar: bit-exact (the sorted output, and the (key, payload) order, are unique).
Two calls in a row on the shared device scratch, the second with a smaller
input, so that a stale tail from the first call would show; then the
rejection of a padding larger than the scratch.
"""
import ctypes

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


def _to_host(t):
    return t.cpu().numpy().view(np.uint32)


def _call(fn, keys, vals, variant):
    """One C-ABI call on the current stream; returns the status."""
    lib = meld.load_library()
    ctx = meld.context(0)
    stream = torch.cuda.current_stream().cuda_stream
    st = fn(ctx, ctypes.c_void_p(keys.data_ptr()),
            None if vals is None else ctypes.c_void_p(vals.data_ptr()), keys.numel(),
            meld._variant(variant), ctypes.c_void_p(stream))
    if st != meld.OK:
        raise meld.MeldError(st, lib.meld_last_error().decode())
    return st


# (n, pairs, seed): padding of 2 (2^21 - n) = 2 072 462 words, then a smaller
# keys-only sort with 61 071 words of padding, then pairs again below the
# first size.
CALLS = [((1 << 20) + 12345, True, 1), (70001, False, 2), ((1 << 18) + 3, True, 3)]


@pytest.mark.parametrize("variant", ["divergent", "melded", "auto"])
def test_noalloc_matches_sort_on_calls_in_a_row(variant):
    _dev()
    lib = meld.load_library()
    for n, pairs, seed in CALLS:
        keys = workloads.keys_u32(seed, n)
        vals = workloads.iota_u32(n) if pairs else None
        # the existing entry point
        ka, va = _to_dev(keys), (None if vals is None else _to_dev(vals))
        _call(lib.meld_sort_u32, ka, va, variant)
        # the no-allocation one
        kb, vb = _to_dev(keys), (None if vals is None else _to_dev(vals))
        _call(lib.meld_sort_u32_noalloc, kb, vb, variant)
        torch.cuda.synchronize()
        assert np.array_equal(_to_host(kb), _to_host(ka)), (n, variant)
        if pairs:
            assert np.array_equal(_to_host(vb), _to_host(va)), (n, variant)
        # and both are the oracle's order
        if pairs:
            rk, rv = oracle.sort_pairs_u32(keys, vals)
            assert np.array_equal(_to_host(kb), rk) and np.array_equal(_to_host(vb), rv)
        else:
            assert np.array_equal(_to_host(kb), oracle.sort_u32(keys))


def test_noalloc_rejects_padding_beyond_scratch():
    _dev()
    lib = meld.load_library()
    n = (1 << 23) + 1  # pairs: 2 (2^24 - n) words of padding > 2^22
    keys = workloads.keys_u32(4, n)
    kd, vd = _to_dev(keys), torch.arange(n, dtype=torch.int32, device=_dev())
    with pytest.raises(meld.MeldError) as err:
        _call(lib.meld_sort_u32_noalloc, kd, vd, "melded")
    assert err.value.status == meld.EINVAL and "scratch" in str(err.value)
    torch.cuda.synchronize()
    assert np.array_equal(_to_host(kd), keys)  # untouched


def test_noalloc_power_of_two_and_one_tile_need_no_scratch():
    # A power of two above the scratch size (no padding at all) and a padded
    # single tile (padding in LDS) are accepted.
    _dev()
    lib = meld.load_library()
    for n, seed in (((1 << 23), 5), (3000, 6)):
        keys = workloads.keys_u32(seed, n)
        kd = _to_dev(keys)
        _call(lib.meld_sort_u32_noalloc, kd, None, "melded")
        torch.cuda.synchronize()
        assert np.array_equal(_to_host(kd), oracle.sort_u32(keys)), n
