"""GPU parity of the bitonic sort (both forms) against the CPU oracle.

Bar: bit-exact. Keys-only output is unique; with a payload the
lexicographic (key, payload) order makes it unique too. The stage tests pin
that the GPU runs the Figure 1 network itself: after every prefix of steps
the array equals the oracle's step-by-step emulation.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
meld = pytest.importorskip("paper_2107_05681_amd")

VARIANTS = ("divergent", "melded")  # for the sorts MELDED_INPLACE == MELDED
# Each form on both paths of the phases k <= 64: the LDS comparator network
# (0) and registers with DPP lane exchanges (1).
FORMS = [(v, x) for x in (0, 1) for v in VARIANTS]


def _path(x):
    meld.set_option(0, meld.OPT_LANE_EXCHANGE, x)


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


def _gpu_sort(keys, vals, variant):
    kd = _to_dev(keys)
    vd = None if vals is None else _to_dev(vals)
    meld.sort(kd, vd, variant=variant)
    torch.cuda.synchronize()
    return _to_host(kd), (None if vd is None else _to_host(vd))


SIZES = [2, 3, 63, 64, 65, 1000, 1025, 4096, 1 << 13, (1 << 13) + 1, 1 << 14, (1 << 14) + 1,
         1 << 16, (1 << 17) + 3, 1 << 20]


@pytest.mark.parametrize("n", SIZES)
def test_sort_keys(n):
    keys = workloads.keys_u32(n, n)
    ref = oracle.sort_u32(keys)
    for v, x in FORMS:
        _path(x)
        got, _ = _gpu_sort(keys, None, v)
        assert np.array_equal(got, ref), (n, v, x)


@pytest.mark.parametrize("n", SIZES)
def test_sort_pairs(n):
    keys = workloads.keys_u32(n + 1, n)
    vals = workloads.iota_u32(n)
    rk, rv = oracle.sort_pairs_u32(keys, vals)
    for v, x in FORMS:
        _path(x)
        gk, gv = _gpu_sort(keys, vals, v)
        assert np.array_equal(gk, rk) and np.array_equal(gv, rv), (n, v, x)


def test_sort_pairs_heavy_ties_and_extremes():
    n = (1 << 15) + 77
    keys = (workloads.keys_u32(8, n) % np.uint32(5)).astype(np.uint32)
    keys[::97] = 0xFFFFFFFF  # real elements equal to the padding sentinel
    vals = (workloads.keys_u32(9, n) % np.uint32(3)).astype(np.uint32)
    vals[::89] = 0xFFFFFFFF
    rk, rv = oracle.sort_pairs_u32(keys, vals)
    for v, x in FORMS:
        _path(x)
        gk, gv = _gpu_sort(keys, vals, v)
        assert np.array_equal(gk, rk) and np.array_equal(gv, rv), (v, x)


def test_sort_n_below_two_is_noop():
    for n in (0, 1):
        k = _to_dev(np.array([7] * n, np.uint32))
        meld.sort(k)
        assert _to_host(k).tolist() == [7] * n


@pytest.mark.parametrize("log_n,pairs", [(10, False), (10, True), (15, False), (14, True),
                                         (16, True)])
def test_stage_parity_with_figure1_emulator(log_n, pairs):
    n = 1 << log_n
    keys = workloads.keys_u32(log_n, n)
    vals = workloads.iota_u32(n) if pairs else None
    total = oracle.bitonic_num_steps(n)
    rng = np.random.default_rng(log_n)
    if log_n <= 10:
        checks = list(range(1, total + 1))
    else:
        checks = sorted(set([1, 2, 3, 21, 28, total - 1, total] +
                            rng.integers(1, total, 12).tolist()))
    for s in checks:
        ref = oracle.bitonic_emulate(keys, vals, max_steps=s)
        for v, x in FORMS:
            _path(x)
            kd = _to_dev(keys)
            vd = None if vals is None else _to_dev(vals)
            meld.sort_steps(kd, vd, max_steps=s, variant=v)
            torch.cuda.synchronize()
            if pairs:
                assert np.array_equal(_to_host(kd), ref[0]) and \
                    np.array_equal(_to_host(vd), ref[1]), (s, v, x)
            else:
                assert np.array_equal(_to_host(kd), ref), (s, v, x)


def test_sort_pairs_full_size_properties():
    # 2^28 (key, payload = index) pairs. A non-decreasing composite order plus
    # key[i] == in_key[payload[i]] plus payload being a permutation fixes the
    # output completely, so this is an exact check at full size.
    dev = _dev()
    n = 1 << 28
    keys = workloads.keys_u32(1, n)
    kin = torch.from_numpy(keys.view(np.int32)).to(dev)
    del keys
    for v, x in FORMS:
        _path(x)
        k = kin.clone()
        p = torch.arange(n, dtype=torch.int32, device=dev)
        meld.sort(k, p, variant=v)
        torch.cuda.synchronize()
        # (key - 2^31) * 2^32 + payload orders like the unsigned (key, payload)
        # pair and fits a signed 64-bit integer.
        k64 = (k.to(torch.int64) & 0xFFFFFFFF) - (1 << 31)
        comp = (k64 << 32) + (p.to(torch.int64) & 0xFFFFFFFF)
        del k64
        assert bool((comp[1:] > comp[:-1]).all()), (v, x)
        del comp
        seen = torch.zeros(n, dtype=torch.bool, device=dev)
        seen[p.long()] = True
        assert bool(seen.all()), (v, x)
        del seen
        assert torch.equal(kin[p.long()], k), (v, x)
        del k, p
        torch.cuda.empty_cache()


def test_sort_keys_full_size_exact():
    # 2^28 keys alone: their streaming passes differ from the pairs' (gathered
    # tiles of 2^14 keys, the two-pass phases' first passes at array bits 20
    # and 21, in XCD runs). The output must equal the input sorted, which a
    # library sort of the same keys as 64-bit values (unsigned order) gives.
    dev = _dev()
    n = 1 << 28
    keys = workloads.keys_u32(2, n)
    kin = torch.from_numpy(keys.view(np.int32)).to(dev)
    del keys
    ref = torch.sort(kin.to(torch.int64) & 0xFFFFFFFF).values
    for v, x in FORMS:
        _path(x)
        k = kin.clone()
        meld.sort(k, None, variant=v)
        torch.cuda.synchronize()
        assert torch.equal(k.to(torch.int64) & 0xFFFFFFFF, ref), (v, x)
        del k
        torch.cuda.empty_cache()


def test_sort_rejects_host_pointer():
    import ctypes
    lib = meld.load_library()
    _dev()
    host = (ctypes.c_uint32 * 64)()
    st = lib.meld_sort_u32(meld.context(0), ctypes.cast(host, ctypes.c_void_p), None, 64, 1, None)
    assert st == meld.EINVAL
    assert b"device pointer" in lib.meld_last_error()


@pytest.fixture
def tile_option():
    """Restores the automatic sort tile after a test that forces one."""
    yield lambda t: meld.set_option(0, meld.OPT_SORT_LOG_TILE, t)
    meld.set_option(0, meld.OPT_SORT_LOG_TILE, 0)


@pytest.mark.parametrize("log_t", [8, 9, 10, 11, 12, 13, 14])
def test_sort_every_tile_size(log_t, tile_option):
    _dev()
    tile_option(log_t)
    # several tiles with a ragged tail, and one padded tile
    for n in ((1 << (log_t + 3)) + 17, (1 << log_t) - 5):
        keys = workloads.keys_u32(100 + log_t, n)
        ref = oracle.sort_u32(keys)
        vals = workloads.iota_u32(n)
        rk, rv = oracle.sort_pairs_u32(keys, vals)
        for v, x in FORMS:
            _path(x)
            got, _ = _gpu_sort(keys, None, v)
            assert np.array_equal(got, ref), (log_t, n, v, x)
            gk, gv = _gpu_sort(keys, vals, v)
            assert np.array_equal(gk, rk) and np.array_equal(gv, rv), (log_t, n, v, x)


@pytest.mark.parametrize("log_t,log_n,pairs", [(8, 12, False), (8, 11, True), (11, 13, True)])
def test_stage_parity_small_tiles(log_t, log_n, pairs, tile_option):
    # Every step prefix, with tiles forced small so that the register-window
    # phases, the merges and the streaming passes all take part.
    _dev()
    tile_option(log_t)
    n = 1 << log_n
    keys = workloads.keys_u32(200 + log_n, n)
    vals = workloads.iota_u32(n) if pairs else None
    total = oracle.bitonic_num_steps(n)
    for s in range(1, total + 1):
        ref = oracle.bitonic_emulate(keys, vals, max_steps=s)
        for v, x in FORMS:
            _path(x)
            kd = _to_dev(keys)
            vd = None if vals is None else _to_dev(vals)
            meld.sort_steps(kd, vd, max_steps=s, variant=v)
            torch.cuda.synchronize()
            if pairs:
                assert np.array_equal(_to_host(kd), ref[0]) and \
                    np.array_equal(_to_host(vd), ref[1]), (s, v, x)
            else:
                assert np.array_equal(_to_host(kd), ref), (s, v, x)


@pytest.mark.parametrize("log_t", [9, 13])
@pytest.mark.parametrize("pairs", [False, True])
def test_merge_tail_stage_parity(log_t, pairs, tile_option):
    # The merge tails of 2^9 and 2^13 end in layout W0 with three lane steps
    # (element bits 6, 5 and 4; the one on bit 6 exchanges with lane t ^ 4):
    # every step prefix of the last phase of a 2^(log_t + 1) array, its
    # streaming step and the whole merge tail.
    _dev()
    tile_option(log_t)
    n = 1 << (log_t + 1)
    keys = workloads.keys_u32(600 + log_t, n)
    vals = workloads.iota_u32(n) if pairs else None
    total = oracle.bitonic_num_steps(n)
    for s in range(total - (log_t + 1), total + 1):
        ref = oracle.bitonic_emulate(keys, vals, max_steps=s)
        for v, x in FORMS:
            _path(x)
            kd = _to_dev(keys)
            vd = None if vals is None else _to_dev(vals)
            meld.sort_steps(kd, vd, max_steps=s, variant=v)
            torch.cuda.synchronize()
            if pairs:
                assert np.array_equal(_to_host(kd), ref[0]) and \
                    np.array_equal(_to_host(vd), ref[1]), (s, v, x)
            else:
                assert np.array_equal(_to_host(kd), ref), (s, v, x)


@pytest.mark.parametrize("n", [1 << 12, (1 << 15) + 9])
def test_sort_unaligned_arrays(n):
    # Views one element into their buffers: not 16-byte aligned, so the
    # per-element load and store paths run.
    keys = workloads.keys_u32(300, n)
    vals = workloads.iota_u32(n)
    rk, rv = oracle.sort_pairs_u32(keys, vals)
    for v, x in FORMS:
        _path(x)
        kb = _to_dev(np.concatenate([[0], keys]).astype(np.uint32))
        vb = _to_dev(np.concatenate([[0], vals]).astype(np.uint32))
        kd, vd = kb[1:], vb[1:]
        assert kd.data_ptr() % 16 != 0
        meld.sort(kd, vd, variant=v)
        torch.cuda.synchronize()
        assert np.array_equal(_to_host(kd), rk) and np.array_equal(_to_host(vd), rv), (n, v, x)
        assert _to_host(kb)[0] == 0 and _to_host(vb)[0] == 0


def test_sort_tile_option_rejects_out_of_range(tile_option):
    _dev()
    for bad in (1, 7, 15, -1):
        with pytest.raises(meld.MeldError):
            tile_option(bad)
    tile_option(0)


@pytest.mark.parametrize("pairs", [False, True])
def test_gathered_passes_stage_parity(pairs, tile_option):
    # Tiles of 2^8 in a 2^15 array: the last three phases (k = 2^13 .. 2^15)
    # have 5, 6 and 7 streaming steps; keys run 7 as one gathered LDS pass and
    # 5, 6 in registers, pairs all three as gathered passes. Every step prefix
    # of these three phases is checked.
    _dev()
    tile_option(8)
    log_n = 15
    n = 1 << log_n
    keys = workloads.keys_u32(400 + pairs, n)
    vals = workloads.iota_u32(n) if pairs else None
    plan = meld.sort_plan(n, pairs, variant="melded", device=0)
    gathered = sorted(p["steps"] for p in plan["passes"] if p["kind"] == "gather")
    assert gathered == ([5, 6, 7] if pairs else [7])
    total = oracle.bitonic_num_steps(n)
    for s in range(total - 15 - 14 - 13, total + 1):
        ref = oracle.bitonic_emulate(keys, vals, max_steps=s)
        for v, x in FORMS:
            _path(x)
            kd = _to_dev(keys)
            vd = None if vals is None else _to_dev(vals)
            meld.sort_steps(kd, vd, max_steps=s, variant=v)
            torch.cuda.synchronize()
            if pairs:
                assert np.array_equal(_to_host(kd), ref[0]) and \
                    np.array_equal(_to_host(vd), ref[1]), (s, v, x)
            else:
                assert np.array_equal(_to_host(kd), ref), (s, v, x)


@pytest.mark.parametrize("log_t", [8, 9])
@pytest.mark.parametrize("n", [1 << 17, (1 << 17) - 3, (1 << 18) + 5])
def test_gathered_passes_full_sort(log_t, n, tile_option):
    # Small tiles make phases with up to 10 streaming steps, so gathered passes
    # (pairs from 5 steps, keys from 7; with their per-element tail path for
    # ragged n) run.
    _dev()
    tile_option(log_t)
    keys = workloads.keys_u32(500 + log_t, n)
    vals = workloads.iota_u32(n)
    ref = oracle.sort_u32(keys)
    rk, rv = oracle.sort_pairs_u32(keys, vals)
    for v, x in FORMS:
        _path(x)
        got, _ = _gpu_sort(keys, None, v)
        assert np.array_equal(got, ref), (log_t, n, v, x)
        gk, gv = _gpu_sort(keys, vals, v)
        assert np.array_equal(gk, rk) and np.array_equal(gv, rv), (log_t, n, v, x)
