"""GPU parity of Batcher's odd-even merge network on buckets (the PCM network),
divergent and melded forms, against the CPU oracle. Bar: bit-exact (keys are
u32; a sorted bucket is unique) and, for every step prefix, equal to the
oracle's emulation of the network itself."""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
meld = pytest.importorskip("paper_2107_05681_amd")

VARIANTS = ("divergent", "melded", "auto")
PAD = np.uint32(0xFFFFFFFF)


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.uint32).view(np.int32)).to(_dev())


def _host(t):
    return t.cpu().numpy().view(np.uint32)


def _ref_buckets(keys, log_b, max_steps=-1):
    """Each bucket through the oracle network; a ragged last bucket is padded
    with the sentinel and cut back."""
    T = 1 << log_b
    out = keys.copy()
    for b0 in range(0, len(keys), T):
        chunk = keys[b0:b0 + T]
        full = np.concatenate([chunk, np.full(T - len(chunk), PAD, np.uint32)])
        out[b0:b0 + len(chunk)] = oracle.oddeven_emulate(full, max_steps)[:len(chunk)]
    return out


@pytest.mark.parametrize("log_b", list(range(6, 15)))
def test_oddeven_every_bucket_size(log_b):
    T = 1 << log_b
    for n in (3 * T + 17, T, T - 3):
        keys = workloads.keys_u32(60 + log_b, n)
        ref = _ref_buckets(keys, log_b)
        for b0 in range(0, n, T):
            assert np.array_equal(ref[b0:b0 + T], np.sort(keys[b0:b0 + T]))
        for v in VARIANTS:
            kd = _to_dev(keys)
            meld.oddeven_sort_buckets(kd, log_b, variant=v)
            torch.cuda.synchronize()
            assert np.array_equal(_host(kd), ref), (log_b, n, v)


@pytest.mark.parametrize("log_b", [6, 8, 11, 13, 14])
def test_oddeven_stage_parity(log_b):
    # every step prefix of the network, three buckets plus a ragged one
    T = 1 << log_b
    keys = workloads.keys_u32(70 + log_b, 3 * T + 5)
    total = log_b * (log_b + 1) // 2
    for s in range(1, total + 1):
        ref = _ref_buckets(keys, log_b, s)
        for v in ("divergent", "melded"):
            kd = _to_dev(keys)
            meld.oddeven_sort_buckets(kd, log_b, max_steps=s, variant=v)
            torch.cuda.synchronize()
            assert np.array_equal(_host(kd), ref), (log_b, s, v)


def test_oddeven_ties_and_sentinel_keys():
    log_b, n = 10, (1 << 13) + 100
    keys = (workloads.keys_u32(80, n) % np.uint32(3)).astype(np.uint32)
    keys[::37] = PAD
    ref = _ref_buckets(keys, log_b)
    for v in VARIANTS:
        kd = _to_dev(keys)
        meld.oddeven_sort_buckets(kd, log_b, variant=v)
        torch.cuda.synchronize()
        assert np.array_equal(_host(kd), ref), v


def test_oddeven_full_size_properties():
    # 2^26 keys in 2^13-key buckets: each bucket sorted and a permutation of
    # its input (checked against the input's own bucket-wise sort).
    dev = _dev()
    n, log_b = 1 << 26, 13
    kin = torch.from_numpy(workloads.keys_u32(2, n).view(np.int32)).to(dev)
    expect = (kin.to(torch.int64) & 0xFFFFFFFF).view(-1, 1 << log_b).sort(dim=1).values
    for v in ("divergent", "melded"):
        k = kin.clone()
        meld.oddeven_sort_buckets(k, log_b, variant=v)
        got = (k.to(torch.int64) & 0xFFFFFFFF).view(-1, 1 << log_b)
        assert torch.equal(got, expect), v
        del k, got
    torch.cuda.empty_cache()


def test_oddeven_rejects_bad_arguments():
    kd = _to_dev(np.zeros(256, np.uint32))
    for bad in (5, 15):
        with pytest.raises(meld.MeldError) as e:
            meld.oddeven_sort_buckets(kd, bad)
        assert e.value.status == meld.EINVAL
    meld.oddeven_sort_buckets(kd, 8, max_steps=0)  # no steps: a no-op
    assert np.all(_host(kd) == 0)
