"""The single-array sorts at the largest n they accept, 2^31 - 1 keys (one short
of the 2^31-element network, so the last position is a virtual sentinel):
tiles, passes and merge cuts must not wrap at 32 bits.

Exact at full size: for (key, payload = index) pairs, a strictly increasing
composite order plus key[i] == in_key[payload[i]] plus payload being a
permutation fixes the output. The keys-only bitonic sort and the merge sort
must then equal its key column. The odd-even bucket sort is checked on every
bucket by properties and on sampled buckets against the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
meld = pytest.importorskip("paper_2107_05681_amd")

N = (1 << 31) - 1
VARIANTS = ("divergent", "melded")


@pytest.fixture(scope="module")
def data():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    if torch.cuda.get_device_properties(dev).total_memory < (96 << 30):
        pytest.skip("needs 96 GiB of device memory")
    print(f"\n[sort max] n = {N} keys", flush=True)
    keys = workloads.keys_u32(2, N)
    kin = torch.from_numpy(keys.view(np.int32)).to(dev)
    del keys
    out = dict(dev=dev, kin=kin, sorted=None)
    yield out
    out.clear()
    torch.cuda.empty_cache()


def _unsigned_order(k):
    # flipping the sign bit maps unsigned order onto int32 order
    return k ^ torch.iinfo(torch.int32).min


def test_sort_pairs_max(data):
    kin, dev = data["kin"], data["dev"]
    for v in VARIANTS:
        print(f"[sort max] pairs {v}", flush=True)
        k = kin.clone()
        p = torch.arange(N, dtype=torch.int32, device=dev)
        meld.sort(k, p, variant=v)
        torch.cuda.synchronize()
        comp = ((k.to(torch.int64) & 0xFFFFFFFF) - (1 << 31)) << 32
        comp += p.to(torch.int64)
        assert bool((comp[1:] > comp[:-1]).all()), v
        del comp
        pl = p.long()
        seen = torch.zeros(N, dtype=torch.bool, device=dev)
        seen[pl] = True
        assert bool(seen.all()), v
        del seen
        assert torch.equal(kin[pl], k), v
        del pl, p
        if data["sorted"] is None:
            data["sorted"] = k
        else:
            assert torch.equal(data["sorted"], k), v
            del k
        torch.cuda.empty_cache()


def test_sort_keys_max(data):
    if data["sorted"] is None:
        pytest.skip("needs the pairs result")
    for v in VARIANTS:
        print(f"[sort max] keys {v}", flush=True)
        k = data["kin"].clone()
        meld.sort(k, None, variant=v)
        torch.cuda.synchronize()
        assert torch.equal(k, data["sorted"]), v
        del k
        torch.cuda.empty_cache()


def test_merge_sort_max(data):
    if data["sorted"] is None:
        pytest.skip("needs the pairs result")
    for v in VARIANTS:
        print(f"[sort max] merge sort {v}", flush=True)
        k = data["kin"].clone()
        meld.merge_sort(k, variant=v)
        torch.cuda.synchronize()
        assert torch.equal(k, data["sorted"]), v
        del k
        torch.cuda.empty_cache()


def test_oddeven_buckets_max(data):
    log_b = 13
    b = 1 << log_b
    full = N // b
    kin = data["kin"]
    rng = np.random.default_rng(5)
    picks = sorted(set(rng.integers(0, full, 48).tolist()) | {0, full - 1})
    for v in VARIANTS:
        print(f"[sort max] odd-even buckets 2^{log_b} {v}", flush=True)
        k = kin.clone()
        meld.oddeven_sort_buckets(k, log_b, variant=v)
        torch.cuda.synchronize()
        rows = _unsigned_order(k[:full * b].view(full, b))
        assert bool((rows[:, 1:] >= rows[:, :-1]).all()), v
        del rows
        # per-bucket sums are kept (a permutation inside every bucket)
        s_in = (kin[:full * b].view(full, b).to(torch.int64) & 0xFFFFFFFF).sum(dim=1)
        s_out = (k[:full * b].view(full, b).to(torch.int64) & 0xFFFFFFFF).sum(dim=1)
        assert torch.equal(s_in, s_out), v
        del s_in, s_out
        host_in = kin.view(torch.int32)
        for r in picks:
            ref = oracle.sort_u32(host_in[r * b:(r + 1) * b].cpu().numpy().view(np.uint32))
            got = k[r * b:(r + 1) * b].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, ref), (v, r)
        # the ragged last bucket (2^13 - 1 keys)
        ref = oracle.sort_u32(host_in[full * b:].cpu().numpy().view(np.uint32))
        assert np.array_equal(k[full * b:].cpu().numpy().view(np.uint32), ref), v
        del k
        torch.cuda.empty_cache()
