"""The segmented sort near the largest total it accepts (u32 offsets, so fewer
than 2^32 keys): 65536 segments holding 4294836226 keys (16 GiB). The first
segment has the maximum length 2^16, the second is empty, the rest have
2^16 - 1 keys (padded to 2^16 inside the network).

Every segment is checked for order and for its key sum (a permutation inside
each segment); sampled segments, the first, second and last among them, are
checked against the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
meld = pytest.importorskip("paper_2107_05681_amd")

NSEG = 1 << 16
LONG = 1 << 16
REST = LONG - 1
TOTAL = LONG + 0 + (NSEG - 2) * REST
VARIANTS = ("divergent", "melded", "auto")
ROWS = 4096  # segments per check chunk


def _offsets():
    lens = np.full(NSEG, REST, np.int64)
    lens[0], lens[1] = LONG, 0
    off = np.zeros(NSEG + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    assert off[-1] == TOTAL < (1 << 32)
    return off


def _flip(k):
    return k ^ torch.iinfo(torch.int32).min  # unsigned order as int32 order


def test_segmented_sort_max_total():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    if torch.cuda.get_device_properties(dev).total_memory < (64 << 30):
        pytest.skip("needs 64 GiB of device memory")
    print(f"\n[segsort max] {NSEG} segments, {TOTAL} keys", flush=True)
    off = _offsets()
    offd = torch.from_numpy(off.astype(np.uint32).view(np.int32)).to(dev)
    kin = torch.from_numpy(workloads.keys_u32(4, TOTAL).view(np.int32)).to(dev)
    rng = np.random.default_rng(8)
    picks = sorted(set(rng.integers(2, NSEG, 24).tolist()) | {0, 1, 2, NSEG - 1})
    refs = {}
    for s in picks:
        seg = kin[int(off[s]):int(off[s + 1])].cpu().numpy().view(np.uint32)
        refs[s] = oracle.sort_u32(seg)
    for v in VARIANTS:
        print(f"[segsort max] {v}", flush=True)
        k = kin.clone()
        meld.segmented_sort(k, offd, variant=v)
        torch.cuda.synchronize()
        # the maximum-length segment
        first = _flip(k[:LONG])
        assert bool((first[1:] >= first[:-1]).all()), v
        # the 2^16 - 1 key segments, in chunks of rows
        body_in = kin[LONG:].view(NSEG - 2, REST)
        body = k[LONG:].view(NSEG - 2, REST)
        for r0 in range(0, NSEG - 2, ROWS):
            rows = _flip(body[r0:r0 + ROWS])
            assert bool((rows[:, 1:] >= rows[:, :-1]).all()), (v, r0)
            s_in = (body_in[r0:r0 + ROWS].to(torch.int64) & 0xFFFFFFFF).sum(dim=1)
            s_out = (body[r0:r0 + ROWS].to(torch.int64) & 0xFFFFFFFF).sum(dim=1)
            assert torch.equal(s_in, s_out), (v, r0)
        for s in picks:
            got = k[int(off[s]):int(off[s + 1])].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, refs[s]), (v, s)
        del k
        torch.cuda.empty_cache()
