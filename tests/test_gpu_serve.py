"""GPU serving: every job's result in the mix equals the job run alone (bit for bit)."""
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


TAB_SEED, TAB_LOG2 = 9, 18


def test_results_in_the_mix_equal_results_alone():
    dev = _dev()
    from paper_2107_05681_amd import serve
    trace = workloads.serving_trace(3, rate=3000.0, duration_s=0.15, sort_log2=(10, 17),
                                    region_log2=(12, 15), tab_log2=TAB_LOG2)
    assert len(trace) > 200
    results = {}

    def keep(c, job):
        assert c["status"] == meld.OK, c
        results[c["job_id"]] = (job, c, serve_read(srv, c, job))

    def serve_read(s, c, job):
        return s.read(c["job_id"], job["n"], "uint32" if job["kind"] == 0 else "float32")

    with serve.Server(budget_bytes=16 << 20, slots=4, variant="melded", table_seed=TAB_SEED,
                      table_log2=TAB_LOG2) as srv:
        done = serve.replay(srv, trace, on_complete=keep, timeout_s=120)
        st = srv.stats()
    assert len(done) == len(trace) and st["failed"] == 0
    assert st["max_inflight_bytes"] <= 16 << 20
    assert st["batched_jobs"] > 0            # continuous batching happened
    assert st["max_concurrent"] >= 2         # slots overlapped
    spans = sorted((c["start_s"], c["done_s"]) for _, c, _ in results.values())
    assert any(b[0] < a[1] for a, b in zip(spans, spans[1:]))  # some jobs overlapped in time

    tab_h = workloads.tab_f32(TAB_SEED, 1 << TAB_LOG2)
    tab_d = torch.from_numpy(tab_h).to(dev)
    for jid, (job, c, got) in results.items():
        if job["kind"] == 0:
            keys = workloads.keys_u32(job["seed"], job["n"])
            alone = torch.from_numpy(keys.view(np.int32)).to(dev)
            meld.sort(alone, variant="melded")
            alone_h = alone.cpu().numpy().view(np.uint32)
            assert np.array_equal(got, alone_h), jid
            assert np.array_equal(got, np.sort(keys)), jid
        else:
            x = workloads.x_f32(job["seed"], job["n"])
            y = meld.divergent_region(torch.from_numpy(x).to(dev), tab_d, job["seed"],
                                      job["thr"], job["side_true"], job["side_false"],
                                      variant="melded")
            alone_h = y.cpu().numpy()
            assert np.array_equal(got.view(np.uint32), alone_h.view(np.uint32)), jid
            ref = oracle.region_f32(x, tab_h, job["seed"], job["thr"], job["side_true"],
                                    job["side_false"])
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), jid


def test_oversize_job_rejected_on_gpu():
    _dev()
    from paper_2107_05681_amd import serve
    with serve.Server(budget_bytes=1 << 16, slots=2, table_log2=10) as srv:
        with pytest.raises(meld.MeldError) as e:
            srv.submit(dict(kind=0, n=1 << 20, seed=1))
        assert e.value.status == meld.ENOMEM


def test_full_size_slice_alone_in_the_mix_and_oracle():
    # A slice of the serving workload at its full sizes: Poisson 2000 jobs/s,
    # sorts log-uniform in [2^10, 2^22] keys, regions in [2^16, 2^20] lanes at
    # p = 0.5 over the 2^24-entry table. Every result equals the job run alone
    # and the oracle.
    dev = _dev()
    from paper_2107_05681_amd import serve
    tab_log2, tab_seed = 24, 1
    trace = workloads.serving_trace(11, rate=2000.0, duration_s=0.04, tab_log2=tab_log2)
    assert len(trace) >= 40
    assert max(j["n"] for j in trace if j["kind"] == 0) > 1 << 20
    results = {}

    with serve.Server(budget_bytes=2 << 30, slots=8, variant="melded", table_seed=tab_seed,
                      table_log2=tab_log2) as srv:
        def keep(c, job):
            assert c["status"] == meld.OK, c
            results[c["job_id"]] = (job, srv.read(c["job_id"], job["n"],
                                                  "uint32" if job["kind"] == 0 else "float32"))
        done = serve.replay(srv, trace, on_complete=keep, timeout_s=120)
        st = srv.stats()
    assert len(done) == len(trace) and st["failed"] == 0
    assert st["max_concurrent"] >= 2
    tab_h = workloads.tab_f32(tab_seed, 1 << tab_log2)
    tab_d = torch.from_numpy(tab_h).to(dev)
    for jid, (job, got) in results.items():
        if job["kind"] == 0:
            keys = workloads.keys_u32(job["seed"], job["n"])
            alone = torch.from_numpy(keys.view(np.int32)).to(dev)
            meld.sort(alone, variant="melded")
            assert np.array_equal(got, alone.cpu().numpy().view(np.uint32)), jid
            assert np.array_equal(got, oracle.sort_u32(keys)), jid
        else:
            x = workloads.x_f32(job["seed"], job["n"])
            y = meld.divergent_region(torch.from_numpy(x).to(dev), tab_d, job["seed"],
                                      job["thr"], job["side_true"], job["side_false"],
                                      variant="melded")
            assert np.array_equal(got.view(np.uint32), y.cpu().numpy().view(np.uint32)), jid
            ref = oracle.region_f32(x, tab_h, job["seed"], job["thr"], job["side_true"],
                                    job["side_false"])
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), jid
