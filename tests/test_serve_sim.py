"""Host-only tests of the serving scheduler over the simulated executor."""
import os
import time

import pytest


def _serve():
    import paper_2107_05681_amd as meld
    if not os.path.exists(meld.LIB_PATH):
        from paper_2107_05681_amd import build
        build.build()
    from paper_2107_05681_amd import serve
    return meld, serve


def _sort(n, seed=1):
    return dict(kind=0, n=n, seed=seed)


def _region(n, seed=1):
    return dict(kind=1, n=n, seed=seed, thr=1 << 31,
                side_true=dict(a=0.5, off=0, step=3, trips=4),
                side_false=dict(a=0.75, off=64, step=5, trips=4))


def test_budget_is_never_exceeded_and_all_jobs_finish():
    meld, serve = _serve()
    trace = []
    t = 0.0
    for i in range(200):
        t += 0.0002
        n = [1000, 70000, 5000, 100000, 3000][i % 5]
        job = _region(n // 4, i) if i % 3 == 0 else _sort(n, i)
        job["arrival_s"] = t
        trace.append(job)
    budget = 1 << 20
    with serve.Server(budget_bytes=budget, slots=4, simulated_ns_per_item=20) as srv:
        done = serve.replay(srv, trace, timeout_s=60)
        st = srv.stats()
    assert len(done) == 200 and all(c["status"] == meld.OK for c in done)
    assert st["max_inflight_bytes"] <= budget
    assert st["completed"] == 200 and st["rejected"] == 0


def test_oversize_job_is_rejected():
    meld, serve = _serve()
    with serve.Server(budget_bytes=1024, slots=2, simulated_ns_per_item=1) as srv:
        with pytest.raises(meld.MeldError) as e:
            srv.submit(_sort(1000))
        assert e.value.status == meld.ENOMEM
        assert srv.stats()["rejected"] == 1


def test_non_finite_arrival_is_rejected():
    meld, serve = _serve()
    with serve.Server(budget_bytes=1 << 20, slots=1, simulated_ns_per_item=1) as srv:
        for bad in (float("inf"), float("nan")):
            with pytest.raises(meld.MeldError) as e:
                srv.submit(_sort(100), arrival_s=bad)
            assert e.value.status == meld.EINVAL
        assert srv.stats()["pending"] == 0


def test_fifo_admission_order():
    meld, serve = _serve()
    trace = [dict(_region(20000, i), arrival_s=0.0) for i in range(30)]
    with serve.Server(budget_bytes=1 << 30, slots=3, simulated_ns_per_item=50) as srv:
        done = serve.replay(srv, trace, timeout_s=60)
    by_id = sorted(done, key=lambda c: c["job_id"])
    starts = [c["start_s"] for c in by_id]
    assert starts == sorted(starts)


def test_small_sorts_arriving_together_are_batched():
    meld, serve = _serve()
    with serve.Server(budget_bytes=1 << 30, slots=1, simulated_ns_per_item=200) as srv:
        srv.submit(_region(100000))  # occupies the only slot for ~20 ms
        ids = [srv.submit(_sort(2000 + i, i)) for i in range(50)]
        srv.drain(30)
        comps = srv.poll()
        st = srv.stats()
    assert len(comps) == 51
    assert st["launches"] == 2 and st["batched_jobs"] == 50
    assert all(c["batched"] == 50 for c in comps if c["job_id"] in ids)


def test_memory_bound_admission_serialises():
    meld, serve = _serve()
    trace = [dict(_region(5000, i), arrival_s=0.0) for i in range(10)]  # 40 KB each
    with serve.Server(budget_bytes=64 << 10, slots=4, simulated_ns_per_item=100) as srv:
        done = serve.replay(srv, trace, timeout_s=60)
        st = srv.stats()
    assert len(done) == 10
    assert st["max_concurrent"] == 1 and st["max_inflight_bytes"] <= 64 << 10


def test_injected_failures_are_isolated():
    meld, serve = _serve()
    trace = [dict(_region(1000, i), arrival_s=0.0) for i in range(12)]
    with serve.Server(budget_bytes=1 << 24, slots=2, simulated_ns_per_item=10,
                      fail_ids=(3, 7)) as srv:
        done = serve.replay(srv, trace, timeout_s=60)
    status = {c["job_id"]: c["status"] for c in done}
    assert status[3] == meld.EHIP and status[7] == meld.EHIP
    assert all(s == meld.OK for j, s in status.items() if j not in (3, 7))


def test_release_of_unknown_job_fails():
    meld, serve = _serve()
    with serve.Server(budget_bytes=1 << 20, slots=1, simulated_ns_per_item=1) as srv:
        with pytest.raises(meld.MeldError):
            srv.release(12345)


def test_latency_summary_busy_fraction_and_waits():
    from paper_2107_05681_amd import serve

    def job(sub, start, done, kind=serve.JOB_SORT, n=10):
        return dict(submit_s=sub, start_s=start, done_s=done, kind=kind, n=n)
    # runs [1, 3) and [2, 4) overlap into [1, 4); [6, 7) alone; span [0, 10)
    done = [job(0.0, 1.0, 3.0), job(0.5, 2.0, 4.0), job(5.0, 6.0, 7.0), job(9.0, 9.5, 10.0)]
    s = serve.latency_summary(done)
    assert s["span_s"] == 10.0
    assert abs(s["busy_fraction"] - (3.0 + 1.0 + 0.5) / 10.0) < 1e-12
    assert abs(s["wait_p50_ms"] - 1000.0) < 1e-9  # waits 1.0, 1.5, 1.0, 0.5: median 1.0
    assert s["jobs"] == 4 and abs(s["keys_per_s"] - 4.0) < 1e-12


def test_jobs_scheduled_ahead_start_no_earlier_than_their_arrival():
    meld, serve = _serve()
    with serve.Server(budget_bytes=1 << 30, slots=4, simulated_ns_per_item=1) as srv:
        t0 = srv.now()
        arrivals = [t0 + 0.05 + 0.002 * i for i in range(20)]
        ids = [srv.submit(_sort(1000 + i, i), arrival_s=a) for i, a in enumerate(arrivals)]
        assert srv.stats()["pending"] == 20  # not yet arrived
        srv.drain(30)
        comps = {c["job_id"]: c for c in srv.poll()}
    for jid, a in zip(ids, arrivals):
        c = comps[jid]
        assert c["arrival_s"] == a and c["submit_s"] < a
        assert c["start_s"] >= a and c["done_s"] >= c["start_s"]


def test_latency_counts_from_the_arrival_not_the_submit():
    meld, serve = _serve()
    with serve.Server(budget_bytes=1 << 30, slots=1, simulated_ns_per_item=1) as srv:
        time.sleep(0.6)
        late = srv.now() - 0.5  # submitted half a second after its arrival
        jid = srv.submit(_sort(100), arrival_s=late)
        srv.drain(30)
        c = srv.poll()[0]
    assert c["job_id"] == jid and c["arrival_s"] == late
    s = serve.latency_summary([c])
    assert s["p50_ms"] >= 500.0 and s["submit_lead_min_ms"] <= -500.0


def test_replay_schedules_the_trace_on_the_server_clock():
    meld, serve = _serve()
    trace = [dict(_sort(500 + i, i), arrival_s=0.001 * i) for i in range(50)]
    with serve.Server(budget_bytes=1 << 30, slots=2, simulated_ns_per_item=1) as srv:
        done = serve.replay(srv, trace, timeout_s=60)
    done.sort(key=lambda c: c["job_id"])
    base = done[0]["arrival_s"]
    for job, c in zip(trace, done):
        assert abs(c["arrival_s"] - base - job["arrival_s"]) < 1e-9
        assert c["start_s"] >= c["arrival_s"] and c["submit_s"] <= c["arrival_s"]
