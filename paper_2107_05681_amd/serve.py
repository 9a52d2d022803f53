"""Python driver of the serving loop (ctypes over meld_server_* in libmeld.so)."""
from __future__ import annotations

import ctypes
import time

from . import MeldError, OK, Side, _as_side, _variant, load_library

JOB_SORT, JOB_REGION = 0, 1


class Job(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("n", ctypes.c_size_t), ("seed", ctypes.c_uint64),
                ("thr", ctypes.c_uint64), ("side_true", Side), ("side_false", Side),
                ("arrival_s", ctypes.c_double)]


class Completion(ctypes.Structure):
    _fields_ = [("job_id", ctypes.c_uint64), ("status", ctypes.c_int), ("kind", ctypes.c_int),
                ("n", ctypes.c_size_t), ("arrival_s", ctypes.c_double),
                ("submit_s", ctypes.c_double),
                ("start_s", ctypes.c_double), ("done_s", ctypes.c_double),
                ("result_dev", ctypes.c_void_p), ("batched", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("batched_jobs", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_size_t), ("inflight_bytes", ctypes.c_size_t),
                ("max_inflight_bytes", ctypes.c_size_t), ("pending", ctypes.c_size_t),
                ("slots", ctypes.c_int), ("max_concurrent", ctypes.c_int)]


def _lib():
    lib = load_library()
    if not getattr(lib, "_serve_bound", False):
        vp, sz, u64, st = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int
        lib.meld_server_create.restype = st
        lib.meld_server_create.argtypes = [ctypes.c_int, sz, ctypes.c_int, st, u64,
                                           ctypes.c_uint32, ctypes.POINTER(vp)]
        lib.meld_server_create_simulated.restype = st
        lib.meld_server_create_simulated.argtypes = [sz, ctypes.c_int, ctypes.c_double,
                                                     ctypes.POINTER(u64), sz, ctypes.POINTER(vp)]
        lib.meld_server_submit.restype = st
        lib.meld_server_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.POINTER(u64)]
        lib.meld_server_poll.restype = st
        lib.meld_server_poll.argtypes = [vp, ctypes.POINTER(Completion), sz,
                                         ctypes.POINTER(sz)]
        lib.meld_server_release.restype = st
        lib.meld_server_release.argtypes = [vp, u64]
        lib.meld_server_read.restype = st
        lib.meld_server_read.argtypes = [vp, u64, vp, sz]
        lib.meld_server_drain.restype = st
        lib.meld_server_drain.argtypes = [vp, ctypes.c_double]
        lib.meld_server_stats_get.restype = st
        lib.meld_server_stats_get.argtypes = [vp, ctypes.POINTER(Stats)]
        lib.meld_server_last_error.restype = ctypes.c_char_p
        lib.meld_server_last_error.argtypes = []
        lib.meld_server_destroy.restype = None
        lib.meld_server_destroy.argtypes = [vp]
        lib.meld_server_now.restype = ctypes.c_double
        lib.meld_server_now.argtypes = [vp]
        lib._serve_bound = True
    return lib


def _check(status):
    if status != OK:
        raise MeldError(status, _lib().meld_server_last_error().decode(errors="replace"))


class Server:
    """A serving loop on one GPU (or simulated with ``simulated_ns_per_item``)."""

    def __init__(self, budget_bytes=8 << 30, slots=8, variant="melded", table_seed=1,
                 table_log2=24, device=0, simulated_ns_per_item=None, fail_ids=()):
        lib = _lib()
        self._h = ctypes.c_void_p()
        if simulated_ns_per_item is None:
            _check(lib.meld_server_create(device, budget_bytes, slots, _variant(variant),
                                          table_seed, table_log2, ctypes.byref(self._h)))
        else:
            arr = (ctypes.c_uint64 * max(len(fail_ids), 1))(*fail_ids)
            _check(lib.meld_server_create_simulated(budget_bytes, slots,
                                                    float(simulated_ns_per_item), arr,
                                                    len(fail_ids), ctypes.byref(self._h)))
        self._buf = (Completion * 4096)()

    def now(self) -> float:
        """Seconds on the server's clock (the clock of arrival_s and the completions)."""
        return float(_lib().meld_server_now(self._h))

    def submit(self, job: dict, arrival_s: float = 0.0) -> int:
        """Queues a job; with arrival_s (server clock) ahead of now it waits until then."""
        j = Job(int(job["kind"]), int(job["n"]), int(job["seed"]), int(job.get("thr", 0)),
                _as_side(job.get("side_true", dict(a=1, off=0, step=1, trips=0))),
                _as_side(job.get("side_false", dict(a=1, off=0, step=1, trips=0))),
                float(arrival_s))
        jid = ctypes.c_uint64()
        _check(_lib().meld_server_submit(self._h, ctypes.byref(j), ctypes.byref(jid)))
        return int(jid.value)

    def poll(self) -> list[dict]:
        n = ctypes.c_size_t()
        out = []
        while True:
            _check(_lib().meld_server_poll(self._h, self._buf, len(self._buf), ctypes.byref(n)))
            for i in range(n.value):
                c = self._buf[i]
                out.append(dict(job_id=int(c.job_id), status=int(c.status), kind=int(c.kind),
                                n=int(c.n), arrival_s=c.arrival_s, submit_s=c.submit_s,
                                start_s=c.start_s,
                                done_s=c.done_s, result_dev=c.result_dev, batched=c.batched))
            if n.value < len(self._buf):
                return out

    def read(self, job_id: int, n: int, dtype="uint32"):
        import numpy as np
        arr = np.empty(n, dtype=dtype)
        _check(_lib().meld_server_read(self._h, job_id, arr.ctypes.data, arr.nbytes))
        return arr

    def release(self, job_id: int) -> None:
        _check(_lib().meld_server_release(self._h, job_id))

    def drain(self, timeout_s=60.0) -> None:
        _check(_lib().meld_server_drain(self._h, timeout_s))

    def stats(self) -> dict:
        s = Stats()
        _check(_lib().meld_server_stats_get(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def close(self) -> None:
        if self._h:
            _lib().meld_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def replay(server: Server, trace: list[dict], on_complete=None, release=True,
           timeout_s=120.0, lead_s=None) -> list[dict]:
    """Runs a trace: every job is submitted ahead with its scheduled arrival on the
    server's clock (start + the trace's arrival_s, start = now + lead_s), so the
    server admits it at its arrival however late the host loop runs; then collects
    every completion. ``on_complete(completion, job)`` runs before the result is
    released."""
    if lead_s is None:
        lead_s = 0.05 + 2e-5 * len(trace)  # time to submit the whole trace
    start = server.now() + lead_s
    by_id = {}
    for job in trace:
        by_id[server.submit(job, arrival_s=start + job["arrival_s"])] = job
    done = []
    deadline = time.perf_counter() + lead_s + (trace[-1]["arrival_s"] if trace else 0) + timeout_s
    while len(done) < len(trace):
        comps = server.poll()
        for c in comps:
            job = by_id[c["job_id"]]
            if on_complete is not None:
                on_complete(c, job)
            if release and c["status"] == OK:
                server.release(c["job_id"])
            done.append(c)
        if not comps:
            if time.perf_counter() > deadline:
                raise TimeoutError(f"{len(done)} of {len(trace)} jobs completed")
            time.sleep(1e-4)
    return done


def latency_summary(done: list[dict]) -> dict:
    """Latency from each job's arrival (its submit time where it has none) to its
    completion, the queue wait (arrival to start), the submit lead (arrival minus
    submit: how far ahead of its arrival the job was handed over), throughput over
    the span from the first arrival to the last completion, and the share of that
    span during which at least one job ran."""
    import numpy as np
    arr = np.array([c.get("arrival_s", c["submit_s"]) for c in done])
    sub = np.array([c["submit_s"] for c in done])
    lat = np.array([c["done_s"] for c in done]) - arr
    wait = np.array([c["start_s"] for c in done]) - arr
    lead = arr - sub
    span = max(c["done_s"] for c in done) - float(arr.min())
    keys = sum(c["n"] for c in done if c["kind"] == JOB_SORT)
    lanes = sum(c["n"] for c in done if c["kind"] == JOB_REGION)
    busy, end = 0.0, -np.inf
    for a, b in sorted((c["start_s"], c["done_s"]) for c in done):
        if a > end:
            busy += b - a
            end = b
        elif b > end:
            busy += b - end
            end = b
    return dict(jobs=len(done), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
                wait_p50_ms=float(np.percentile(wait, 50) * 1e3),
                wait_p99_ms=float(np.percentile(wait, 99) * 1e3),
                submit_lead_p50_ms=float(np.percentile(lead, 50) * 1e3),
                submit_lead_min_ms=float(lead.min() * 1e3),
                jobs_per_s=len(done) / span, keys_per_s=keys / span, lanes_per_s=lanes / span,
                span_s=span, busy_fraction=busy / span if span > 0 else 0.0)
