"""Host logic of the request loop: footprint-based admission, bounded
concurrency, completion and rejection, with the device step replaced by a
timed stand-in (no GPU needed)."""
import threading
import time

import numpy as np
import pytest

from paper_2511_09546_amd import binding, inputs, serve


def _req(D, chi, key=None):
    A = inputs.random_state(D * 100 + chi, 1, 1, 2, D)
    return serve.Request(A=A, chi=chi, terms=inputs.terms_j1j2(1, 1, 1.0, 0.2),
                         state_key=key)


def test_footprint_formula():
    o = binding.default_opts()
    f = binding.footprint_bytes(1, 1, 2, 6, 72, o)
    q = 72 * 72 * 6 ** 4
    dbl = 4 * (4 + 1) * 6 ** 8
    env = 4 * 72 * 72 + 4 * 72 * 36 * 72
    assert f == int(8.0 * (q * (46 * 20 + 220) + dbl + env))
    # grows with every size and with K; zero for invalid sizes
    assert binding.footprint_bytes(1, 1, 2, 6, 108, o) > f
    assert binding.footprint_bytes(2, 2, 2, 6, 72, o) > 3.9 * f
    o.grad_K = 40
    assert binding.footprint_bytes(1, 1, 2, 6, 72, o) > 1.6 * f
    assert binding.footprint_bytes(0, 1, 2, 6, 72, o) == 0
    # checkpointed gradient: one iteration's intermediates instead of K
    o.grad_K = 20
    o.grad_checkpoint = 1
    assert binding.footprint_bytes(1, 1, 2, 6, 72, o) == int(
        8.0 * (q * (46 * 1 + 220) + dbl + env))


def test_admission_respects_budget_and_workers(monkeypatch):
    live = {"used": 0.0, "peak": 0.0, "n": 0, "nmax": 0}
    lock = threading.Lock()

    def fake_step(self, req, start, sidx=0):
        fp = self.footprint(req)
        with lock:
            live["used"] += fp
            live["n"] += 1
            live["peak"] = max(live["peak"], live["used"])
            live["nmax"] = max(live["nmax"], live["n"])
        time.sleep(0.02)
        with lock:
            live["used"] -= fp
            live["n"] -= 1
        return serve.Result(e=float(req.chi), g=np.zeros(1), x=np.zeros(1),
                            ctm_iters=0, delta=0.0, cg_iters=0, warm=False,
                            arrival=req.arrival, start=start,
                            finish=time.perf_counter())

    monkeypatch.setattr(serve.Server, "_step", fake_step)
    reqs = [_req(D, chi) for D, chi in
            [(6, 72), (3, 18), (4, 32), (6, 108), (3, 27), (5, 50), (4, 48),
             (3, 18), (5, 75), (6, 72)]]
    big = max(serve.request_footprint(r, 0) for r in reqs)
    budget = 1.2 * big
    srv = serve.Server(budget, workers=3)
    futs = [srv.submit(r) for r in reqs]
    out = [f.result(timeout=30) for f in futs]
    srv.close()
    assert [r.e for r in out] == [float(r.chi) for r in reqs]
    assert live["peak"] <= budget + 1.0
    assert srv.peak_used <= budget + 1.0
    assert 1 <= live["nmax"] <= 3 and srv.max_running <= 3


def test_request_over_budget_is_rejected():
    srv = serve.Server(1e6, workers=1)
    f = srv.submit(_req(4, 32))
    with pytest.raises(MemoryError):
        f.result(timeout=5)
    srv.close()


def test_request_stream_is_seeded():
    a = serve.request_stream(8, 20.0, 5, binding.FP32)
    b = serve.request_stream(8, 20.0, 5, binding.FP32)
    assert [t for t, _ in a] == [t for t, _ in b]
    for (_, ra), (_, rb) in zip(a, b):
        D = ra.A.shape[3]
        assert 3 <= D <= 6 and 2 * D * D <= ra.chi <= 3 * D * D
        assert ra.chi == rb.chi and np.array_equal(ra.A, rb.A)


def test_large_requests_are_checkpointed():
    """A request whose all-resident gradient exceeds budget / workers runs
    checkpointed (and is admitted with the smaller footprint); small ones
    and requests that fix the option keep their setting."""
    small, large = _req(3, 18), _req(6, 72)
    srv = serve.Server(2.0 * serve.request_footprint(large, 0), workers=4)
    try:
        assert srv.checkpoint(small) == 0
        assert srv.checkpoint(large) == 1
        assert srv.footprint(large) == serve.request_footprint(large, 1)
        assert srv.footprint(large) < 0.4 * serve.request_footprint(large, 0)
        large.grad_checkpoint = 0
        assert srv.checkpoint(large) == 0
    finally:
        srv.close()


def test_max_overlap_of_windows():
    assert serve.max_overlap([]) == 0
    assert serve.max_overlap([(0, 1), (2, 3)]) == 1
    assert serve.max_overlap([(0, 2), (1, 3), (1.5, 1.8)]) == 3
    # touching windows do not overlap
    assert serve.max_overlap([(0, 1), (1, 2)]) == 1


def test_worker_errors_reach_the_caller():
    """A request that fails inside its worker process (here: no GPU, so
    ctm_init fails; with a GPU: arguments the library rejects) fails its
    future with the library's message; the worker keeps serving."""
    srv = serve.Server(1e12, workers=1)
    bad = _req(3, 18)
    bad.chi = 0  # rejected by ctm_init before any device call
    try:
        for _ in range(2):
            with pytest.raises(RuntimeError, match="ctm_init"):
                srv.submit(bad).result(timeout=120)
        assert srv._procs[0] is not None and srv._procs[0][0].is_alive()
    finally:
        srv.close()
    assert srv._procs == [None]


def test_dead_worker_fails_only_its_request():
    """A worker that is gone when its request is sent fails that request
    with the exit code; the slot starts a new worker for the next one."""
    srv = serve.Server(1e12, workers=1)
    bad = _req(3, 18)
    bad.chi = 0
    try:
        srv.start()
        proc = srv._procs[0][0]
        proc.terminate()
        proc.join(timeout=30)
        with pytest.raises(RuntimeError, match="worker 0 ended"):
            srv.submit(bad).result(timeout=120)
        with pytest.raises(RuntimeError, match="ctm_init"):
            srv.submit(bad).result(timeout=120)
        assert srv._procs[0][0] is not proc and srv._procs[0][0].is_alive()
    finally:
        srv.close()


def test_environment_routing_and_eviction():
    """Scheduler bookkeeping of the resident environments: a request with a
    known key goes to the worker that holds it when that worker is free,
    eviction tells the holding worker to drop the key and returns the
    bytes to the budget."""
    srv = serve.Server(1e9, workers=3)
    try:
        with srv.cv:
            srv.envs["k"] = ((1, 1, 2, 3, 18), 0, 4e8)
            srv.env_bytes = srv.used = 4e8
            r = _req(3, 18, key="k")
            assert srv._pick_slot(r) == 0 and 0 not in srv._free_slots
            # the holder is busy now: another worker, cold
            assert srv._pick_slot(r) in (1, 2)
            srv._free_slots = [0, 1, 2]
            assert srv._evict_for(8e8)
            assert srv._drops[0] == ["k"] and not srv.envs
            assert srv.used == 0.0 and srv.env_bytes == 0.0
    finally:
        srv.close()


def test_sweep_stream_shares_keys_per_state():
    """The coupling sweep: every state at every coupling, one state_key per
    state, couplings round robin over the states, seeded."""
    a = serve.sweep_stream(3, 4, 20.0, 7, binding.FP32)
    b = serve.sweep_stream(3, 4, 20.0, 7, binding.FP32)
    assert len(a) == 12 and [t for t, _ in a] == [t for t, _ in b]
    keys = [r.state_key for _, r in a]
    assert keys[:3] == keys[3:6] == keys[9:12] and len(set(keys)) == 3
    for i, (_, r) in enumerate(a):
        same = a[i % 3][1]
        assert np.array_equal(r.A, same.A) and r.chi == same.chi
        D = r.A.shape[3]
        assert 3 <= D <= 6 and 2 * D * D <= r.chi <= 3 * D * D
    # the couplings rise from 0 to 0.6 across the rounds (the J2 term's
    # coefficient of the diagonal terms)
    j2 = [([t[4] for t in r.terms if t[2] == 1 and abs(t[3]) == 1] or
           [0.0])[0] for _, r in a[::3]]
    assert j2[0] == 0.0 and abs(j2[-1] - 0.6) < 1e-12
    assert all(x < y for x, y in zip(j2, j2[1:]))


def test_requests_of_a_running_state_wait_for_it(monkeypatch):
    """Requests that share a state_key never run at the same time (each
    can start from the environment of the one before); requests of other
    states go ahead of them."""
    lock = threading.Lock()
    running, seen, order = {}, [], []

    def fake_step(self, req, start, sidx=0):
        with lock:
            running[req.state_key] = running.get(req.state_key, 0) + 1
            seen.append(running[req.state_key])
            order.append(req.state_key)
        time.sleep(0.05)
        with lock:
            running[req.state_key] -= 1
        return serve.Result(e=0.0, g=np.zeros(1), x=np.zeros(1), ctm_iters=0,
                            delta=0.0, cg_iters=0, warm=False,
                            arrival=req.arrival, start=start,
                            finish=time.perf_counter())

    monkeypatch.setattr(serve.Server, "_step", fake_step)
    srv = serve.Server(1e15, workers=4)
    reqs = [_req(3, 18, key="a") for _ in range(3)] + [_req(3, 18, key="b")]
    futs = [srv.submit(r) for r in reqs]
    for f in futs:
        f.result(timeout=30)
    srv.close()
    assert max(seen) == 1
    # "b" arrived last but did not wait behind the queued "a" requests
    assert order.index("b") < 3
