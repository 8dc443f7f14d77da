"""Request loop: many independent preconditioned steps sharing one GPU.

Each request is one step of the method on its own state (CTMRG environment,
energy and K-step gradient, preconditioned direction; Sec. III) and runs in
its own library context in one of `workers` worker processes (started once,
with the spawn method; each context on a stream of its own), so up to
`workers` requests execute concurrently and their kernels overlap on the
device, from separate processes: every process issues its launches from one
host thread.  Requests that arrive while others run are admitted as soon as
a worker and enough memory are free.  Admission follows the device-memory
footprint that ipeps_footprint_bytes predicts for each request: a request
starts only when its footprint fits the budget next to those already
running and the cached environments (first come first served; later
requests may start ahead of a waiting large one when they fit).  Contexts
are freed when their request ends, and each worker then returns the memory
its finished contexts left cached beyond a small reserve to HIP
(ipeps_release_cache), so that the budget stays the only large holder.  A
worker that dies fails its request only; it is started again for the next.

Checkpointing: a request whose gradient with every unrolled iteration
resident would take more than its share of the budget (budget / workers)
runs with the checkpointed gradient (ipeps_opts.grad_checkpoint: one
iteration resident, recomputed in the backward pass), unless the request
fixes grad_checkpoint itself.

Warm starts: a request that carries a `state_key` seen before (same cell,
D and chi) starts CTMRG from the environment that the earlier request left;
while a request of that key runs, later ones of the key wait for it
(others go ahead), so that they can start from its environment.
Those environments stay resident in device memory, in the worker process
that computed them (ipeps_get_env_dev / ipeps_set_env_dev into device
buffers of their own, hipMalloc); a request with a known key goes to that worker when it is free
(elsewhere it starts cold and its environment replaces the old one).  They
count against the budget, and the least recently used ones are dropped when
a waiting request needs the room.  The environment depends only on the
state, not on the Hamiltonian, so a sweep of couplings on one state
converges in a few iterations after the first request.

Every request records the host clock (CLOCK_MONOTONIC, common to all
processes) right before its context is created and right after its last
call returned (every library call waits for its stream), as
`Result.window` in milliseconds after the server started: the interval
holds all of the request's device work, so overlapping windows are
requests whose work shared the device.

    python -m paper_2511_09546_amd.serve [--requests 256] [--rate 20]
        [--workers 8] [--prec fp32] [--budget-gb 230] [--seed 5]
        [--check-solo 16] [--sweep STATES COUPLINGS]

replays a seeded stream of requests (exponential inter-arrival times, D in
3..6, chi in 2D^2..3D^2, J1-J2 with J2 in [0, 0.6], random states) in real
time and prints one JSON line: latency percentiles (finish - arrival),
throughput, the admission statistics, the overlap of the request windows,
and how many of a sample of requests gave bitwise the results of the same
request run alone.
"""
from __future__ import annotations

import argparse
import collections
import concurrent.futures as cf
import ctypes
import json
import multiprocessing
import sys
import threading
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import binding


@dataclass
class Request:
    A: np.ndarray                 # [Ly][Lx][d][D][D][D][D]
    chi: int
    terms: list                   # (kind, site, dx, dy, coef, mat) tuples
    tol: float = 1e-10
    max_iter: int = 200
    delta: float = 1e-4
    cg_tol: float = 0.0
    cg_maxiter: int = 20
    prec: int = binding.FP32
    grad_K: int = 20
    grad_checkpoint: Optional[int] = None   # None: the server decides
    state_key: Optional[str] = None
    arrival: float = field(default_factory=time.perf_counter)


@dataclass
class Result:
    e: float
    g: np.ndarray
    x: np.ndarray
    ctm_iters: int
    delta: float
    cg_iters: int
    warm: bool
    arrival: float
    start: float
    finish: float
    window: tuple = (0.0, 0.0)    # device work within, ms after the start

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


def _shape(A):
    """(Lx, Ly, d, D) of a state [Ly][Lx][d][D][D][D][D]."""
    A = np.asarray(A)
    if A.ndim != 7:
        raise ValueError("A must be [Ly, Lx, d, D, D, D, D]")
    return A.shape[1], A.shape[0], A.shape[2], A.shape[3]


def request_footprint(req: Request, ckpt: int) -> float:
    """Device bytes of one request (ipeps_footprint_bytes)."""
    Lx, Ly, d, D = _shape(req.A)
    o = binding.default_opts()
    o.grad_K = req.grad_K
    o.grad_checkpoint = ckpt
    return float(binding.footprint_bytes(Lx, Ly, d, D, req.chi, o))


def max_overlap(windows) -> int:
    """Largest number of device-work windows [a, b] open at one time."""
    ev = sorted([(a, 1) for a, _ in windows] + [(b, -1) for _, b in windows],
                key=lambda t: (t[0], t[1]))
    cur = best = 0
    for _, s in ev:
        cur += s
        best = max(best, cur)
    return best


# Device memory that a worker keeps cached after each request (of what its
# finished contexts left, ipeps_release_cache): its next context allocates
# from it first.
WORKER_CACHE_BYTES = 2 << 30


class _DeviceBuffer:
    """Device memory of a worker's resident environment (hipMalloc /
    hipFree of the HIP runtime the library uses; no caching allocator, so
    a dropped environment goes straight back to HIP)."""
    _hip = None

    def __init__(self, nbytes: int):
        if _DeviceBuffer._hip is None:
            # the runtime libipeps.so is linked against (same soname)
            try:
                _DeviceBuffer._hip = ctypes.CDLL("libamdhip64.so.7")
            except OSError:
                _DeviceBuffer._hip = ctypes.CDLL("libamdhip64.so")
            _DeviceBuffer._hip.hipMalloc.argtypes = [
                ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
            _DeviceBuffer._hip.hipFree.argtypes = [ctypes.c_void_p]
        p = ctypes.c_void_p()
        st = _DeviceBuffer._hip.hipMalloc(ctypes.byref(p), nbytes)
        if st != 0 or not p.value:
            raise MemoryError(f"hipMalloc of {nbytes} bytes: status {st}")
        self.ptr, self.nbytes = p.value, nbytes

    def data_ptr(self) -> int:
        return self.ptr

    def free(self) -> None:
        if self.ptr:
            _DeviceBuffer._hip.hipFree(self.ptr)
            self.ptr = 0


def _worker_run(msg: dict, envs: dict) -> dict:
    """One request inside a worker process (envs: the worker's resident
    environments, state_key -> (shape key, device buffer))."""
    o = binding.default_opts()
    o.prec = msg["prec"]
    o.grad_K = msg["grad_K"]
    o.grad_checkpoint = msg["ckpt"]
    skey, shape = msg["state_key"], msg["shape"]
    warm, nbytes = False, 0
    t0 = time.perf_counter()
    with binding.Context(msg["A"], msg["chi"], opts=o) as ctx:
        held = envs.get(skey) if skey is not None else None
        if held is not None and held[0] == shape:
            ctx.set_env_dev(held[1].data_ptr())
            warm = True
        it, dl, ok = ctx.converge(msg["tol"], msg["max_iter"])
        if skey is not None:
            old = envs.pop(skey, None)
            if old is not None:
                old[1].free()
            buf = _DeviceBuffer(ctx.env_size() * 8)
            envs[skey] = (shape, buf)
            ctx.get_env_dev(buf.data_ptr())
            nbytes = buf.nbytes
        e, g = ctx.energy_grad(msg["terms"], grad=True)
        x, cg_it, res, brk = ctx.precond(g, msg["delta"], msg["cg_tol"],
                                         msg["cg_maxiter"])
    t1 = time.perf_counter()
    return dict(e=e, g=g, x=x, it=it, delta=dl, cg=cg_it, warm=warm, t0=t0,
                t1=t1, env_bytes=nbytes)


def _worker_main(conn) -> None:
    """Worker process: requests in, ("ok", result) or ("err", message) out,
    until None or the end of the pipe."""
    binding.load()
    envs: dict = {}
    while True:
        try:
            msg = conn.recv()
        except EOFError:
            return
        if msg is None:
            return
        for k in msg["drop"]:
            held = envs.pop(k, None)
            if held is not None:
                held[1].free()
        try:
            out = ("ok", _worker_run(msg, envs))
        except Exception as ex:  # delivered to the caller
            out = ("err", f"{type(ex).__name__}: {ex}")
        try:
            binding.release_cache(WORKER_CACHE_BYTES)
        except Exception as ex:
            if out[0] == "ok":
                out = ("err", f"{type(ex).__name__}: {ex}")
        conn.send(out)


class Server:
    """Footprint-admitted concurrent execution of Requests."""

    def __init__(self, budget_bytes: float, workers: int = 8):
        binding.load()
        self.budget = float(budget_bytes)
        self.used = 0.0
        self.workers = workers
        self.running = 0
        self.queue = collections.deque()
        self.cv = threading.Condition()
        # state_key -> (shape key, worker, bytes), least recently used first
        self.envs = collections.OrderedDict()
        self.env_bytes = 0.0
        self.pool = cf.ThreadPoolExecutor(max_workers=workers)
        self.closed = False
        self.peak_used = 0.0
        self.max_running = 0
        self._procs = [None] * workers   # (process, pipe end), on first use
        self._drops = [[] for _ in range(workers)]  # keys to drop, per worker
        self._free_slots = list(range(workers))
        self._running_keys = set()     # state_keys of running requests
        self._t0 = time.perf_counter()
        self.sched = threading.Thread(target=self._schedule, daemon=True)
        self.sched.start()

    def checkpoint(self, req: Request) -> int:
        """Checkpointed gradient for this request (see the module doc)."""
        if req.grad_checkpoint is not None:
            return int(req.grad_checkpoint)
        return int(request_footprint(req, 0) > self.budget / self.workers)

    def footprint(self, req: Request) -> float:
        return request_footprint(req, self.checkpoint(req))

    def submit(self, req: Request) -> cf.Future:
        fut = cf.Future()
        fp = self.footprint(req)
        if fp > self.budget:
            fut.set_exception(MemoryError(
                f"request needs {fp / 1e9:.1f} GB, budget "
                f"{self.budget / 1e9:.1f} GB"))
            return fut
        with self.cv:
            self.queue.append((req, fp, fut))
            self.cv.notify_all()
        return fut

    def start(self) -> None:
        """Starts every worker process now (otherwise each on its first
        request), so that their start-up is not part of request times."""
        for i in range(self.workers):
            self._worker(i)

    def _worker(self, sidx: int):
        """(process, pipe end) of worker sidx, started if needed (only the
        thread that holds slot sidx calls this, or start() before any)."""
        if self._procs[sidx] is None:
            mp = multiprocessing.get_context("spawn")
            here, there = mp.Pipe()
            proc = mp.Process(target=_worker_main, args=(there,), daemon=True)
            proc.start()
            there.close()
            self._procs[sidx] = (proc, here)
        return self._procs[sidx]

    def _lost_worker(self, sidx: int) -> int:
        """Forgets worker sidx after it died and the environments it held;
        returns its exit code."""
        proc, conn = self._procs[sidx]
        self._procs[sidx] = None
        conn.close()
        proc.join(timeout=10)
        with self.cv:
            for k in [k for k, v in self.envs.items() if v[1] == sidx]:
                nbytes = self.envs.pop(k)[2]
                self.env_bytes -= nbytes
                self.used -= nbytes
            self._drops[sidx] = []
        return proc.exitcode

    def _evict_for(self, fp: float) -> bool:
        """Drop least recently used environments until fp fits (cv held)."""
        while self.envs and self.used + fp > self.budget:
            key, (_, sidx, nbytes) = self.envs.popitem(last=False)
            self._drops[sidx].append(key)
            self.env_bytes -= nbytes
            self.used -= nbytes
        return self.used + fp <= self.budget

    def _pick_slot(self, req: Request) -> int:
        """A free worker, the one holding the request's environment when it
        is free (cv held)."""
        held = self.envs.get(req.state_key) if req.state_key else None
        if held is not None and held[1] in self._free_slots:
            self._free_slots.remove(held[1])
            return held[1]
        return self._free_slots.pop()

    def _schedule(self):
        while True:
            with self.cv:
                while True:
                    if self.closed and not self.queue:
                        return
                    pick = None
                    if self.running < self.workers:
                        for i, (req, fp, fut) in enumerate(self.queue):
                            # a request whose state is being computed waits
                            # for it, to start from its environment
                            if req.state_key in self._running_keys:
                                continue
                            if self.used + fp <= self.budget:
                                pick = i
                                break
                        if pick is None and self.queue and self.running == 0:
                            # nothing runs: room can only come from the
                            # environment cache
                            if self._evict_for(self.queue[0][1]):
                                pick = 0
                    if pick is not None:
                        break
                    self.cv.wait()
                req, fp, fut = self.queue[pick]
                del self.queue[pick]
                if req.state_key is not None:
                    self._running_keys.add(req.state_key)
                self.used += fp
                self.running += 1
                self.peak_used = max(self.peak_used, self.used)
                self.max_running = max(self.max_running, self.running)
                sidx = self._pick_slot(req)
            self.pool.submit(self._run, req, fp, fut, sidx)

    def _run(self, req: Request, fp: float, fut: cf.Future, sidx: int = 0):
        start = time.perf_counter()
        try:
            res = self._step(req, start, sidx)
            fut.set_result(res)
        except BaseException as ex:  # delivered to the caller
            fut.set_exception(ex)
        finally:
            with self.cv:
                self.used -= fp
                self.running -= 1
                self._free_slots.append(sidx)
                self._running_keys.discard(req.state_key)
                self.cv.notify_all()

    def _step(self, req: Request, start: float, sidx: int = 0) -> Result:
        proc, conn = self._worker(sidx)
        Lx, Ly, d, D = _shape(req.A)
        shape = (Lx, Ly, d, D, req.chi)
        with self.cv:
            drop, self._drops[sidx] = self._drops[sidx], []
            if req.state_key in self.envs:
                self.envs.move_to_end(req.state_key)
        msg = dict(A=np.asarray(req.A), chi=req.chi, terms=req.terms,
                   tol=req.tol, max_iter=req.max_iter, delta=req.delta,
                   cg_tol=req.cg_tol, cg_maxiter=req.cg_maxiter,
                   prec=req.prec, grad_K=req.grad_K,
                   ckpt=self.checkpoint(req), state_key=req.state_key,
                   shape=shape, drop=drop)
        try:
            conn.send(msg)
            status, out = conn.recv()
        except (EOFError, OSError) as ex:
            code = self._lost_worker(sidx)
            raise RuntimeError(f"worker {sidx} ended (exit code {code}) "
                               "during the request") from ex
        if status != "ok":
            raise RuntimeError(out)
        if req.state_key is not None:
            with self.cv:
                old = self.envs.pop(req.state_key, None)
                if old is not None:
                    self.env_bytes -= old[2]
                    self.used -= old[2]
                    if old[1] != sidx:
                        self._drops[old[1]].append(req.state_key)
                self.envs[req.state_key] = (shape, sidx, out["env_bytes"])
                self.env_bytes += out["env_bytes"]
                self.used += out["env_bytes"]
                self.peak_used = max(self.peak_used, self.used)
        ms = lambda t: (t - self._t0) * 1e3  # noqa: E731
        return Result(e=out["e"], g=out["g"], x=out["x"], ctm_iters=out["it"],
                      delta=out["delta"], cg_iters=out["cg"],
                      warm=out["warm"], arrival=req.arrival, start=start,
                      finish=time.perf_counter(),
                      window=(ms(out["t0"]), ms(out["t1"])))

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        self.sched.join()
        self.pool.shutdown(wait=True)
        for i, w in enumerate(self._procs):
            if w is None:
                continue
            proc, conn = w
            try:
                conn.send(None)
            except OSError:
                pass
            proc.join(timeout=30)
            if proc.is_alive():
                proc.terminate()
                proc.join(timeout=10)
            conn.close()
            self._procs[i] = None


def request_stream(n: int, rate: float, seed: int, prec: int):
    """(offset seconds, Request) of the seeded serving workload: exponential
    inter-arrivals of mean 1/rate, D uniform in 3..6, chi uniform in
    2D^2..3D^2, J1 = 1, J2 uniform in [0, 0.6], state seed 5000 + i."""
    from . import inputs
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate)
        D = int(rng.integers(3, 7))
        chi = int(rng.integers(2 * D * D, 3 * D * D + 1))
        J2 = float(rng.uniform(0.0, 0.6))
        A = inputs.random_state(5000 + i, 1, 1, 2, D)
        terms = inputs.terms_j1j2(1, 1, 1.0, J2)
        out.append((t, Request(A=A, chi=chi, terms=terms, prec=prec)))
    return out


def solo(req: Request, ckpt: int):
    """(e, g, x, ctm iterations) of a request run alone on its own context."""
    o = binding.default_opts()
    o.prec = req.prec
    o.grad_K = req.grad_K
    o.grad_checkpoint = ckpt
    with binding.Context(req.A, req.chi, opts=o) as ctx:
        it, dl, ok = ctx.converge(req.tol, req.max_iter)
        e, g = ctx.energy_grad(req.terms, grad=True)
        x, cg, res, brk = ctx.precond(g, req.delta, req.cg_tol,
                                      req.cg_maxiter)
    return e, g, x, it


def sweep_stream(n_states: int, n_couplings: int, rate: float, seed: int,
                 prec: int):
    """(offset seconds, Request) of a coupling sweep: n_states random states
    (D uniform in 3..6, chi uniform in 2D^2..3D^2, state seed 6000 + s),
    each at n_couplings values of J2 evenly spaced in [0, 0.6], all requests
    of one state with one state_key (so that every one after the first can
    start from the environment the previous one left); the couplings go
    round robin over the states, with exponential inter-arrivals of mean
    1/rate."""
    from . import inputs
    rng = np.random.default_rng(seed)
    states = []
    for st in range(n_states):
        D = int(rng.integers(3, 7))
        chi = int(rng.integers(2 * D * D, 3 * D * D + 1))
        states.append((D, chi, inputs.random_state(6000 + st, 1, 1, 2, D)))
    t = 0.0
    out = []
    for c in range(n_couplings):
        J2 = 0.6 * c / max(n_couplings - 1, 1)
        for st, (D, chi, A) in enumerate(states):
            t += rng.exponential(1.0 / rate)
            out.append((t, Request(A=A, chi=chi,
                                   terms=inputs.terms_j1j2(1, 1, 1.0, J2),
                                   prec=prec, state_key=f"sweep{seed}-{st}")))
    return out


def replay(n: int, rate: float, seed: int, prec: int, workers: int,
           budget_gb: float, check_solo: int = 0, log=sys.stderr,
           sweep=None) -> dict:
    """Replays the seeded stream in real time (or, with sweep = (states,
    couplings), the coupling sweep of sweep_stream; n is then ignored);
    returns the record."""
    if sweep is not None:
        stream = sweep_stream(sweep[0], sweep[1], rate, seed, prec)
        n = len(stream)
    else:
        stream = request_stream(n, rate, seed, prec)
    # device memory this process keeps cached (contexts it has freed,
    # torch's allocator) goes back to HIP: the workers need it
    binding.release_cache(0)
    if "torch" in sys.modules:
        sys.modules["torch"].cuda.empty_cache()
    srv = Server(budget_gb * 1e9, workers)
    srv.start()
    n_ckpt = sum(srv.checkpoint(r) for _, r in stream)
    t0 = time.perf_counter()
    futs = []
    for off, req in stream:
        now = time.perf_counter() - t0
        if off > now:
            time.sleep(off - now)
        req.arrival = time.perf_counter()
        futs.append((req, srv.submit(req)))
    results, errors = [], 0
    for i, (req, f) in enumerate(futs):
        try:
            results.append((req, f.result()))
        except Exception as ex:  # counted, reported
            errors += 1
            print(f"request {i}: {ex}", file=log, flush=True)
        if (i + 1) % 32 == 0:
            print(f"{i + 1} requests done", file=log, flush=True)
    makespan = time.perf_counter() - t0
    srv.close()
    lat = np.array([r.latency for _, r in results])
    svc = np.array([r.finish - r.start for _, r in results])
    wins = [r.window for _, r in results]
    busy = sum(b - a for a, b in wins)
    if sweep is not None:
        wl = (f"coupling sweep: {sweep[0]} random states x {sweep[1]} values "
              f"of J2 in [0, 0.6] = {n} requests, Poisson arrivals at "
              f"{rate}/s (seed {seed}), D 3..6, chi 2D^2..3D^2, one "
              "state_key per state (warm starts from resident "
              "environments)")
    else:
        wl = (f"{n} requests, Poisson arrivals at {rate}/s (seed {seed}), "
              "D 3..6, chi 2D^2..3D^2, J1-J2 random states, cold starts")
    out = {
        "workload": wl,
        "requests": n, "errors": errors,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_service_s": float(svc.mean()),
        "throughput_req_per_s": len(results) / makespan,
        "makespan_s": makespan, "workers": workers,
        "budget_gb": budget_gb,
        "peak_admitted_gb": srv.peak_used / 1e9,
        "max_concurrent": srv.max_running,
        "max_concurrent_windows": max_overlap(wins),
        "device_busy_sum_over_makespan": busy / 1e3 / makespan,
        "checkpointed_requests": n_ckpt,
    }
    if sweep is not None:
        warm = [r for _, r in results if r.warm]
        cold = [r for _, r in results if not r.warm]
        out["warm_requests"] = len(warm)
        out["mean_ctm_iters_cold"] = (float(np.mean([r.ctm_iters
                                                     for r in cold]))
                                      if cold else None)
        out["mean_ctm_iters_warm"] = (float(np.mean([r.ctm_iters
                                                     for r in warm]))
                                      if warm else None)
        out["mean_service_s_cold"] = (float(np.mean([r.finish - r.start
                                                     for r in cold]))
                                      if cold else None)
        out["mean_service_s_warm"] = (float(np.mean([r.finish - r.start
                                                     for r in warm]))
                                      if warm else None)
    if check_solo > 0 and results:
        idx = np.linspace(0, len(results) - 1, min(check_solo, len(results)))
        same = 0
        for i in sorted(set(int(round(v)) for v in idx)):
            req, r = results[i]
            e, g, x, it = solo(req, srv.checkpoint(req))
            same += int(e == r.e and np.array_equal(g, r.g) and
                        np.array_equal(x, r.x) and it == r.ctm_iters)
        out["solo_checked"] = len(set(int(round(v)) for v in idx))
        out["solo_bitwise_equal"] = same
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--rate", type=float, default=20.0)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--prec", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--budget-gb", type=float, default=230.0)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--check-solo", type=int, default=16)
    ap.add_argument("--sweep", type=int, nargs=2, metavar=("STATES",
                                                           "COUPLINGS"),
                    help="replay a coupling sweep instead (warm starts)")
    args = ap.parse_args(argv)
    prec = binding.FP32 if args.prec == "fp32" else binding.FP64
    out = replay(args.requests, args.rate, args.seed, prec, args.workers,
                 args.budget_gb, 0 if args.sweep else args.check_solo,
                 sweep=tuple(args.sweep) if args.sweep else None)
    out["prec"] = args.prec
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
