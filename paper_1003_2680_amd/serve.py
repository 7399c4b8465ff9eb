"""Serving loop: sample and solve requests on grids of different sizes, as they arrive.

* Device-resident pools: one hierarchy per grid shape with S chain slots (its components),
  kept on the device between requests; idle pools are evicted least-recently-used when a new
  shape needs room.
* Admission by HBM budget: a pool is created only if the bytes of every live pool plus its own
  fit the budget; a request whose shape has no pool (and no room for one) waits.
* Continuous batching: a pool advances all its active sample chains together in rounds of
  `stride` cycles (one batched launch sequence per round).  Solve requests of one pool are
  solved together between rounds (they share the server's rtol).  A request that arrives while
  others run joins at the next round in a free slot; a finished chain's slot is refilled
  immediately (the last active chain moves into it, so active slots stay contiguous).  Queued
  solves of a shape are solved together in one batched solve between rounds.
* Each pool has its own host thread and HIP stream, so pools overlap on the device.  A pool is
  built (host plan, workspace, table upload) on its own thread; requests routed to it wait in
  its queue meanwhile.
* Admission runs on the server's own thread: submitting a request only queues it, so the
  thread that receives requests never waits for a plan, an upload, an eviction or the device.
  The admission thread sizes a new shape's pool (host planning) outside the server's lock, so
  a submission does not wait for that either.
  A solve's right-hand side may come as a generator (`make_f`) that the pool calls on its own
  stream.

A sample request of k samples on seed s gets exactly what a hierarchy of one component with
stride = burn_in = `stride` produces alone: samples at cycles 2*stride, 3*stride, ... of chain
(s, first cycle 0).  A solve gets exactly the result of solving alone.  Latency is measured
from the request's arrival time (in the simulated stream: its scheduled Poisson arrival, not
the moment the submitting thread got to it) to the end of the round (or solve) that completes
it, so time spent queued anywhere is counted.
"""
import collections
import threading
import time

import numpy as np
import torch

from . import abi
from .api import Hierarchy, plan_bytes


class Request:
    __slots__ = ("rid", "dims", "kind", "k", "seed", "rtol", "f", "make_f", "t_arrival",
                 "t_done", "result", "info", "error")

    def __init__(self, rid, dims, kind, seed, k=1, rtol=1e-10, f=None, make_f=None):
        self.rid = rid
        self.dims = tuple(int(d) for d in dims)
        self.kind = kind              # "sample" or "solve"
        self.k = int(k)
        self.seed = int(seed)
        self.rtol = float(rtol)
        self.f = f                    # solve right-hand side, device float64 [nz, ny, nx]
        self.make_f = make_f          # or a generator of it, called by the pool on its stream
        self.t_arrival = None
        self.t_done = None
        self.result = None            # samples [k, nz, ny, nx] float32, or u [nz, ny, nx]
        self.info = None
        self.error = None


class _Chain:
    __slots__ = ("req", "cycle", "rounds", "emitted")

    def __init__(self, req):
        self.req = req
        self.cycle = 0        # cycles run so far
        self.rounds = 0
        self.emitted = 0


class Pool:
    def __init__(self, server, dims):
        self.server = server
        self.dims = dims
        self.bytes = server.pool_bytes(dims)
        self.H = None                          # built on the pool's own thread
        self.stream = None
        self.state = None
        self.chains = []                       # active sample chains, slot = index
        self._fresh = []                       # slots admitted since the last round
        self.samples = collections.deque()     # waiting sample requests
        self.solves = collections.deque()      # waiting solve requests
        self.cv = threading.Condition()
        self.last_used = time.perf_counter()
        self.stop = False
        self.thread = threading.Thread(target=self._run, daemon=True)
        self.thread.start()

    def idle(self):
        with self.cv:
            return not self.chains and not self.samples and not self.solves

    def submit(self, req):
        with self.cv:
            (self.samples if req.kind == "sample" else self.solves).append(req)
            self.cv.notify()

    def shutdown(self):
        with self.cv:
            self.stop = True
            self.cv.notify()
        self.thread.join()

    # ---------------------------------------------------------------- worker
    def _build(self):
        server = self.server
        self.stream = torch.cuda.Stream(device=server.device)
        with torch.cuda.stream(self.stream):
            self.H = Hierarchy(*self.dims, ncomp=server.slots, kT=server.kT, levels=0, nu1=2,
                               nu2=2, stride=server.stride, precision=server.precision,
                               device=server.device)
            self.state = torch.zeros(self.H.shape, dtype=torch.float64, device=server.device)
        self.stream.synchronize()

    def _run(self):
        try:
            torch.cuda.set_device(self.server.device)
            self._build()
            self._loop()
        except Exception as e:  # a dead worker must not leave requests pending
            with self.cv:
                pending = [c.req for c in self.chains] + list(self.samples) + list(self.solves)
                self.chains, self.samples, self.solves = [], collections.deque(), collections.deque()
            for r in pending:
                r.error = "pool worker failed: %r" % (e,)
                self.server._complete(r)

    def _loop(self):
        while True:
            with self.cv:
                while not self.stop and not self.chains and not self.samples and not self.solves:
                    self.cv.wait()
                if self.stop:
                    return
                # admission into free slots (continuous batching)
                while self.samples and len(self.chains) < self.server.slots:
                    self.chains.append(_Chain(self.samples.popleft()))
                    self._fresh.append(len(self.chains) - 1)
                solves = []
                while self.solves and len(solves) < self.server.slots:
                    solves.append(self.solves.popleft())
            self.last_used = time.perf_counter()
            try:
                with torch.cuda.stream(self.stream):
                    if solves:
                        self._solve(solves)
                    if self.chains:
                        self._round()
            except Exception as e:  # report on every request involved, keep serving
                for r in solves + [c.req for c in self.chains]:
                    r.error = repr(e)
                    self.server._complete(r)
                with self.cv:
                    self.chains = []
            self.last_used = time.perf_counter()

    def _solve(self, reqs):
        n = len(reqs)
        for r in reqs:
            if r.f is None:
                r.f = r.make_f(r)   # drawn on this pool's stream
        f = torch.stack([r.f for r in reqs]).contiguous()
        u, infos = self.H.solve_batch(f, nchains=n, comps_per_chain=1, rtol=reqs[0].rtol,
                                      raise_on_notconv=False)
        self.stream.synchronize()
        for k, r in enumerate(reqs):
            r.result = u[k]
            r.info = infos[k]
            self.server._complete(r)

    def _round(self):
        stride = self.server.stride
        nact = len(self.chains)
        for i in self._fresh:
            self.state[i].zero_()
        self._fresh.clear()
        out = torch.empty((1, nact) + self.H.shape[1:], dtype=torch.float32,
                          device=self.server.device)
        self.H.sample_batch(1, seeds=[c.req.seed for c in self.chains],
                            first_cycles=[c.cycle for c in self.chains], comps_per_chain=1,
                            state=self.state[:nact], out=out, out_dtype=torch.float32)
        done = []
        for i, c in enumerate(self.chains):
            c.cycle += stride
            c.rounds += 1
            if c.rounds >= 2:   # the first round is the burn-in
                if c.req.result is None:
                    c.req.result = torch.empty((c.req.k,) + self.H.shape[1:],
                                               dtype=torch.float32, device=self.server.device)
                c.req.result[c.emitted].copy_(out[0, i])
                c.emitted += 1
                if c.emitted == c.req.k:
                    done.append(i)
        self.stream.synchronize()
        with self.cv:
            # retire finished chains; the last active chain moves into each freed slot
            for i in sorted(done, reverse=True):
                req = self.chains[i].req
                last = len(self.chains) - 1
                if i != last:
                    self.state[i].copy_(self.state[last])
                    self.chains[i] = self.chains[last]
                self.chains.pop()
                self.server._complete(req)
        if done:
            self.stream.synchronize()


def pool_bytes(dims, slots, precision):
    """Device bytes of a pool: the hierarchy's workspace and the chain states."""
    ws = plan_bytes(dims, slots, precision)
    return ws + slots * dims[0] * dims[1] * dims[2] * 8


class Server:
    """Serves requests with per-shape pools inside an HBM budget (bytes)."""

    def __init__(self, budget_bytes=32 << 30, slots=16, stride=2, precision="fp32_refined",
                 kT=1.0, device=None):
        dev = torch.device(device if device is not None else "cuda")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.stride = int(stride)
        self.precision = precision
        self.kT = kT
        self.pools = collections.OrderedDict()   # dims -> Pool (LRU order)
        self.waiting = collections.deque()       # requests whose shape has no pool yet
        self.lock = threading.Lock()
        self.admit_cv = threading.Condition(self.lock)
        self.done = []
        self.done_cv = threading.Condition()
        self.evictions = 0
        self._bytes = {}                         # dims -> pool bytes, or the planning error
        self._stop = False
        self._admitter = threading.Thread(target=self._admit_loop, daemon=True)
        self._admitter.start()

    def pool_bytes(self, dims):
        b = self._bytes.get(dims)
        if b is None:
            b = self._bytes[dims] = pool_bytes(dims, self.slots, self.precision)
        return b

    def used_bytes(self):
        return sum(p.bytes for p in self.pools.values())

    def submit(self, req):
        """Queue a request for admission (never blocks on the device or on planning)."""
        req.t_arrival = time.perf_counter() if req.t_arrival is None else req.t_arrival
        with self.lock:
            self.waiting.append(req)
            self.admit_cv.notify()

    def _admit_loop(self):
        while True:
            with self.lock:
                if self._stop:
                    return
                unplanned = {r.dims for r in self.waiting if r.dims not in self._bytes}
            # host planning of new shapes outside the lock, so a submission never waits for it;
            # a shape that cannot be planned fails its requests, not the admission thread
            for dims in unplanned:
                try:
                    self.pool_bytes(dims)
                except Exception as e:
                    self._bytes[dims] = e
            with self.lock:
                if self._stop:
                    return
                if self.waiting:
                    self._dispatch()
                # woken by a submission; polls while requests wait (a pool may go idle, a
                # shape may still need planning)
                self.admit_cv.wait(0.002 if self.waiting else None)

    def _dispatch(self):
        """Route waiting requests to pools, creating pools inside the budget (lock held, on
        the admission thread; shapes not yet planned wait for the next pass)."""
        keep = collections.deque()
        while self.waiting:
            req = self.waiting.popleft()
            pool = self.pools.get(req.dims)
            if pool is None:
                need = self._bytes.get(req.dims)
                if need is None:            # planned outside the lock on the next pass
                    keep.append(req)
                    continue
                if isinstance(need, Exception):
                    req.error = "shape cannot be planned: %r" % (need,)
                    self._complete(req)
                    continue
                if need > self.budget:
                    req.error = "request does not fit the HBM budget"
                    self._complete(req)
                    continue
                # evict idle pools, least recently used first, until the new one fits
                while self.used_bytes() + need > self.budget:
                    idle = [d for d, p in self.pools.items() if p.idle()]
                    if not idle:
                        break
                    victim = min(idle, key=lambda d: self.pools[d].last_used)
                    self.pools.pop(victim).shutdown()
                    self.evictions += 1
                if self.used_bytes() + need > self.budget:
                    keep.append(req)        # admitted later, when a pool goes idle
                    continue
                pool = Pool(self, req.dims)
                self.pools[req.dims] = pool
            self.pools.move_to_end(req.dims)
            pool.submit(req)
        self.waiting = keep

    def _complete(self, req):
        # called from pool threads (or the admission thread, lock held): never dispatches
        # itself; waiting requests are retried by the admission thread, which polls while any
        # wait
        req.t_done = time.perf_counter()
        with self.done_cv:
            self.done.append(req)
            self.done_cv.notify_all()

    def wait(self, n, timeout=120.0, poll=0.002):
        """Block until n requests completed."""
        t_end = time.perf_counter() + timeout
        while True:
            with self.done_cv:
                if len(self.done) >= n:
                    return True
                self.done_cv.wait(poll)
            if time.perf_counter() > t_end:
                return False

    def shutdown(self):
        with self.lock:
            self._stop = True
            self.admit_cv.notify()
        self._admitter.join()
        with self.lock:
            for p in self.pools.values():
                p.shutdown()
            self.pools.clear()


def make_requests(n, rate, seed=7, nxy=(32, 64, 128, 256), nzs=(16, 32, 64, 128), kmax=16,
                  sample_frac=0.5, rtol=1e-10):
    """A seeded Poisson request stream: (arrival offset s, Request without f)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    reqs = []
    for i in range(n):
        nx = int(rng.choice(nxy))
        nz = int(rng.choice(nzs))
        kind = "sample" if rng.random() < sample_frac else "solve"
        k = int(rng.integers(1, kmax + 1))
        reqs.append((float(t[i]), Request(i, (nx, nx, nz), kind, seed=1000 + i, k=k, rtol=rtol)))
    return reqs


def simulate(server, timed_requests, make_f, timeout=120.0):
    """Submit requests at their arrival offsets (real time).  A request's arrival time is its
    scheduled time t0 + offset, whenever the submitting thread gets to it, so a late submission
    still counts its delay; solve right-hand sides are drawn by the pools (make_f).  Returns
    (all completed, wall time from the start to the last completion, latencies in s); the
    largest lag of a submission behind its schedule is left in server.max_submit_lag (s)."""
    t0 = time.perf_counter()
    lag = 0.0
    for off, req in timed_requests:
        while True:
            now = time.perf_counter() - t0
            if off <= now:
                break
            time.sleep(min(0.002, off - now))
        if req.kind == "solve" and req.f is None and req.make_f is None:
            req.make_f = make_f
        req.t_arrival = t0 + off
        lag = max(lag, time.perf_counter() - req.t_arrival)
        server.submit(req)
    server.max_submit_lag = lag
    ok = server.wait(len(timed_requests), timeout=timeout)
    wall = time.perf_counter() - t0
    lat = np.array([r.t_done - r.t_arrival for r in server.done])
    return ok, wall, lat


def main(argv=None):
    """Rate sweep of the serving loop: one JSON line per arrival rate."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--rates", default="50,100,200,500,1000,2000")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--stride", type=int, default=2, help="burn-in = stride of sample requests")
    ap.add_argument("--slots", type=int, default=16)
    ap.add_argument("--budget-gb", type=float, default=32.0)
    ap.add_argument("--precision", default="fp32_refined")
    ap.add_argument("--timeout", type=float, default=300.0)
    args = ap.parse_args(argv)
    from .inputs import gaussian_field_device
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    for rate in [float(r) for r in args.rates.split(",")]:
        srv = Server(budget_bytes=int(args.budget_gb * (1 << 30)), slots=args.slots,
                     stride=args.stride, precision=args.precision, device=dev)
        reqs = make_requests(args.requests, rate, seed=7)
        ok, wall, lat = simulate(
            srv, reqs, lambda r: gaussian_field_device(r.dims[::-1], r.seed, dev),
            timeout=args.timeout)
        kinds = {"sample": [], "solve": []}
        for r in srv.done:
            kinds[r.kind].append(r.t_done - r.t_arrival)
        errors = sum(1 for r in srv.done if r.error)
        line = {"rate_req_s": rate, "requests": args.requests, "completed": len(lat),
                "errors": errors, "all_completed": bool(ok),
                "throughput_req_s": round(len(lat) / wall, 2),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
                "sample_p50_ms": round(float(np.percentile(kinds["sample"], 50)) * 1e3, 2)
                if kinds["sample"] else None,
                "solve_p50_ms": round(float(np.percentile(kinds["solve"], 50)) * 1e3, 2)
                if kinds["solve"] else None,
                "pools_created": len(srv.pools) + srv.evictions, "evictions": srv.evictions,
                "max_submit_lag_ms": round(srv.max_submit_lag * 1e3, 2)}
        srv.shutdown()
        torch.cuda.empty_cache()
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
