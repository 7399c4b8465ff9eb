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
* Each pool has its own host thread and HIP stream, so pools overlap on the device.

A sample request of k samples on seed s gets exactly what a hierarchy of one component with
stride = burn_in = `stride` produces alone: samples at cycles 2*stride, 3*stride, ... of chain
(s, first cycle 0).  A solve gets exactly the result of solving alone.  Latency is measured
from arrival to the end of the round (or solve) that completes the request.
"""
import collections
import threading
import time

import numpy as np
import torch

from . import abi
from .api import Hierarchy, plan_bytes


class Request:
    __slots__ = ("rid", "dims", "kind", "k", "seed", "rtol", "f", "t_arrival", "t_done",
                 "result", "info", "error")

    def __init__(self, rid, dims, kind, seed, k=1, rtol=1e-10, f=None):
        self.rid = rid
        self.dims = tuple(int(d) for d in dims)
        self.kind = kind              # "sample" or "solve"
        self.k = int(k)
        self.seed = int(seed)
        self.rtol = float(rtol)
        self.f = f                    # solve right-hand side, device float64 [nz, ny, nx]
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
        S = server.slots
        self.H = Hierarchy(*dims, ncomp=S, kT=server.kT, levels=0, nu1=2, nu2=2,
                           stride=server.stride, precision=server.precision,
                           device=server.device)
        self.bytes = pool_bytes(dims, S, server.precision)
        self.stream = torch.cuda.Stream(device=server.device)
        self.state = torch.zeros(self.H.shape, dtype=torch.float64, device=server.device)
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
    def _run(self):
        try:
            torch.cuda.set_device(self.server.device)
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
        self.done = []
        self.done_cv = threading.Condition()
        self.evictions = 0

    def used_bytes(self):
        return sum(p.bytes for p in self.pools.values())

    def submit(self, req):
        req.t_arrival = time.perf_counter() if req.t_arrival is None else req.t_arrival
        with self.lock:
            self.waiting.append(req)
            self._dispatch()

    def _dispatch(self):
        """Route waiting requests to pools, creating pools inside the budget (lock held)."""
        keep = collections.deque()
        while self.waiting:
            req = self.waiting.popleft()
            pool = self.pools.get(req.dims)
            if pool is None:
                need = pool_bytes(req.dims, self.slots, self.precision)
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
        # called from pool threads: never dispatches (an eviction joins pool threads); the
        # submitting thread retries waiting requests in poll()
        req.t_done = time.perf_counter()
        with self.done_cv:
            self.done.append(req)
            self.done_cv.notify_all()

    def poll(self):
        """Retry the admission of waiting requests (a pool may have gone idle)."""
        with self.lock:
            if self.waiting:
                self._dispatch()

    def wait(self, n, timeout=120.0, poll=0.002):
        """Block until n requests completed (retrying admission of waiting ones)."""
        t_end = time.perf_counter() + timeout
        while True:
            with self.done_cv:
                if len(self.done) >= n:
                    return True
                self.done_cv.wait(poll)
            with self.lock:
                if self.waiting:
                    self._dispatch()
            if time.perf_counter() > t_end:
                return False

    def shutdown(self):
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
    """Submit requests at their arrival offsets (real time); returns the completed requests,
    the wall time from the first arrival to the last completion and the latencies (s)."""
    t0 = time.perf_counter()
    for off, req in timed_requests:
        while True:
            now = time.perf_counter() - t0
            if off <= now:
                break
            server.poll()
            time.sleep(min(0.002, off - now))
        if req.kind == "solve" and req.f is None:
            req.f = make_f(req)
            # the pools use their own (non-blocking) streams
            torch.cuda.current_stream().synchronize()
        req.t_arrival = time.perf_counter()
        server.submit(req)
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
                "pools_created": len(srv.pools) + srv.evictions, "evictions": srv.evictions}
        srv.shutdown()
        torch.cuda.empty_cache()
        print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
