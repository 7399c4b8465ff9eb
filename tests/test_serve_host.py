"""Host logic of the serving loop on the CPU: admission by HBM budget, LRU eviction of idle
pools, waiting requests admitted once a pool goes idle, every request completed exactly once.
The device pool is replaced by a stand-in that completes its requests from its own thread."""
import collections
import threading
import time

import pytest

torch = pytest.importorskip("torch")
serve = pytest.importorskip("paper_1003_2680_amd.serve")


class FakePool:
    created = []

    def __init__(self, server, dims):
        self.server = server
        self.dims = dims
        self.bytes = server.pool_bytes(dims)
        self.q = collections.deque()
        self.cv = threading.Condition()
        self.busy = 0
        self.last_used = time.perf_counter()
        self.stop = False
        self.t = threading.Thread(target=self._run, daemon=True)
        self.t.start()
        FakePool.created.append(dims)

    def idle(self):
        with self.cv:
            return not self.q and not self.busy

    def submit(self, req):
        with self.cv:
            self.q.append(req)
            self.cv.notify()

    def shutdown(self):
        with self.cv:
            self.stop = True
            self.cv.notify()
        self.t.join()

    def _run(self):
        while True:
            with self.cv:
                while not self.stop and not self.q:
                    self.cv.wait()
                if self.stop:
                    return
                req = self.q.popleft()
                self.busy = 1
            time.sleep(0.002)
            req.result = ("done", self.dims)
            with self.cv:
                self.busy = 0
            self.last_used = time.perf_counter()
            self.server._complete(req)


def test_admission_eviction_and_completion(monkeypatch):
    """Also: a submission never waits for planning or pool creation (the stand-in plan takes
    0.1 s per shape and runs on the admission thread)."""
    sizes = {(16, 16, 8): 100, (32, 32, 8): 200, (16, 16, 16): 300, (64, 64, 64): 10 ** 9}
    def slow_plan(dims, slots, prec):   # host planning that takes a while
        time.sleep(0.1)
        return sizes[dims]
    monkeypatch.setattr(serve, "pool_bytes", slow_plan)
    monkeypatch.setattr(serve, "Pool", FakePool)
    FakePool.created = []
    # any two of the three small pools fit the budget, never all three
    srv = serve.Server(budget_bytes=520, slots=4, stride=2, precision="fp32_refined",
                       device=torch.device("cuda", 0))
    shapes = [(16, 16, 8), (32, 32, 8), (16, 16, 16)]
    reqs = [serve.Request(i, shapes[i % 3], "sample", seed=i) for i in range(30)]
    reqs.append(serve.Request(30, (64, 64, 64), "solve", seed=1))   # larger than the budget
    t0 = time.perf_counter()
    for r in reqs:
        srv.submit(r)
    # submitting only queues: the admission thread plans and creates pools
    assert time.perf_counter() - t0 < 0.2
    assert srv.wait(len(reqs), timeout=20.0)
    srv.shutdown()
    assert len(srv.done) == len(reqs) and len({r.rid for r in srv.done}) == len(reqs)
    assert all(r.result == ("done", r.dims) for r in reqs[:30])
    assert reqs[30].error is not None
    assert srv.evictions >= 1
    assert max(sum(sizes[d] for d in srv.pools) for _ in [0]) <= 520


def test_paced_submissions_never_wait_for_planning(monkeypatch):
    """Requests submitted one by one while new shapes are being planned (0.1 s each, on the
    admission thread): no submission waits for the planning."""
    sizes = {(16, 16, 8): 100, (32, 32, 8): 100, (16, 16, 16): 100, (8, 8, 8): 100}
    def slow_plan(dims, slots, prec):
        time.sleep(0.1)
        return sizes[dims]
    monkeypatch.setattr(serve, "pool_bytes", slow_plan)
    monkeypatch.setattr(serve, "Pool", FakePool)
    srv = serve.Server(budget_bytes=10 ** 6, slots=4, stride=2, precision="fp32_refined",
                       device=torch.device("cuda", 0))
    shapes = list(sizes)
    reqs = [serve.Request(i, shapes[i % 4], "sample", seed=i) for i in range(24)]
    worst = 0.0
    for r in reqs:
        t = time.perf_counter()
        srv.submit(r)
        worst = max(worst, time.perf_counter() - t)
        time.sleep(0.01)
    assert srv.wait(len(reqs), timeout=20.0)
    srv.shutdown()
    assert worst < 0.05, worst
    assert len({r.rid for r in srv.done}) == len(reqs)
    assert all(r.result == ("done", r.dims) for r in reqs)


def test_unplannable_shape_fails_its_requests_only(monkeypatch):
    """A shape whose planning raises completes its requests with an error; the admission
    thread keeps serving the other shapes."""
    def plan(dims, slots, prec):
        if dims == (10, 10, 3):
            raise ValueError("unsupported grid")
        return 100
    monkeypatch.setattr(serve, "pool_bytes", plan)
    monkeypatch.setattr(serve, "Pool", FakePool)
    srv = serve.Server(budget_bytes=10 ** 6, slots=4, stride=2, precision="fp32_refined",
                       device=torch.device("cuda", 0))
    reqs = [serve.Request(i, (10, 10, 3) if i % 3 == 0 else (16, 16, 8), "sample", seed=i)
            for i in range(9)]
    for r in reqs:
        srv.submit(r)
    assert srv.wait(len(reqs), timeout=20.0)
    srv.shutdown()
    for r in reqs:
        if r.dims == (10, 10, 3):
            assert r.error is not None and "unsupported grid" in r.error
        else:
            assert r.error is None and r.result == ("done", r.dims)

