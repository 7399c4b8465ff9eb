"""Host logic of the serving loop on the CPU: admission by HBM budget, LRU eviction of idle
pools, waiting requests admitted once a pool goes idle, every request completed exactly once.
The device pool is replaced by a stand-in that completes its requests from its own thread."""
import collections
import threading
import time

import pytest

serve = pytest.importorskip("paper_1003_2680_amd.serve")


class FakePool:
    created = []

    def __init__(self, server, dims):
        self.server = server
        self.dims = dims
        self.bytes = serve.pool_bytes(dims, server.slots, server.precision)
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
    sizes = {(16, 16, 8): 100, (32, 32, 8): 200, (16, 16, 16): 300, (64, 64, 64): 10 ** 9}
    monkeypatch.setattr(serve, "pool_bytes", lambda dims, slots, prec: sizes[dims])
    monkeypatch.setattr(serve, "Pool", FakePool)
    FakePool.created = []
    srv = serve.Server.__new__(serve.Server)
    srv.device = None
    srv.budget = 520          # any two of the three small pools, never all three
    srv.slots, srv.stride, srv.precision, srv.kT = 4, 2, "fp32_refined", 1.0
    srv.pools = collections.OrderedDict()
    srv.waiting = collections.deque()
    srv.lock = threading.Lock()
    srv.done = []
    srv.done_cv = threading.Condition()
    srv.evictions = 0
    shapes = [(16, 16, 8), (32, 32, 8), (16, 16, 16)]
    reqs = [serve.Request(i, shapes[i % 3], "sample", seed=i) for i in range(30)]
    reqs.append(serve.Request(30, (64, 64, 64), "solve", seed=1))   # larger than the budget
    for r in reqs:
        srv.submit(r)
    assert srv.wait(len(reqs), timeout=20.0)
    srv.shutdown()
    assert len(srv.done) == len(reqs) and len({r.rid for r in srv.done}) == len(reqs)
    assert all(r.result == ("done", r.dims) for r in reqs[:30])
    assert reqs[30].error is not None
    assert srv.evictions >= 1
    assert max(sum(sizes[d] for d in srv.pools) for _ in [0]) <= 520
