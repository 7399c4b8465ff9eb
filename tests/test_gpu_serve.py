"""Serving loop: continuous batching with HBM-budget admission.  Every request's result, in
the mix, equals the same request served alone (bit for bit); a budget that holds only two of
the three shapes' pools forces waiting and eviction; latency percentiles are reported."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SHAPES = [(16, 16, 8), (32, 32, 8), (16, 16, 16)]


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)


def test_serving_mix_equals_alone():
    from paper_1003_2680_amd.api import Hierarchy
    from paper_1003_2680_amd.inputs import gaussian_field_device
    from paper_1003_2680_amd.serve import Server, Request, pool_bytes, simulate
    _announce("serving mix")
    slots, stride, prec = 4, 2, "fp32_refined"
    sizes = sorted(pool_bytes(d, slots, prec) for d in SHAPES)
    budget = sizes[-1] + sizes[-2] + 4096        # room for two pools at a time
    srv = Server(budget_bytes=budget, slots=slots, stride=stride, precision=prec)
    rng = np.random.default_rng(3)
    timed = []
    t = 0.0
    for i in range(36):
        t += rng.exponential(1.0 / 2000.0)
        dims = SHAPES[int(rng.integers(0, 3))]
        kind = "sample" if rng.random() < 0.6 else "solve"
        timed.append((t, Request(i, dims, kind, seed=500 + i, k=int(rng.integers(1, 6)),
                                 rtol=1e-10)))

    def make_f(req):
        return gaussian_field_device(req.dims[::-1], req.seed, "cuda")

    ok, wall, lat = simulate(srv, timed, make_f, timeout=60.0)
    srv.shutdown()
    assert ok, "requests did not complete: %d of 36" % len(srv.done)
    print("  wall %.3f s, p50 %.2f ms, p99 %.2f ms, evictions %d"
          % (wall, np.percentile(lat, 50) * 1e3, np.percentile(lat, 99) * 1e3, srv.evictions),
          flush=True)
    assert len(srv.done) == 36 and all(r.error is None for r in srv.done)
    assert srv.evictions >= 1
    alone = {}
    for _, r in timed:
        key = (r.dims, r.kind)
        if key not in alone:
            if r.kind == "sample":
                alone[key] = Hierarchy(*r.dims, ncomp=1, stride=stride, burn_in=stride,
                                       precision=prec)
            else:
                alone[key] = Hierarchy(*r.dims, ncomp=1, precision=prec)
        H = alone[key]
        if r.kind == "sample":
            ref, _ = H.sample(r.k, r.seed, out_dtype=torch.float32)
            assert torch.equal(r.result, ref[:, 0]), r.rid
        else:
            u, cyc, rel = H.solve(r.f[None].contiguous(), rtol=r.rtol)
            assert torch.equal(r.result, u[0]) and r.info[0] == cyc, r.rid
