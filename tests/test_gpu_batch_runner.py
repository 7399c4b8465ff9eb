"""Uneven-instance batch runner and autotuner: every instance's result in the mix equals the
same instance run alone with the same configuration (bit for bit), for samples, solves and
graph replays; the tuner returns a configuration that runs."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CFG = {"levels": 0, "nu1": 2, "nu2": 2}


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)


def _instances():
    from paper_1003_2680_amd.batch import Instance
    dims = [(16, 16, 16), (32, 32, 16), (16, 16, 16), (16, 16, 8), (32, 32, 16), (16, 16, 16)]
    return [Instance(d, seed=100 + i, first_cycle=3 * i) for i, d in enumerate(dims)]


def _alone(inst, precision, cfg, n):
    from paper_1003_2680_amd.api import Hierarchy
    H = Hierarchy(*inst.dims, ncomp=1, levels=cfg["levels"], nu1=cfg["nu1"], nu2=cfg["nu2"],
                  precision=precision)
    return H, H.sample(n, inst.seed, first_cycle=inst.first_cycle, out_dtype=torch.float32)[0]


@pytest.mark.parametrize("engine", ["library", "streams"])
@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_runner_samples_and_solves_equal_alone(precision, engine):
    from paper_1003_2680_amd.batch import BatchRunner
    from paper_1003_2680_amd.inputs import gaussian_field
    _announce("batch runner %s %s" % (precision, engine))
    insts = _instances()
    R = BatchRunner(insts, precision=precision, configs={i.dims: CFG for i in insts},
                    engine=engine)
    assert len(R.groups) == 3
    outs = R.sample(3)
    torch.cuda.synchronize()
    for i, inst in enumerate(insts):
        _, ref = _alone(inst, precision, CFG, 3)
        assert torch.equal(outs[i], ref[:, 0]), i
    fs = {i: torch.from_numpy(gaussian_field(inst.dims[::-1], 50 + i)).cuda()
          for i, inst in enumerate(insts)}
    us, infos = R.solve(fs, rtol=1e-10)
    from paper_1003_2680_amd.api import Hierarchy
    for i, inst in enumerate(insts):
        H = Hierarchy(*inst.dims, ncomp=1, precision=precision)
        u, cyc, rel = H.solve(fs[i][None].contiguous(), rtol=1e-10)
        assert torch.equal(us[i], u[0]) and infos[i][0] == cyc, i


@pytest.mark.parametrize("groups", [1, 2])
def test_runner_graph_replay_continues_chains(groups):
    """The replayed graph (captured in the one-stream form whatever the runner's stream
    groups) continues the chains as eager one-stream calls, and eager calls in stream groups
    after the replays continue them the same way."""
    from paper_1003_2680_amd.batch import BatchRunner
    _announce("batch runner graph replay, %d stream group(s)" % groups)
    insts = _instances()
    eager = BatchRunner(insts, precision="fp32_refined", configs={i.dims: CFG for i in insts})
    graph = BatchRunner(insts, precision="fp32_refined", configs={i.dims: CFG for i in insts},
                        stream_groups=groups)
    eager.start()
    graph.start()
    graph.capture(2)
    for k in range(3):
        eager.sample(2, emit=False)
        graph.replay()
        torch.cuda.synchronize()
        for ge, gg in zip(eager.groups, graph.groups):
            assert torch.equal(ge.state, gg.state), (k, ge.dims)
        torch.randn(100, device="cuda").sum().item()   # eager work between replays
    # and the chains continue after the replays exactly as the eager ones do
    a = eager.sample(1)
    b = graph.sample(1)
    for i in a:
        assert torch.equal(a[i], b[i])


def test_autotune_small_grid():
    from paper_1003_2680_amd import autotune
    from paper_1003_2680_amd.batch import BatchRunner, Instance
    _announce("autotune 16^3 x 2")
    cfg = autotune.tune((16, 16, 16), 2, precision="fp32_refined", cycles=2)
    assert cfg["levels"] >= 2 and (cfg["nu1"], cfg["nu2"]) in autotune.NU_CANDIDATES
    assert 0.0 < cfg["rho"] < 0.5 and cfg["k_dec"] >= 1 and cfg["t_cycle"] > 0
    assert len(cfg["table"]) >= len(autotune.NU_CANDIDATES)
    insts = [Instance((16, 16, 16), seed=s) for s in (1, 2)]
    R = BatchRunner(insts, precision="fp32_refined", configs={(16, 16, 16): cfg})
    out = R.sample(2)
    for i, inst in enumerate(insts):
        H, ref = _alone(inst, "fp32_refined", cfg, 2)
        assert torch.equal(out[i], ref[:, 0])
