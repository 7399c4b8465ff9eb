"""Batched chains: many independent chains of one grid in the same launches.

Every chain of a batch must give, bit for bit, what the same chain gives alone (same seed,
same first cycle, same parameters), in FP64 and FP32-refined mode, for samples, statistics and
solves; a graph-captured batched call, replayed, must continue the chains exactly like eager
calls do.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SEEDS = [5, 77, 2 ** 40 + 3]
FIRST = [0, 10, 2 ** 33 + 1]


def _hier(*args, **kw):
    from paper_1003_2680_amd.api import Hierarchy
    return Hierarchy(*args, **kw)


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)


@pytest.mark.parametrize("dims,levels,precision,extra", [
    ((16, 16, 8), 3, "fp64", {}), ((16, 16, 8), 3, "fp32_refined", {}),
    ((32, 16, 16), 4, "fp64", {"stride": 2, "burn_in": 1}), ((4, 4, 4), 1, "fp64", {}),
    ((32, 32, 16), 4, "fp64", {"coarsest": "smooth"})])
def test_batch_samples_equal_alone(dims, levels, precision, extra):
    _announce("batch samples %s L=%d %s %s" % (dims, levels, precision, extra))
    cpc, n = 2, 3
    kw = dict(levels=levels, precision=precision, kT=1.3, **extra)
    # 8 components, 6 of them used: the idle tail must not disturb anything
    HB = _hier(*dims, ncomp=8, **kw)
    out, _, state = HB.sample_batch(n, seeds=SEEDS, first_cycles=FIRST, comps_per_chain=cpc)
    torch.cuda.synchronize()
    for c, (sd, fc) in enumerate(zip(SEEDS, FIRST)):
        H = _hier(*dims, ncomp=cpc, **kw)
        o, st = H.sample(n, sd, first_cycle=fc)
        assert torch.equal(o, out[:, c * cpc:(c + 1) * cpc]), "chain %d" % c
        assert torch.equal(st, state[c * cpc:(c + 1) * cpc])


def test_batch_continues_and_stats():
    _announce("batch continuation + stats")
    dims = (16, 16, 16)
    HB = _hier(*dims, ncomp=3, levels=3)
    o1, b1, st = HB.sample_batch(2, seeds=SEEDS, first_cycles=FIRST, comps_per_chain=1,
                                 with_obs=True)
    o2, b2, st = HB.sample_batch(2, nchains=3, comps_per_chain=1, state=st, with_obs=True)
    obs = torch.cat([b1, b2])
    for c, (sd, fc) in enumerate(zip(SEEDS, FIRST)):
        H = _hier(*dims, ncomp=1, levels=3)
        ob, _ = H.sample_stats(4, sd, first_cycle=fc)
        assert torch.equal(ob[:, 0], obs[:, c])


@pytest.mark.parametrize("precision", ["fp64", "fp32_refined"])
def test_batch_solve_equals_alone(precision):
    from paper_1003_2680_amd.inputs import gaussian_field
    _announce("batch solve %s" % precision)
    dims = (32, 32, 16)
    cpc = 2
    f = gaussian_field((3 * cpc, dims[2], dims[1], dims[0]), 4)
    f[2:4] *= 1e-3   # a chain with a smaller right-hand side
    f[4:6] = 0.0     # a chain with f = 0
    fd = torch.from_numpy(f).cuda()
    # two idle components, and a sampling call first so the workspace holds old values
    HB = _hier(*dims, ncomp=3 * cpc + 2, levels=4, precision=precision)
    HB.sample(2, 9)
    u, infos = HB.solve_batch(fd, nchains=3, comps_per_chain=cpc, rtol=1e-11)
    for c in range(3):
        H = _hier(*dims, ncomp=cpc, levels=4, precision=precision)
        uc, cyc, rel = H.solve(fd[c * cpc:(c + 1) * cpc].contiguous(), rtol=1e-11)
        assert torch.equal(uc, u[c * cpc:(c + 1) * cpc]), c
        assert infos[c][0] == cyc and infos[c][1] == rel and infos[c][2] == H.last_ratio
    assert infos[2][0] == 0 and float(u[4:6].abs().max()) == 0.0


@pytest.mark.parametrize("groups", [1, 2])
def test_batch_graph_replay_continues_chains(groups):
    """A captured batched call replayed K times equals K eager one-stream calls (trap check:
    every replay compared, with eager work and synchronisation between replays); with two
    stream groups the side streams join the capture through the fork event."""
    _announce("batch graph replay, %d stream group(s)" % groups)
    dims = (16, 16, 8)
    n = 2
    HE = _hier(*dims, ncomp=3, levels=3)
    a0, _, se = HE.sample_batch(n, seeds=SEEDS, first_cycles=FIRST, comps_per_chain=1)
    ref = []
    for _ in range(3):
        o, _, se = HE.sample_batch(n, nchains=3, comps_per_chain=1, state=se)
        ref.append(o.clone())
    HG = _hier(*dims, ncomp=3, levels=3)
    HG.set_stream_groups(groups)
    b0, _, sg = HG.sample_batch(n, seeds=SEEDS, first_cycles=FIRST, comps_per_chain=1)
    assert torch.equal(a0, b0)
    out = torch.empty_like(ref[0])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        HG.sample_batch(n, nchains=3, comps_per_chain=1, state=sg, out=out)
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref[k]), "replay %d" % k
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        del junk


def test_batch_errors():
    from paper_1003_2680_amd.abi import SMGError, SMG_EINVAL, SMG_ESTATE
    H = _hier(16, 16, 8, ncomp=4, levels=3)
    with pytest.raises(ValueError):
        H.sample_batch(1, seeds=[1, 2, 3], comps_per_chain=2)
    with pytest.raises(SMGError) as e:
        H.sample_batch(1, nchains=2, comps_per_chain=2)   # no table written yet
    assert e.value.code == SMG_ESTATE
    H.sample_batch(1, seeds=[1, 2], comps_per_chain=2)
    with pytest.raises(SMGError) as e:
        H.sample_batch(1, nchains=4, comps_per_chain=1)   # table of another shape
    assert e.value.code == SMG_ESTATE
    assert SMG_EINVAL == -1
    # caller outputs are checked before the library writes into them: their dtype decides the
    # element type written, and a wrong shape, dtype or layout is refused
    fshape = (4, 8, 16, 16)
    for bad in (torch.empty((2,) + fshape, dtype=torch.float64, device="cuda"),
                torch.empty((1, 2, 8, 16, 16), dtype=torch.float64, device="cuda"),
                torch.empty((1,) + fshape, dtype=torch.float16, device="cuda"),
                torch.empty((1, 4, 16, 16, 8), dtype=torch.float64, device="cuda")
                .transpose(2, 4)):
        with pytest.raises(ValueError):
            H.sample_batch(1, nchains=2, comps_per_chain=2, out=bad)
    with pytest.raises(ValueError):
        H.sample_batch(1, nchains=2, comps_per_chain=2,
                       moments=torch.zeros((2, 2, 8, 16, 16), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        H.sample(1, 3, out=torch.empty((1,) + fshape, dtype=torch.float32, device="cuda")[:, :2])
    o32 = torch.empty((1,) + fshape, dtype=torch.float32, device="cuda")
    H.sample_batch(1, nchains=2, comps_per_chain=2, out=o32)  # float32 written as float32
    o64, _, _ = H.sample_batch(1, seeds=[1, 2], comps_per_chain=2)
    st = torch.zeros(fshape, dtype=torch.float64, device="cuda")
    H.sample_batch(0, seeds=[1, 2], comps_per_chain=2, state=st)
    o32 = torch.empty((1,) + fshape, dtype=torch.float32, device="cuda")
    H.sample_batch(1, nchains=2, comps_per_chain=2, state=st, out=o32)
    torch.cuda.synchronize()
    assert torch.equal(o32, o64.float())


def test_batch_solve_one_level_cholesky_chains_finish_apart():
    """One-level hierarchy (level 0 drawn exactly by the dense Cholesky factor): a chain that
    reaches rtol a cycle before the others keeps its exported solution.  rtol is set between
    the two chains' relative residuals after one cycle (read from solves alone), so one chain
    stops after cycle 1 while the other runs on; the stopped chain's u must equal its solve
    alone bit for bit (the residual passes of later cycles go to the library's own buffer)."""
    from paper_1003_2680_amd.inputs import gaussian_field
    _announce("batch solve one-level cholesky, chains finishing apart")
    dims = (8, 8, 8)
    f = gaussian_field((2, dims[2], dims[1], dims[0]), 21)
    f[1] += 50.0 * np.cos(np.arange(8) * np.pi / 4.0)[None, None, :]  # another residual floor
    fd = torch.from_numpy(f).cuda()
    rel = []
    for c in range(2):
        H = _hier(*dims, ncomp=1, levels=1)
        _, _, r1 = H.solve(fd[c:c + 1].contiguous(), rtol=0.0, max_cycles=1,
                           raise_on_notconv=False)
        rel.append(r1)
    if rel[0] == rel[1]:
        pytest.skip("equal one-cycle residuals; no rtol separates the chains")
    lo = int(np.argmin(rel))
    rtol = float(np.sqrt(rel[0] * rel[1]))
    HB = _hier(*dims, ncomp=2, levels=1)
    u, infos = HB.solve_batch(fd, nchains=2, comps_per_chain=1, rtol=rtol, max_cycles=3,
                              raise_on_notconv=False)
    assert infos[lo][0] == 1
    H = _hier(*dims, ncomp=1, levels=1)
    ul, cyc, _ = H.solve(fd[lo:lo + 1].contiguous(), rtol=rtol, max_cycles=1)
    assert cyc == 1 and torch.equal(ul, u[lo:lo + 1]), "stopped chain's solution overwritten"
    assert float(ul.abs().max()) > 1e-3  # a solution, not a residual of roundoff size
