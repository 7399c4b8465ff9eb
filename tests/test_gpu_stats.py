"""GPU statistics of emitted samples (fused with emission) against the oracle.

* parity: eigenmode projections, energy 1/2 x^T A x and per-cell moments of the GPU chain
  against the oracle's observables of the oracle's chain on the same Philox streams
  (1e-12 relative; a projection's error is measured against the sample's norm);
* the emitted samples are the same bits as smg_sample_field's;
* distribution checks of the sampler itself through its observables: the mean energy is
  kT N / 2 and the mode variances are kT / lambda under N(0, kT A^-1), within Monte Carlo
  error of a correlated chain.
"""
import numpy as np
import pytest

from oracle.mg import StochasticMG
from oracle import observables as ob

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _hier(*args, **kw):
    from paper_1003_2680_amd.api import Hierarchy
    return Hierarchy(*args, **kw)


def _host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)


# rows of 64/128 cells (a wave per row, shared x factors), of 192 cells (a wave per row, x
# factors per cell) and of fewer than 64 cells
@pytest.mark.parametrize("dims,ncomp,levels,K,precision,cmax", [
    ((16, 16, 8), 2, 3, 8, "fp64", 64), ((12, 8, 6), 1, 2, 20, "fp64", 64),
    ((4, 4, 4), 2, 1, 5, "fp64", 64), ((64, 32, 16), 1, 4, 32, "fp64", 64),
    ((16, 16, 8), 2, 3, 3, "fp32_refined", 64), ((128, 8, 4), 1, 2, 0, "fp64", 64),
    ((128, 8, 4), 2, 2, 8, "fp64", 512), ((192, 8, 8), 1, 3, 8, "fp64", 512)])
def test_stats_parity(dims, ncomp, levels, K, precision, cmax):
    _announce("stats %s ncomp=%d L=%d K=%d %s" % (dims, ncomp, levels, K, precision))
    from paper_1003_2680_amd.api import lowest_modes
    nx, ny, nz = dims
    modes = lowest_modes(nx, ny, nz, K)
    assert modes == ob.lowest_modes(nx, ny, nz, K)
    n = 5
    kw = dict(ncomp=ncomp, kT=1.4, levels=levels, coarsest_max=cmax)
    H = _hier(*dims, precision=precision, **kw)
    out = torch.empty((n,) + H.shape, dtype=torch.float64, device="cuda")
    mom = torch.zeros((2,) + H.shape, dtype=torch.float64, device="cuda")
    obs, state = H.sample_stats(n, 17, modes=modes, out=out, moments=mom)
    got_obs, got_out, got_mom = _host(obs), _host(out), _host(mom)
    # emission is unchanged by the statistics
    ref_out, _ = _hier(*dims, precision=precision, **kw).sample(n, 17)
    assert np.array_equal(_host(ref_out), got_out)
    # observables of the emitted samples (the GPU samples themselves match the oracle chain to
    # 1e-12 in FP64 -- see the chain parity tests; here the statistics are checked)
    mg = StochasticMG(*dims, kT=1.4, levels=levels, coarsest_max=cmax)
    if precision == "fp64":
        ref, _ = mg.sample_chain(n, 17, ncomp=ncomp)
        assert np.max(np.abs(got_out.reshape(ref.shape) - ref)) <= 1e-12 * np.max(np.abs(ref))
    samples = got_out.reshape(n, ncomp, -1)
    for i in range(n):
        for c in range(ncomp):
            x = samples[i, c]
            want = ob.observables(x, nx, ny, nz, modes, h=1.0)
            nrm = np.linalg.norm(x)
            if K > 0:
                assert np.max(np.abs(got_obs[i, c, :K] - want[:K])) <= 1e-12 * nrm
            assert abs(got_obs[i, c, K] - want[K]) <= 1e-12 * want[K]
    m1, m2 = ob.moments(samples)
    assert np.max(np.abs(got_mom[0].reshape(ncomp, -1) - m1)) <= 1e-12 * np.max(np.abs(m1))
    assert np.max(np.abs(got_mom[1].reshape(ncomp, -1) - m2)) <= 1e-12 * np.max(np.abs(m2))


def test_stats_only_no_output_and_accumulation():
    _announce("stats accumulate")
    H = _hier(16, 16, 8, ncomp=1, levels=3)
    mom = torch.zeros((2,) + H.shape, dtype=torch.float64, device="cuda")
    o1, st = H.sample_stats(3, 5, moments=mom)
    o2, st = H.sample_stats(3, 5, first_cycle=3, state=st, moments=mom)
    out, _ = _hier(16, 16, 8, ncomp=1, levels=3).sample(6, 5)
    s = _host(out).reshape(6, -1)
    assert np.max(np.abs(_host(mom)[0].ravel() - s.sum(0))) <= 1e-12 * np.max(np.abs(s.sum(0)))
    ob_all = np.concatenate([_host(o1), _host(o2)])
    modes = ob.lowest_modes(16, 16, 8, 8)
    for i in range(6):
        want = ob.observables(s[i], 16, 16, 8, modes)
        assert np.max(np.abs(ob_all[i, 0] - want)) <= 1e-12 * max(np.linalg.norm(s[i]), want[-1])


def test_stats_invalid_modes():
    from paper_1003_2680_amd.abi import SMGError, SMG_EINVAL
    H = _hier(16, 16, 8, levels=3)
    for bad in ([(16, 0, 1)], [(0, 0, 0)], [(0, 0, 9)], [(0, 0, 1)] * 33):
        with pytest.raises(SMGError) as e:
            H.sample_stats(1, 0, modes=bad)
        assert e.value.code == SMG_EINVAL


def test_energy_and_mode_variance_match_target_law():
    """E[1/2 x^T A x] = kT N / 2 and E[<phi_q, x>^2] = kT / lambda_q for x ~ N(0, kT A^-1)."""
    _announce("energy / mode variance 16^3 x 4 comps, 600 samples")
    nx = ny = nz = 16
    kT = 2.0
    n, burn = 600, 10
    H = _hier(nx, ny, nz, ncomp=4, kT=kT, levels=3, burn_in=burn)
    modes = ob.lowest_modes(nx, ny, nz, 8)
    obs, _ = H.sample_stats(n, 123, modes=modes)
    o = _host(obs)  # [n, 4, 9]
    N = nx * ny * nz
    E = o[:, :, -1].ravel()
    # effective sample size from the measured autocorrelation (lag-1 ~ 0.08 for this cycle)
    se = np.sqrt(kT * kT * N / 2.0 / E.size * 3.0)
    assert abs(E.mean() - kT * N / 2.0) <= 5.0 * se, (E.mean(), kT * N / 2.0, se)
    lam = np.array([ob.mode_eigenvalue(nx, ny, nz, md) for md in modes])
    var = (o[:, :, :8] ** 2).reshape(-1, 8).mean(0)
    rel = var * lam / kT
    # relative standard error of a variance from ~2400 draws (correlation allowance x3)
    assert np.all(np.abs(rel - 1.0) <= 5.0 * np.sqrt(2.0 * 3.0 / (n * 4))), rel
