"""GPU parity of the 2D wall-bounded sampler (C-ABI smg2d_*) against the 2D oracle.

* Chains: three stochastic cycles from the zero start, two components, on identical Philox
  streams, every value within 1e-12 relative to the largest (FP64): multigrid hierarchies with
  two to five levels (exact coarsest draw), a smoothing-only coarsest level, the one-level
  Gauss-Seidel sampler and a one-level exact draw; nz odd and non-power-of-two extents.
* Solve: against the oracle's sparse direct solve (1e-9 relative) within a grid-independent
  number of cycles.
* Decorrelation: the GPU chains' lag-1..4 correlations of the three lowest modes match the
  oracle's exact phi^T T^k C phi / phi^T C phi within five Bartlett standard deviations, for the
  multigrid and the Gauss-Seidel chain.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import mg2d
from oracle.analysis import exact_lag_correlation, extract_linear_part
from oracle.philox import PhiloxNoise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    ((16, 8), dict(levels=3)),
    ((32, 16), dict(levels=0, coarsest_max=64)),
    ((24, 12), dict(levels=2)),
    ((64, 32), dict(levels=5)),
    ((16, 16), dict(levels=3, coarsest="smooth")),
    ((8, 8), dict(levels=1, coarsest="smooth")),
    ((6, 5), dict(levels=1)),
    ((40, 10), dict(levels=2)),
]


def _announce(msg):
    print("[gpu-case] " + msg, flush=True)


@pytest.mark.parametrize("dims,kw", CASES)
def test_chain_against_oracle(dims, kw):
    from paper_1003_2680_amd.grid2d import Hierarchy2D
    _announce("2D chain %s %s" % (dims, kw))
    nx, nz = dims
    H = Hierarchy2D(nx, nz, ncomp=2, kT=1.3, **kw)
    mg = mg2d.StochasticMG2D(nx, nz, kT=1.3, **kw)
    assert H.level_dims == [L.dims for L in mg.levels]
    out, _ = H.sample(3, 77, first_cycle=4)
    got = out.cpu().numpy().reshape(3, 2, -1)
    zero = np.zeros(nx * nz)
    for c in range(2):
        x = zero.copy()
        for k in range(3):
            x = mg.vcycle(x, zero, PhiloxNoise(77), 4 + k, c)
            err = np.max(np.abs(got[k, c] - x)) / np.max(np.abs(x))
            assert err <= 1e-12, (dims, kw, c, k, err)


@pytest.mark.parametrize("dims", [(32, 16), (128, 64)])
def test_solve_against_direct(dims):
    from paper_1003_2680_amd.grid2d import Hierarchy2D
    from paper_1003_2680_amd.inputs import gaussian_field
    _announce("2D solve %s" % (dims,))
    nx, nz = dims
    H = Hierarchy2D(nx, nz, ncomp=1, levels=0, coarsest_max=64)
    f = gaussian_field((1, nz, nx), 9)
    u, cycles, relres = H.solve(torch.from_numpy(f).cuda(), rtol=1e-11)
    ref = spla.spsolve(mg2d.assemble_A2(nx, nz).tocsc(), f.ravel())
    err = np.max(np.abs(u.cpu().numpy().ravel() - ref)) / np.max(np.abs(ref))
    assert relres <= 1e-11 and cycles <= 14 and err <= 1e-9, (cycles, relres, err)


def _bartlett_sd(rho, k, n):
    M = rho.size - k - 1
    r = lambda m: rho[abs(m)] if abs(m) < rho.size else 0.0
    s = sum(r(m) ** 2 + r(m + k) * r(m - k) - 4 * r(k) * r(m) * r(m - k)
            + 2 * r(m) ** 2 * r(k) ** 2 for m in range(-M, M + 1))
    return np.sqrt(max(s, 0.0) / n)


@pytest.mark.parametrize("kind,n,burn", [("gs", 20000, 600), ("mg", 20000, 20)])
def test_lag_correlations_match_exact(kind, n, burn):
    from paper_1003_2680_amd.decorrelation import autocorrelation, make_chain_2d, projections_2d
    dims = (16, 16)
    _announce("2D decorrelation %s n=%d" % (kind, n))
    H = make_chain_2d(dims, kind, nchains=8)
    modes = [(0, 1), (1, 1), (2, 1)]
    _, st = H.sample(burn, 5)
    xs, _ = H.sample(n, 5, first_cycle=burn, state=st)
    obs = projections_2d(xs, dims, modes).cpu().numpy()
    est = autocorrelation(obs, 4)
    if kind == "gs":
        mg = mg2d.StochasticMG2D(*dims, levels=1, coarsest="smooth")
    else:
        mg = mg2d.StochasticMG2D(*dims, levels=0)
    T = extract_linear_part(mg)
    C = np.linalg.inv(mg2d.assemble_A2(*dims).toarray())
    for q, (a, m) in enumerate(modes):
        phi = mg2d.mode_vector_2d(*dims, a, m)
        exact = exact_lag_correlation(T, C, phi, 400)
        for k in range(1, 5):
            sd = _bartlett_sd(exact, k, n * 8)
            assert abs(est[k, q] - exact[k]) <= 5 * sd + 2e-3, (kind, a, m, k, est[k, q],
                                                               exact[k], sd)
