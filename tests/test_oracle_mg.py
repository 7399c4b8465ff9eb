"""Pins for the oracle's stochastic multigrid cycle and solve (CPU only).

* Heat-bath conditionals: a colour pass with injected noise reproduces the conditional
  mean and standard deviation of the target Gaussian, computed here by Gaussian
  conditioning on the dense covariance kT A^-1 (not from the precision shortcut the
  smoother uses).
* Exact invariance: the stationary covariance of the extracted affine map of one full
  stochastic V-cycle (solution of C = T C T^T + G G^T) equals kT A^-1 (eq. J_eq_C_R).
* Uniqueness and rate: spectral radius of T below 0.1 and grid independent.
* Special cases: the one-level Cholesky cycle is an exact independent draw; the one-level
  smoothing-only cycle is the textbook stochastic Gauss-Seidel sampler (also invariant).
* Solve: the noise-free cycle converges to the direct solution.
* Law: chain covariance against dense kT A^-1 within Monte Carlo error.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.operator import assemble_A
from oracle.mg import StochasticMG
from oracle.analysis import (extract_affine_map, stationary_covariance, _InjectedNoise,
                             autocorrelation)
from oracle import spectral


def _conditional(Sigma, mu, x, idx):
    """Mean and covariance of x[idx] given the other entries under N(mu, Sigma)."""
    n = Sigma.shape[0]
    rest = np.setdiff1d(np.arange(n), idx)
    S_ir = Sigma[np.ix_(idx, rest)]
    S_rr = Sigma[np.ix_(rest, rest)]
    K = S_ir @ np.linalg.inv(S_rr)
    mean = mu[idx] + K @ (x[rest] - mu[rest])
    cov = Sigma[np.ix_(idx, idx)] - K @ S_ir.T
    return mean, cov


class _Const:
    def __init__(self, value):
        self.value = value

    def draw(self, cycle, level, slot, colour, comp, kind, sites):
        return np.full(len(sites), self.value)


def test_point_heat_bath_conditional():
    nx, ny, nz, kT = 4, 4, 3, 1.7
    mg = StochasticMG(nx, ny, nz, kT=kT, levels=1, coarsest="smooth")
    L = mg.levels[0]
    A = L.A.toarray()
    Sigma = kT * np.linalg.inv(A)
    rng = np.random.default_rng(1)
    b = rng.standard_normal(L.n)
    mu = np.linalg.solve(A, b)
    x0 = rng.standard_normal(L.n)
    for colour in range(2):
        x = x0.copy()
        mg._point_pass(L, x, b, colour, _Const(0.8), (0, 0, 0))
        for i in L.sets[colour][:7]:
            # conditional of one site given all others
            m, c = _conditional(Sigma, mu, x0, np.array([i]))
            assert x[i] == pytest.approx(m[0] + 0.8 * np.sqrt(c[0, 0]), rel=1e-12, abs=1e-12)
        others = L.sets[1 - colour]
        assert np.array_equal(x[others], x0[others])


def test_block_heat_bath_conditional():
    kT = 0.6
    mg = StochasticMG(8, 8, 4, kT=kT, levels=3)
    L = mg.levels[1]
    assert L.kind == "block" and L.dims == (4, 4, 2)
    A = L.A.toarray()
    Sigma = kT * np.linalg.inv(A)
    rng = np.random.default_rng(2)
    b = rng.standard_normal(L.n)
    mu = np.linalg.solve(A, b)
    x0 = rng.standard_normal(L.n)
    for colour in (0, 5):
        x = x0.copy()
        n = rng.standard_normal(8 * len(L.blocks[colour]["bid"]))
        mg._block_pass(L, x, b, colour, _InjectedNoise(n), (0, 0, 0))
        cells = L.blocks[colour]["cells"]
        for k, blk in enumerate(cells):
            m, c = _conditional(Sigma, mu, x0, blk)
            # any factor F with F F^T = c maps n to the right covariance; the oracle uses
            # sqrt(kT) L^-T with A_BB = L L^T, i.e. F = chol(c) ... up to an orthogonal
            # factor, so check the mean with zero noise and the covariance separately
            xb = x0.copy()
            mg._block_pass(L, xb, b, colour, _Const(0.0), (0, 0, 0))
            assert np.allclose(xb[blk], m, rtol=1e-11, atol=1e-11)
            ABB = L.blocks[colour]["ABB"][k]
            F = np.sqrt(kT) * np.linalg.inv(np.linalg.cholesky(ABB).T)
            assert np.allclose(F @ F.T, c, rtol=1e-10, atol=1e-12)
            assert np.allclose(x[blk], m + F @ n[8 * k:8 * k + 8], rtol=1e-10, atol=1e-11)


@pytest.mark.parametrize("dims,levels", [((8, 8, 8), 3), ((8, 8, 16), 3), ((8, 8, 8), 2)])
def test_cycle_preserves_target_law_exactly(dims, levels):
    kT = 1.3
    mg = StochasticMG(*dims, kT=kT, levels=levels)
    T, G = extract_affine_map(mg)
    C = stationary_covariance(T, G @ G.T)
    Ct = kT * np.linalg.inv(assemble_A(*dims).toarray())
    assert np.max(np.abs(C - Ct)) / np.max(np.abs(Ct)) < 1e-12
    rho = np.max(np.abs(np.linalg.eigvals(T)))
    assert rho < 0.1


def test_single_level_cholesky_is_exact_draw():
    kT = 2.0
    mg = StochasticMG(4, 4, 4, kT=kT, levels=1)
    T, G = extract_affine_map(mg)
    assert np.max(np.abs(T)) == 0.0
    Ct = kT * np.linalg.inv(assemble_A(4, 4, 4).toarray())
    assert np.allclose(G @ G.T, Ct, rtol=1e-12, atol=1e-14)


def test_single_level_gauss_seidel_sampler_is_invariant():
    mg = StochasticMG(4, 4, 4, levels=1, coarsest="smooth")
    T, G = extract_affine_map(mg)
    C = stationary_covariance(T, G @ G.T)
    Ct = np.linalg.inv(assemble_A(4, 4, 4).toarray())
    assert np.max(np.abs(C - Ct)) / np.max(np.abs(Ct)) < 1e-10
    # plain Gauss-Seidel converges far more slowly than the multigrid cycle
    assert np.max(np.abs(np.linalg.eigvals(T))) > 0.3


def _power_rho(mg, iters=30, seed=0):
    N = mg.levels[0].n
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(N)
    zero = np.zeros(N)
    A = mg.levels[0].A
    rates = []
    for _ in range(iters):
        nrm0 = np.sqrt(e @ (A @ e))
        e = mg.vcycle(e, zero, None)
        nrm1 = np.sqrt(e @ (A @ e))
        rates.append(nrm1 / nrm0)
        e /= nrm1
    return rates[-1]


def test_contraction_grid_independent():
    rhos = [_power_rho(StochasticMG(n, n, n, levels=0, coarsest_max=64)) for n in (8, 16, 32)]
    assert max(rhos) < 0.1
    assert max(rhos) - min(rhos) < 0.03


def test_solve_matches_direct():
    nx = ny = nz = 16
    mg = StochasticMG(nx, ny, nz, levels=3)
    rng = np.random.default_rng(1)
    f = rng.standard_normal(nx * ny * nz)
    u, cycles, relres = mg.solve(f, rtol=1e-12)
    assert relres <= 1e-12 and cycles < 20
    u_dir = spla.spsolve(assemble_A(nx, ny, nz).tocsc(), f)
    assert np.max(np.abs(u - u_dir)) <= 1e-10 * np.max(np.abs(u_dir))
    assert np.max(np.abs(u - spectral.solve(f, nx, ny, nz))) <= 1e-10 * np.max(np.abs(u_dir))


def test_kT_scaling():
    a, _ = StochasticMG(8, 8, 8, kT=1.0, levels=3).sample_chain(3, seed=5)
    b, _ = StochasticMG(8, 8, 8, kT=4.0, levels=3).sample_chain(3, seed=5)
    assert np.allclose(b, 2.0 * a, rtol=1e-12, atol=1e-13)


def test_chain_resume_is_bitwise():
    mg = StochasticMG(8, 8, 8, levels=3)
    full, _ = mg.sample_chain(6, seed=9)
    part1, state = mg.sample_chain(3, seed=9)
    part2, _ = mg.sample_chain(3, seed=9, first_cycle=3, x0=state)
    assert np.array_equal(full, np.concatenate([part1, part2]))


@pytest.mark.slow
def test_chain_covariance_against_cholesky():
    kT = 1.0
    mg = StochasticMG(8, 8, 8, kT=kT, levels=3)
    n = 3000
    samples, _ = mg.sample_chain(n, seed=0, burn_in=5)
    X = samples[:, 0, :]
    Ct = kT * np.linalg.inv(assemble_A(8, 8, 8).toarray())
    Cs = X.T @ X / n
    # effective sample size from the slowest mode's autocorrelation
    v = spectral.z_mode(1, 8)
    mode = np.kron(v, np.full(64, 1 / 8.0))
    rho1 = autocorrelation(X @ mode, 3)[1]
    n_eff = n * (1 - abs(rho1)) / (1 + abs(rho1))
    rng = np.random.default_rng(4)
    idx = [(i, i) for i in range(0, 512, 37)] + [tuple(rng.integers(0, 512, 2)) for _ in range(20)]
    for i, j in idx:
        se = np.sqrt((Ct[i, i] * Ct[j, j] + Ct[i, j] ** 2) / n_eff)
        assert abs(Cs[i, j] - Ct[i, j]) < 5 * se, (i, j)
    # every mode variance: sum over modes of (amplitude^2 lambda/kT) averages to one
    amps = np.array([spectral.mode_amplitudes(x, 8, 8, 8) for x in X[::10]])
    lam = spectral.eigenvalues(8, 8, 8)
    ratio = (np.abs(amps) ** 2 * lam / kT).mean()
    assert abs(ratio - 1.0) < 0.02
