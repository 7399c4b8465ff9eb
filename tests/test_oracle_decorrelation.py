"""Pins for the oracle's exact lag correlation of a linear stochastic chain (CPU only).

The lag-k correlation of phi^T x for x' = T x + G n at stationarity is
phi^T T^k C phi / phi^T C phi (C the stationary covariance).  Pinned by cases that fix it
independently: no memory (T = 0), a scalar contraction (T = r I gives r^k), a diagonal chain
(the coordinate's own factor), and the empirical autocorrelation of a directly simulated
two-variable chain; then applied to the oracle's one-level Gauss-Seidel and multigrid cycles,
whose extracted linear parts and target covariance are pinned elsewhere.
"""
import numpy as np

from oracle.analysis import exact_lag_correlation, extract_linear_part
from oracle.mg import StochasticMG
from oracle.operator import assemble_A
from oracle import observables as ob


def test_no_memory_chain():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((5, 5))
    C = M @ M.T + 5 * np.eye(5)
    r = exact_lag_correlation(np.zeros((5, 5)), C, rng.standard_normal(5), 4)
    assert r[0] == 1.0 and np.all(r[1:] == 0.0)


def test_scalar_contraction():
    rng = np.random.default_rng(2)
    M = rng.standard_normal((4, 4))
    C = M @ M.T + np.eye(4)
    r = exact_lag_correlation(0.7 * np.eye(4), C, rng.standard_normal(4), 6)
    assert np.allclose(r, 0.7 ** np.arange(7), rtol=1e-13)


def test_diagonal_chain():
    t = np.array([0.1, -0.5, 0.9])
    C = np.diag([2.0, 1.0, 3.0])
    for j in range(3):
        r = exact_lag_correlation(np.diag(t), C, np.eye(3)[j], 5)
        assert np.allclose(r, t[j] ** np.arange(6), rtol=1e-13)


def test_matches_simulated_two_variable_chain():
    """x' = T x + L n with L L^T = C - T C T^T, simulated directly."""
    T = np.array([[0.6, 0.3], [-0.2, 0.5]])
    C = np.array([[2.0, 0.4], [0.4, 1.0]])
    J = C - T @ C @ T.T
    L = np.linalg.cholesky(J)
    rng = np.random.default_rng(3)
    n, burn = 400000, 100
    x = np.zeros(2)
    xs = np.empty((n, 2))
    noise = rng.standard_normal((n + burn, 2)) @ L.T
    for t in range(n + burn):
        x = T @ x + noise[t]
        if t >= burn:
            xs[t - burn] = x
    phi = np.array([1.0, -2.0])
    s = xs @ phi
    s = s - s.mean()
    emp = np.array([np.dot(s[:n - k], s[k:]) / np.dot(s, s) for k in range(5)])
    assert np.max(np.abs(emp - exact_lag_correlation(T, C, phi, 4))) < 0.01


def test_gauss_seidel_decorrelates_slower_than_multigrid():
    """8^3: the lowest mode's lag-1 correlation of the one-level Gauss-Seidel sampler is far
    above that of the V(2,2) multigrid cycle, which stays below the cycle's contraction."""
    dims = (8, 8, 8)
    C = np.linalg.inv(assemble_A(*dims).toarray())
    phi = ob.mode_vector(*dims, ob.lowest_modes(*dims, 1)[0])
    gs = exact_lag_correlation(extract_linear_part(StochasticMG(*dims, levels=1,
                                                                coarsest="smooth")), C, phi, 3)
    mg = exact_lag_correlation(extract_linear_part(StochasticMG(*dims, levels=2)), C, phi, 3)
    assert gs[1] > 0.3 and abs(mg[1]) < 0.1
    assert np.all(np.diff(gs) < 0)
