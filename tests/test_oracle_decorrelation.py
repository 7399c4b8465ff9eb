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


def test_autocorrelation_hand_computed_series():
    """s = (1, 2, 3, 4): deviations (-1.5, -0.5, 0.5, 1.5), lag-0 sum 5/4 with the 1/n
    weight; lag-1 sum (0.75 - 0.25 + 0.75)/4, lag-2 (-0.75 - 0.75)/4, lag-3 -2.25/4, so the
    normalised values are 1, 1/4, -3/10, -9/20 (dividing by n - k instead, or skipping the
    mean, gives other numbers)."""
    from oracle.analysis import autocorrelation
    r = autocorrelation([1.0, 2.0, 3.0, 4.0], 3)
    assert np.allclose(r, [1.0, 0.25, -0.3, -0.45], rtol=0, atol=1e-15)
    # a shifted and scaled copy has the same correlations; a constant offset is removed
    assert np.allclose(autocorrelation([7.0, 9.0, 11.0, 13.0], 3), r, rtol=0, atol=1e-15)
    # alternating series: lag-k correlation (-1)^k (n - k)/n
    alt = np.array([1.0, -1.0] * 5)
    ra = autocorrelation(alt, 4)
    assert np.allclose(ra, [(-1) ** k * (10 - k) / 10 for k in range(5)], rtol=0, atol=1e-15)


def test_autocorrelation_of_simulated_ar1_matches_exact():
    """x' = a x + sqrt(1 - a^2) n, simulated directly: the estimator's lag-k values match the
    exact a^k (exact_lag_correlation of the scalar chain) within four Bartlett standard
    deviations sqrt((1 + a^2)(1 - a^(2k)) / (1 - a^2) - 2k a^(2k)) / sqrt(n)."""
    from oracle.analysis import autocorrelation
    a, n = 0.8, 200000
    rng = np.random.default_rng(11)
    e = rng.standard_normal(n) * np.sqrt(1 - a * a)
    x = np.empty(n)
    v = rng.standard_normal()
    for t in range(n):
        v = a * v + e[t]
        x[t] = v
    est = autocorrelation(x, 6)
    exact = exact_lag_correlation(np.array([[a]]), np.array([[1.0]]), np.array([1.0]), 6)
    assert np.allclose(exact, a ** np.arange(7), rtol=1e-14)
    for k in range(1, 7):
        var = ((1 + a * a) * (1 - a ** (2 * k)) / (1 - a * a) - 2 * k * a ** (2 * k)) / n
        assert abs(est[k] - exact[k]) < 4 * np.sqrt(var), (k, est[k], exact[k])
