"""Pins of the effective-dynamics oracle for a non-symmetric Laplacian (Appendix A), on the CPU.

* Numerical validation of the appendix's asymptotics.  The exact mean and covariance of
  Gamma * integral_0^dt u, for the stationary linear SDE of the fluid, are computed by quadrature
  of matrix exponentials (scipy's expm on Gauss-Legendre nodes).  This is independent of the
  closed forms.  Per unit time they approach a = -eps Gamma L^-1 f and
  b = -eps Gamma (L^-1 C + C L^-T) Gamma^T, with a relative error that falls like eps/dt.  The
  opposite sign of b is negative definite and fails.
* The J_1 integral: quadrature equals the Lyapunov solution.  The appendix's (1/2) L^-1 [...]
  form is exact for commuting L and C and off for non-commuting ones.
* Uniform-grid reduction: L = -A, C = kT I gives R R^T = 2 kT H.
* Composite mesh (L = M^-1 S non-symmetric):
  - q^2 = c / volume: the Lyapunov solver's C equals (c/2) h^-3 A^-1, L^-1 C is symmetric, and
    R R^T reduces to -2 (alpha/mu) Gamma L^-1 C Gamma^T.
  - uniform q: L^-1 C is not symmetric, R R^T is symmetric positive semi-definite and equals
    R = sqrt(alpha eps/mu) Gamma L^-1 Q squared; Cov(w) = L^-1 Q Q^T L^-T = -(L^-1 C + C L^-T).
  - forced_field agrees with the route through the sampling precision, A w = -(M/h^3) q eta,
    solved densely.  Its Philox draws give the predicted covariance by Monte Carlo.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import effective as eff
from oracle.composite import CompositeGrid


def _quad_nodes(T, panels=160, order=10, first=1e-7):
    """Gauss-Legendre nodes on geometrically graded panels of [0, T] (fine near 0, where the
    integrands of the fast fluid vary)."""
    edges = np.concatenate([[0.0], np.geomspace(first * T, T, panels)])
    xg, wg = np.polynomial.legendre.leggauss(order)
    a, b = edges[:-1, None], edges[1:, None]
    t = 0.5 * (b - a) * xg[None, :] + 0.5 * (a + b)
    w = 0.5 * (b - a) * wg[None, :]
    return t.ravel(), w.ravel()


def _increment_moments(L, C, f, dt, eps):
    """Exact mean and covariance of Y = integral_0^dt u for the stationary SDE
    du = eps^-1 L u dt + f dt + Q dB (u(0) ~ N(0, C), stationary for f = 0):
    E Y = integral_0^dt (dt - t) e^{tL/eps} f dt and
    Cov Y = integral_0^dt (dt - t) [K(t) + K(t)^T] dt with K(t) = e^{tL/eps} C."""
    t, w = _quad_nodes(dt)
    n = L.shape[0]
    mean = np.zeros(n)
    cov = np.zeros((n, n))
    for ti, wi in zip(t, w):
        E = sla.expm(ti * L / eps)
        K = E @ C
        cov += wi * (dt - ti) * (K + K.T)
        mean += wi * (dt - ti) * (E @ f)
    return mean, cov


def _small_composite():
    return CompositeGrid(4, 4, 2, box=(1, 3, 1, 3, 0, 1), h=1.0)


def test_asymptotics_of_increments_by_quadrature():
    g = _small_composite()
    L = g.laplacian().toarray()
    rng = np.random.default_rng(5)
    n = L.shape[0]
    QQ = np.diag(rng.uniform(0.5, 1.5, n))            # a non-symmetric case: L^-1 C asymmetric
    G = rng.standard_normal((3, n)) / np.sqrt(n)
    f = rng.standard_normal(n)
    dt = 1.0
    errs_b, errs_a = [], []
    for eps in (1.0 / 16, 1.0 / 64):
        C = eff.covariance_from_forcing(L, QQ, eps)
        mean, cov = _increment_moments(L, C, f, dt, eps)
        b = eff.increment_covariance_rate(L, C, G, eps)
        a = eff.drift(L, G, f, eps)
        got_b = G @ cov @ G.T / dt
        got_a = G @ mean / dt
        errs_b.append(np.abs(got_b - b).max() / np.abs(b).max())
        errs_a.append(np.abs(got_a - a).max() / np.abs(a).max())
        # b is positive definite and the quadrature is closer to it than to -b
        assert np.linalg.eigvalsh(b).min() > 0.0
        assert np.abs(got_b + b).max() > 1.5 * np.abs(b).max()
    # error O(eps/dt): a factor 4 in eps gives a factor about 4 in the error
    for e in (errs_b, errs_a):
        assert e[1] < 0.1, e
        assert 3.0 < e[0] / e[1] < 5.0, e


def test_j1_integral_general_form():
    rng = np.random.default_rng(2)
    n = 5
    B = rng.standard_normal((n, n))
    L = -(B @ B.T + n * np.eye(n)) @ np.diag(rng.uniform(0.5, 2.0, n))   # non-symmetric
    C = np.diag(rng.uniform(0.5, 1.5, n))
    T = 0.7
    t, w = _quad_nodes(T, panels=60, first=1e-4)
    Y = sum(wi * sla.expm(ti * L) @ C @ sla.expm(ti * L.T) for ti, wi in zip(t, w))
    E = sla.expm(T * L)
    bracket = E @ C @ E.T - C
    Ylyap = sla.solve_continuous_lyapunov(L, bracket)
    assert np.allclose(Y, Ylyap, atol=1e-10 * np.abs(Y).max())
    half = 0.5 * np.linalg.solve(L, bracket)
    assert np.abs(half - Y).max() > 1e-3 * np.abs(Y).max()     # not valid without commuting
    Ls = -(B @ B.T + n * np.eye(n))                                # symmetric, C = I commutes
    Ys = sum(wi * sla.expm(2.0 * ti * Ls) for ti, wi in zip(t, w))
    Es = sla.expm(T * Ls)
    assert np.allclose(Ys, 0.5 * np.linalg.solve(Ls, Es @ Es.T - np.eye(n)),
                       atol=1e-10 * np.abs(Ys).max())


def test_uniform_grid_reduction():
    from oracle.operator import assemble_A
    from oracle import selm
    A = np.kron(np.eye(3), assemble_A(4, 4, 3, h=1.0).toarray())   # three velocity components
    X = np.array([[1.3, 2.2, 1.1], [2.9, 0.7, 1.8]])
    G = selm.gamma_matrix(X, 4, 4, 3).toarray()
    kT, alpha, mu = 0.8, 1.0, 1.7
    H = eff.mobility(-A, G, alpha, mu)
    R = eff.noise_covariance(-A, kT * np.eye(A.shape[0]), G, alpha, mu)
    assert np.allclose(R, 2.0 * kT * H, atol=1e-13 * np.abs(H).max())
    assert np.allclose(H, (alpha / mu) * G @ np.linalg.solve(A, G.T), atol=1e-13)


def test_composite_volume_weighted_forcing_is_symmetric_case():
    g = CompositeGrid(8, 8, 4, box=(2, 6, 2, 6, 0, 2), h=0.5)
    L = g.laplacian().toarray()
    c = 0.9
    QQ = np.diag(c / g.vol)
    C = eff.covariance_from_forcing(L, QQ)
    target = 0.5 * c * g.h ** -3 * np.linalg.inv(g.A.toarray())
    assert np.allclose(C, target, atol=1e-10 * np.abs(target).max())
    LiC = np.linalg.solve(L, C)
    assert np.allclose(LiC, LiC.T, atol=1e-10 * np.abs(LiC).max())
    rng = np.random.default_rng(1)
    G = rng.standard_normal((4, g.n)) / np.sqrt(g.n)
    alpha, mu = 1.3, 0.7
    R = eff.noise_covariance(L, C, G, alpha, mu)
    assert np.allclose(R, -2.0 * (alpha / mu) * G @ LiC @ G.T, atol=1e-10 * np.abs(R).max())


def test_composite_uniform_forcing_is_non_symmetric_case():
    g = CompositeGrid(8, 8, 4, box=(2, 6, 2, 6, 0, 2), h=0.5)
    L = g.laplacian().toarray()
    q = np.full(g.n, 1.2)
    QQ = np.diag(q ** 2)
    eps, alpha, mu = 0.3, 1.1, 2.0
    C = eff.covariance_from_forcing(L, QQ, eps)
    assert np.allclose(C, C.T, atol=1e-10 * np.abs(C).max())
    LiC = np.linalg.solve(L, C)
    assert np.abs(LiC - LiC.T).max() > 1e-2 * np.abs(LiC).max()
    rng = np.random.default_rng(3)
    G = rng.standard_normal((5, g.n)) / np.sqrt(g.n)
    R = eff.noise_covariance(L, C, G, alpha, mu)
    assert np.allclose(R, R.T, atol=1e-12 * np.abs(R).max())
    assert np.linalg.eigvalsh(R).min() > -1e-10 * np.abs(R).max()
    F = eff.noise_factor(L, np.diag(q), G, alpha, mu, eps)
    assert np.allclose(F @ F.T, R, atol=1e-9 * np.abs(R).max())
    # the field covariance at eps = 1: L^-1 Q Q^T L^-T = -(L^-1 C1 + C1 L^-T)
    C1 = eff.covariance_from_forcing(L, QQ, 1.0)
    I = np.eye(g.n)
    W = eff.forced_covariance(g, q)
    assert np.allclose(W, eff.increment_covariance_rate(L, C1, I), atol=1e-9 * np.abs(W).max())


def test_forced_field_two_routes_and_monte_carlo():
    g = _small_composite()
    rng = np.random.default_rng(4)
    qc = rng.uniform(0.5, 1.5, g.nbase)
    qf = rng.uniform(0.5, 1.5, g.nf)
    ec, ef = eff.forcing_noise(7, 3, g.nbase, g.nf)
    wc, wf = eff.forced_field(g, qc, qf, ec, ef)
    # the sampling-precision route: A w = -(vol / h^3) q eta
    b = -g.join(qc * ec, qf * ef) * g.vol / g.h ** 3
    w2 = np.linalg.solve(g.A.toarray(), b)
    assert np.allclose(g.join(wc, wf), w2, atol=1e-12 * np.abs(w2).max())
    assert np.all(wc.ravel()[~np.isin(np.arange(g.nbase), g.coarse_cells)] == 0.0)
    # Monte Carlo over the Philox draws: variance of three projections within 5 standard errors
    q = g.join(qc, qf)
    W = eff.forced_covariance(g, q)
    P = rng.standard_normal((3, g.n))
    n = 4000
    proj = np.empty((n, 3))
    for s in range(n):
        ec, ef = eff.forcing_noise(11, s, g.nbase, g.nf)
        proj[s] = P @ g.join(*eff.forced_field(g, qc, qf, ec, ef))
    var = np.einsum("ij,jk,ik->i", P, W, P)
    emp = (proj ** 2).mean(axis=0)
    assert np.all(np.abs(emp - var) <= 5.0 * var * np.sqrt(2.0 / n)), (emp, var)
