"""Pins of the SELM coupling oracle (CPU).

* a_z^{1/2}: squares to a_z, and maps each closed-form wall eigenvector sin(pi m (z + 1/2)/nz)
  to sqrt(lambda_m) times itself (lambda_m = (4/h^2) sin^2(pi m / (2 nz))), independently of the
  eigensolver that built it.
* D D^T = A exactly; the projection P = I - D^T A^-1 D is symmetric, idempotent, annihilates
  gradients D^T p, leaves discrete curls (delta_y psi, -delta_x psi, 0) unchanged, has D P = 0,
  rank 2N, and commutes with the viscous operator (I_3 x A).
* Peskin's 4-point function: the even and odd sums are 1/2 each, the first moment vanishes and
  the sum of squares is 3/8 at every offset (the kernel's defining identities).
* Gamma: partition of unity and exact reproduction of linear fields away from the walls, and of
  a profile vanishing on the wall near it (which checks the antisymmetric ghost folding).
* H: the mobility computed by spreading, projecting, solving and interpolating equals the dense
  formula (alpha/mu) Gamma P A^-1 P Gamma^T; it is symmetric positive definite.
* <g g^T> = 2 kT H: exactly by covariance propagation through K with Cov(xi) = A^-1/mu, and by
  Monte Carlo with xi drawn by the stochastic multigrid chain (three scalar chains at kT = 1/mu,
  an emitted sample every 2 cycles), within 5 Monte Carlo standard errors.
"""
import numpy as np
import pytest

from oracle import selm
from oracle.operator import assemble_A


def test_sqrt_wall_operator_closed_form():
    for nz, h in ((5, 1.0), (8, 0.5), (2, 1.0)):
        S = selm.sqrt_wall_operator(nz, h)
        a = selm.wall_operator_1d(nz, h)
        assert np.allclose(S, S.T, atol=1e-14) and np.allclose(S @ S, a, atol=1e-12)
        z = np.arange(nz)
        for m in range(1, nz + 1):
            v = np.sin(np.pi * m * (z + 0.5) / nz)
            lam = 4.0 / h ** 2 * np.sin(np.pi * m / (2 * nz)) ** 2
            assert np.allclose(a @ v, lam * v, atol=1e-12)
            assert np.allclose(S @ v, np.sqrt(lam) * v, atol=1e-12)


@pytest.mark.parametrize("dims", [(4, 4, 3), (6, 4, 4), (4, 2, 5)])
def test_projection_properties(dims):
    nx, ny, nz = dims
    N = nx * ny * nz
    A = assemble_A(nx, ny, nz).toarray()
    D = selm.divergence_matrix(nx, ny, nz).toarray()
    assert np.allclose(D @ D.T, A, atol=1e-12)
    P = selm.projection_matrix(nx, ny, nz)
    assert np.allclose(P, P.T, atol=1e-12)
    assert np.allclose(P @ P, P, atol=1e-12)
    assert np.allclose(D @ P, 0.0, atol=1e-12)
    assert np.linalg.matrix_rank(P, tol=1e-9) == 2 * N
    rng = np.random.default_rng(1)
    p = rng.standard_normal(N)
    assert np.allclose(P @ (D.T @ p), 0.0, atol=1e-12)
    # discrete curl of psi in the periodic plane: divergence free, left unchanged
    psi = rng.standard_normal(N)
    dx = selm.divergence_matrix(nx, ny, nz)[:, :N].toarray()
    dy = selm.divergence_matrix(nx, ny, nz)[:, N:2 * N].toarray()
    u = np.concatenate([dy @ psi, -(dx @ psi), np.zeros(N)])
    assert np.allclose(D @ u, 0.0, atol=1e-12) and np.allclose(P @ u, u, atol=1e-12)
    L3 = np.kron(np.eye(3), A)
    assert np.allclose(P @ L3, L3 @ P, atol=1e-11)
    # the sparse-solve route equals the dense matrix
    v = rng.standard_normal(3 * N)
    assert np.allclose(selm.apply_projection(v, nx, ny, nz), P @ v, atol=1e-12)


def test_peskin_identities():
    r = np.linspace(0.0, 1.0, 101, endpoint=False)
    j = np.arange(-3, 5)[:, None]
    phi = selm.peskin4(r[None, :] - j)
    even = phi[(j[:, 0] % 2) == 0].sum(axis=0)
    odd = phi[(j[:, 0] % 2) == 1].sum(axis=0)
    assert np.allclose(even, 0.5, atol=1e-14) and np.allclose(odd, 0.5, atol=1e-14)
    assert np.allclose(((r[None, :] - j) * phi).sum(axis=0), 0.0, atol=1e-14)
    assert np.allclose((phi ** 2).sum(axis=0), 3.0 / 8.0, atol=1e-14)
    # continuous at the breakpoints, zero outside the support
    assert abs(selm.peskin4(1.0 - 1e-12) - selm.peskin4(1.0 + 1e-12)) < 1e-9
    assert selm.peskin4(2.0) == 0.0 and selm.peskin4(2.5) == 0.0


def test_gamma_reproduces_constants_and_linear_fields():
    nx, ny, nz = 8, 8, 8
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    rng = np.random.default_rng(3)
    pts = np.column_stack([rng.uniform(2.5, 5.5, 6), rng.uniform(2.5, 5.5, 6),
                           rng.uniform(2.6, 5.4, 6)])
    W = selm.interpolation_weights(pts, nx, ny, nz)
    assert np.allclose(W @ np.ones(nx * ny * nz), 1.0, atol=1e-14)
    for field, coord in (((x + 0.5).ravel(), 0), ((y + 0.5).ravel(), 1), ((z + 0.5).ravel(), 2)):
        assert np.allclose(W @ field, pts[:, coord], atol=1e-13)
    # near the bottom wall: z + 1/2 vanishes on the wall face, and its antisymmetric
    # extension is the same linear function, so interpolation stays exact
    near = np.column_stack([rng.uniform(0, 8, 5), rng.uniform(0, 8, 5), rng.uniform(0.05, 1.5, 5)])
    Wn = selm.interpolation_weights(near, nx, ny, nz)
    assert np.allclose(Wn @ (z + 0.5).ravel(), near[:, 2], atol=1e-13)
    # and near the top wall for nz*h - (z + 1/2)
    top = near.copy()
    top[:, 2] = nz - near[:, 2]
    Wt = selm.interpolation_weights(top, nx, ny, nz)
    assert np.allclose(Wt @ (nz - (z + 0.5)).ravel(), nz - top[:, 2], atol=1e-13)


def _case():
    S = selm.SELM(8, 8, 6, h=1.0, mu=1.3, kT=0.7)
    X = np.array([[2.3, 4.1, 1.7], [5.6, 3.3, 3.9]])
    return S, X


def test_mobility_equals_dense_formula():
    S, X = _case()
    H = S.mobility_matrix(X)
    G = selm.gamma_matrix(X, *S.dims).toarray()
    P = selm.projection_matrix(*S.dims)
    Ai = np.linalg.inv(S.A.toarray())
    Hd = (S.alpha / S.mu) * G @ P @ np.kron(np.eye(3), Ai) @ P @ G.T
    assert np.allclose(H, Hd, rtol=0, atol=1e-12 * np.abs(Hd).max())
    assert np.allclose(H, H.T, atol=1e-12 * np.abs(H).max())
    assert np.linalg.eigvalsh(0.5 * (H + H.T)).min() > 0.0


def test_drive_covariance_exact_and_monte_carlo():
    S, X = _case()
    H = S.mobility_matrix(X)
    G = selm.gamma_matrix(X, *S.dims).toarray()
    P = selm.projection_matrix(*S.dims)
    K = np.sqrt(2.0 * S.kT * S.alpha) * G @ P
    C = selm.xi_covariance(*S.dims, mu=S.mu)
    assert np.allclose(K @ C @ K.T, 2.0 * S.kT * H, atol=1e-12 * np.abs(H).max())
    # Monte Carlo: xi from the stochastic multigrid chain (three scalar chains with kT = 1/mu)
    from oracle.mg import StochasticMG
    from oracle.philox import PhiloxNoise
    mg = StochasticMG(*S.dims, kT=1.0 / S.mu, levels=2)
    n, stride = 1500, 2
    zero = np.zeros(S.N)
    xs = [zero.copy() for _ in range(3)]
    noise = PhiloxNoise(11)
    gs = np.empty((n, 6))
    cyc = 0
    for t in range(n):
        for _ in range(stride):
            xs = [mg.vcycle(xs[c], zero, noise, cyc, c) for c in range(3)]
            cyc += 1
        gs[t] = S.drive(X, np.concatenate(xs)).ravel()
    emp = gs.T @ gs / n
    target = 2.0 * S.kT * H
    se = np.sqrt((np.outer(np.diag(target), np.diag(target)) + target ** 2) / n)
    assert np.all(np.abs(emp - target) <= 5.0 * se), np.max(np.abs(emp - target) / se)
